"""ADASAP hot path for MI355X (gfx950): HIP kernels behind a C ABI, thin Python binding."""
