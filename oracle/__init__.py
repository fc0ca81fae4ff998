"""Plain CPU FP64 oracle of the ADASAP hot path (test infrastructure only).

This package is the slow, obviously-correct reference that the HIP path is
checked against.  It is test infrastructure: only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.  The product
path (the C-ABI library and its Python binding) never imports, links or calls
anything here, and this package never imports the product path.

Everything is float64 numpy, written step by step in the paper's order and
notation ("Turbocharging Gaussian Process Inference with Approximate
Sketch-and-Project", arXiv 2505.13723):

* ``rng``       counter-based Philox4x64-10 streams, Box-Muller normals,
                Lemire bounded integers and Floyd block sampling (the random
                draws both sides must agree on).
* ``kernels``   RBF and Matern covariance functions (Sec. 2; textbook forms).
* ``nystrom``   randomized Nystrom approximation (Appendix, Alg. NysApprox)
                and the Woodbury applies (Eq. inv_nys_woodbury and
                Eq. inv_sqrt_nys_woodbury).
* ``stepsize``  randomized powering for the preconditioned smoothness
                constant (Appendix, Alg. GetStepsize).
* ``adasap``    the ADASAP iteration (Alg. 2) with the Nesterov update
                (Appendix, Alg. NestAcc), plus SAP (Alg. 1) and ADASAP-I.
* ``linsys``    direct Cholesky solve, residual, posterior-mean predict.
* ``rff``       random Fourier features (Sec. 2.1, pathwise conditioning).
* ``mlp``       the warm-start MLP forward/backward/Adam in float64.

Parity pins: every function here is checked by ``tests/test_oracle_*.py``
against something other than itself (library routines, closed forms,
invariants, brute force); the helpers (``kernel_from_sqdist``, the oracle's own
Cholesky and substitutions, the random-feature cosines and ridge weights) through
the functions that call them (``kernel_matrix`` against scikit-learn,
``direct_solve`` against ``scipy.linalg.solve``, ``features`` and ``ridge_mean``
against their closed forms).  No function is left without a pin.
"""
