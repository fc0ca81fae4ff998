// Random draws of Alg. 2: the row block B (host, Floyd's algorithm) and Gaussian
// matrices (device, Box-Muller) from Philox4x64-10 streams (seed, purpose, t).
//   uniform in (0,1]: ((w >> 11) + 1) 2^-53;  uniform in [0,1): (w >> 11) 2^-53
//   normal number e: sqrt(-2 ln u1) cos(2 pi u2) with u1 from word 2e, u2 from word 2e+1
//   bounded integer in [0, s): Lemire's multiply-shift with rejection
//   permutation of [0, m): Fisher-Yates from the top, i swapped with bounded(i + 1)
#include <algorithm>
#include <vector>

#include "internal.h"

namespace adasap {

namespace {

// one Philox block gives the four words 4i..4i+3 = normals 2i and 2i+1
__global__ void normals_kernel(uint64_t seed, uint64_t purpose, uint64_t t, int64_t count,
                               double* __restrict__ out, const int64_t* __restrict__ t_dev) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t_dev) t += (uint64_t)*t_dev;  // plus a counter in device memory (replayable launches)
  seed += blockIdx.y;  // problem p of a batch draws with seed + p
  out += (int64_t)blockIdx.y * count;
  if (2 * i >= count) return;
  const u64x4 w = philox4x64_10((uint64_t)i + 1, t, 0, 0, seed, purpose);
  const double two_pi = 6.283185307179586;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t e = 2 * i + h;
    if (e >= count) break;
    const double u1 = ((double)(w.v[2 * h] >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(w.v[2 * h + 1] >> 11) * 0x1.0p-53;
    out[e] = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
  }
}

struct HostStream {
  uint64_t seed, purpose, t;
  uint64_t block = 0;
  int pos = 4;
  u64x4 buf{};
  uint64_t next() {
    if (pos == 4) {
      buf = philox4x64_10(block + 1, t, 0, 0, seed, purpose);
      ++block;
      pos = 0;
    }
    return buf.v[pos++];
  }
};

uint64_t bounded(HostStream& hs, uint64_t s) {
  uint64_t x = hs.next();
  unsigned __int128 m = (unsigned __int128)x * s;
  uint64_t low = (uint64_t)m;
  if (low < s) {
    const uint64_t threshold = (0 - s) % s;
    while (low < threshold) {
      x = hs.next();
      m = (unsigned __int128)x * s;
      low = (uint64_t)m;
    }
  }
  return (uint64_t)(m >> 64);
}

}  // namespace

adasap_status_t normals_dev(uint64_t seed, uint64_t purpose, uint64_t t, int64_t count,
                            double* out, hipStream_t s, int P, const int64_t* t_dev) {
  if (count <= 0) return ADASAP_OK;
  const int64_t blocks = (count + 1) / 2;
  hipLaunchKernelGGL(normals_kernel, dim3((unsigned)((blocks + 255) / 256), P), dim3(256), 0, s,
                     seed, purpose, t, count, out, t_dev);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

void sample_block_host(uint64_t seed, uint64_t purpose, uint64_t t, int64_t n, int64_t b,
                       int64_t* out) {
  HostStream hs{seed, purpose, t};
  if (b == n) {
    for (int64_t i = 0; i < n; ++i) out[i] = i;
    // draws are still consumed in the oracle's order; the result is all of [0, n)
    return;
  }
  // the chosen set: open addressing in a power-of-two table of at least 4b slots (empty = -1),
  // multiplicative hashing, linear probing; reused across calls of a thread
  static thread_local std::vector<int64_t> table;
  size_t cap = 16;
  while (cap < (size_t)b * 4) cap <<= 1;
  table.assign(cap, -1);
  const size_t mask = cap - 1;
  int shift = 64;
  for (size_t c = cap; c > 1; c >>= 1) --shift;
  auto slot = [&](int64_t key) {
    size_t i = (size_t)(((uint64_t)key * 0x9E3779B97F4A7C15ull) >> shift);
    while (table[i] != -1 && table[i] != key) i = (i + 1) & mask;
    return i;
  };
  int64_t cnt = 0;
  for (int64_t j = n - b; j < n; ++j) {
    const int64_t v = (int64_t)bounded(hs, (uint64_t)j + 1);
    const size_t sv = slot(v);
    int64_t pick = v;
    if (table[sv] == v) {
      pick = j;  // v taken: j itself (never drawn before, since every earlier draw is < j)
      table[slot(j)] = j;
    } else {
      table[sv] = v;
    }
    out[cnt++] = pick;
  }
  // ascending order: LSD radix sort with 11-bit digits over the bits that [0, n) needs
  static thread_local std::vector<int64_t> tmp;
  tmp.resize((size_t)b);
  int64_t* src = out;
  int64_t* dst = tmp.data();
  for (int shift = 0; shift < 63 && ((uint64_t)(n - 1) >> shift) != 0; shift += 11) {
    int64_t count[2049] = {};
    for (int64_t i = 0; i < b; ++i) ++count[((src[i] >> shift) & 2047) + 1];
    for (int d = 0; d < 2048; ++d) count[d + 1] += count[d];
    for (int64_t i = 0; i < b; ++i) dst[count[(src[i] >> shift) & 2047]++] = src[i];
    std::swap(src, dst);
  }
  if (src != out) std::copy(src, src + b, out);
}

void permutation_host(uint64_t seed, uint64_t purpose, uint64_t t, int64_t m, int64_t* out) {
  HostStream hs{seed, purpose, t};
  for (int64_t i = 0; i < m; ++i) out[i] = i;
  for (int64_t i = m - 1; i > 0; --i) {
    const int64_t j = (int64_t)bounded(hs, (uint64_t)i + 1);
    const int64_t tmp = out[i];
    out[i] = out[j];
    out[j] = tmp;
  }
}

}  // namespace adasap
