"""Counter-based random streams shared (by definition, not by code) with the HIP path.

Test infrastructure (see the package docstring).

The method draws three kinds of random numbers per iteration t (Alg. 2):
the row block B (uniform, Sec. 4.2 / Sec. 5 setup), the Gaussian Nystrom test
matrix Omega (Alg. 2 Step II, Alg. NysApprox) and the Gaussian start vector
of randomized powering (Alg. GetStepsize).  Both implementations derive them
from one published generator so that they can be compared:

* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): 10 rounds of the 4x64 Philox S-box with the
  multipliers and Weyl key increments published there.
* Stream (seed, purpose, t): key = (seed, purpose), block i uses the counter
  (i + 1, t, 0, 0) and yields the four 64-bit words of that block in order.
  (This is exactly what numpy.random.Philox(key=(seed, purpose),
  counter=(0, t, 0, 0)).random_raw() produces; the tests pin it.)
* Uniform double in [0, 1): (w >> 11) * 2**-53;  in (0, 1]: ((w >> 11) + 1) * 2**-53.
* Normal number e of a stream: Box-Muller cosine branch on words 2e and 2e+1,
  sqrt(-2 ln u1) cos(2 pi u2), u1 in (0, 1] from word 2e, u2 in [0, 1) from
  word 2e + 1.
* Bounded integer in [0, s): Lemire's multiply-shift with rejection
  ("Fast random integer generation in an interval", 2019).
* Permutation of [0, m): Fisher-Yates from the top, element i swapped with a
  bounded integer in [0, i + 1) (Durstenfeld, CACM 1964).
* Block B: Floyd's algorithm for a uniform b-subset of [0, n) without
  replacement (Bentley & Floyd, CACM 1987), sorted ascending (reading of
  the paper's "uniform" block distribution: without replacement, independent
  across iterations, ascending order; Omega row i belongs to B[i]).
"""
import numpy as np

MASK64 = (1 << 64) - 1
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B

# purpose codes (the second key word)
PURPOSE_B = 5
PURPOSE_OMEGA = 6
PURPOSE_POW = 7
# minibatch order of the warm-start network's training, epoch e = counter t
PURPOSE_MINIBATCH = 11
# rows of a subsampled residual estimate
PURPOSE_RESROWS = 12
# refinement sweep s draws with purpose + PURPOSE_SWEEP_STRIDE * s
PURPOSE_SWEEP_STRIDE = 16


def philox4x64_10_scalar(ctr, key):
    """One Philox4x64-10 block with Python integers (the published round function)."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for _ in range(10):
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + PHILOX_W0) & MASK64
        k1 = (k1 + PHILOX_W1) & MASK64
    return x0, x1, x2, x3


def _mulhilo64(a, b):
    """(high, low) 64-bit halves of the 128-bit product of uint64 arrays."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo, a_hi = a & m32, a >> s32
    b_lo, b_hi = b & m32, b >> s32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> s32) + (lh & m32) + (hl & m32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    lo = a * b  # wraps modulo 2**64
    return hi, lo


def philox4x64_10(ctr, key):
    """Vectorised Philox4x64-10: ctr is a (4, m) uint64 array, key a pair of ints.

    Returns a (4, m) uint64 array of output words.
    """
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64).copy() for c in ctr)
        k0 = np.uint64(int(key[0]) & MASK64)
        k1 = np.uint64(int(key[1]) & MASK64)
        m0, m1 = np.uint64(PHILOX_M0), np.uint64(PHILOX_M1)
        w0, w1 = np.uint64(PHILOX_W0), np.uint64(PHILOX_W1)
        for _ in range(10):
            hi0, lo0 = _mulhilo64(m0, x0)
            hi1, lo1 = _mulhilo64(m1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            k0 = k0 + w0
            k1 = k1 + w1
    return np.stack([x0, x1, x2, x3])


def stream_words(seed, purpose, t, count, start=0):
    """Words start .. start+count-1 of stream (seed, purpose, t) as uint64."""
    if count <= 0:
        return np.zeros(0, dtype=np.uint64)
    first_block = start // 4
    last_block = (start + count - 1) // 4
    blocks = np.arange(first_block, last_block + 1, dtype=np.uint64)
    nb = blocks.size
    ctr = np.stack([blocks + np.uint64(1),
                    np.full(nb, np.uint64(int(t) & MASK64)),
                    np.zeros(nb, np.uint64), np.zeros(nb, np.uint64)])
    out = philox4x64_10(ctr, (seed, purpose))  # (4, nb)
    words = out.T.reshape(-1)
    off = start - 4 * first_block
    return words[off:off + count]


def uniform_open0(words):
    """Doubles in (0, 1] from 64-bit words."""
    return ((words >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53


def uniform_closed0(words):
    """Doubles in [0, 1) from 64-bit words."""
    return (words >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def normals(seed, purpose, t, count):
    """First `count` standard normals of stream (seed, purpose, t) (Box-Muller, cosine branch)."""
    w = stream_words(seed, purpose, t, 2 * count)
    u1 = uniform_open0(w[0::2])
    u2 = uniform_closed0(w[1::2])
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


class WordStream:
    """Sequential reader of one stream, refilled in vectorised chunks."""

    def __init__(self, seed, purpose, t, chunk=4096):
        self.seed, self.purpose, self.t = seed, purpose, t
        self.chunk = chunk
        self.pos = 0
        self.buf = np.zeros(0, dtype=np.uint64)
        self.buf_start = 0

    def next(self):
        if self.pos - self.buf_start >= self.buf.size:
            self.buf_start = self.pos
            self.buf = stream_words(self.seed, self.purpose, self.t, self.chunk, start=self.pos)
        w = int(self.buf[self.pos - self.buf_start])
        self.pos += 1
        return w


def bounded(ws, s):
    """Uniform integer in [0, s) from a WordStream (Lemire multiply-shift with rejection)."""
    x = ws.next()
    m = x * s
    low = m & MASK64
    if low < s:
        threshold = ((1 << 64) - s) % s
        while low < threshold:
            x = ws.next()
            m = x * s
            low = m & MASK64
    return m >> 64


def sample_block(seed, t, n, b, purpose=PURPOSE_B):
    """Row block B_t: uniform b-subset of [0, n) without replacement, ascending (Floyd)."""
    if not (0 < b <= n):
        raise ValueError("need 0 < b <= n")
    ws = WordStream(seed, purpose, t)
    chosen = set()
    for j in range(n - b, n):
        v = bounded(ws, j + 1)
        chosen.add(j if v in chosen else v)
    return np.array(sorted(chosen), dtype=np.int64)


def permutation(seed, purpose, t, m):
    """Uniform permutation of [0, m): Fisher-Yates, i = m-1 down to 1, swap i with
    bounded(i + 1)."""
    ws = WordStream(seed, purpose, t)
    perm = np.arange(m, dtype=np.int64)
    for i in range(m - 1, 0, -1):
        j = bounded(ws, i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    return perm
