"""Host-side Gaussian test matrix for Step 1 of Algorithm 4.1 (Shabat et al.,
arXiv 1310.7202, Section 4: an n x l matrix of i.i.d. zero-mean, unit-variance
Gaussian entries).

TEST INFRASTRUCTURE ONLY: see the package docstring for who may call this.

The paper names no generator.  The convention used by both this oracle and
the device generator (each written independently from the published
definitions) is:
  * Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and
    Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11):
    multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments
    0x9E3779B9 / 0xBB67AE85, ten rounds.
  * key = (low 32 bits of seed, high 32 bits of seed); for the element with
    column-major index e = i + j*n, the pair index t = e // 2 gives the
    counter (t mod 2^32, t div 2^32, 0, 0).
  * Output words x0..x3 form two 53-bit uniforms
      u1 = (((x1:x0) >> 11) + 1) * 2^-53  in (0, 1]
      u2 = ((x3:x2) >> 11) * 2^-53       in [0, 1)
    and the Box-Muller transform (Box and Muller, 1958)
      r = sqrt(-2 ln u1),  z0 = r cos(2 pi u2),  z1 = r sin(2 pi u2);
    even e takes z0, odd e takes z1.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on arrays of 32-bit words (held in uint64).

    One round: the products M0*c0 and M1*c2 are split into high and low
    32-bit halves; the new words are (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0).
    The key is advanced by the Weyl increments between rounds.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0          # < 2^64: exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def box_muller(x0, x1, x2, x3):
    """Two standard normals from the four Philox words (see module doc)."""
    x0 = np.asarray(x0, dtype=np.uint64)
    x1 = np.asarray(x1, dtype=np.uint64)
    x2 = np.asarray(x2, dtype=np.uint64)
    x3 = np.asarray(x3, dtype=np.uint64)
    a = (x1 << _S32) | x0
    b = (x3 << _S32) | x2
    u1 = ((a >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = (b >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    theta = (2.0 * np.pi) * u2
    return r * np.cos(theta), r * np.sin(theta)


def philox_words(n: int, l: int, seed: int):
    """The raw Philox output words for every pair index of an n x l matrix."""
    total = n * l
    npairs = (total + 1) // 2
    t = np.arange(npairs, dtype=np.uint64)
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64((seed >> 32) & 0xFFFFFFFF)
    zero = np.zeros_like(t)
    return philox4x32_10(t & _MASK, t >> _S32, zero, zero, k0, k1)


def gaussian_matrix(n: int, l: int, seed: int) -> np.ndarray:
    """Step 1 of Algorithm 4.1: the n x l Gaussian G for ``seed``
    (column-major element order, returned as a C-ordered n x l array)."""
    total = n * l
    x0, x1, x2, x3 = philox_words(n, l, seed)
    z0, z1 = box_muller(x0, x1, x2, x3)
    flat = np.empty(2 * z0.size)
    flat[0::2] = z0
    flat[1::2] = z1
    return flat[:total].reshape(l, n).T.copy()


# ---------------------------------------------------------------------------
# The draws of the SRFT of Algorithm 4.4 (Section 3.3), R = D F S: the signs
# of D and the column selection of S, from the same generator and key with
# the third counter word set apart from Step 1's (which is 0):
#   * signs: for element i the 128 output bits of the counter
#     (i div 128, 0, 1, 0); bit t = i mod 128 is bit (t mod 32) of word
#     (t div 32); d_i = +1 if that bit is 0, -1 if it is 1.
#   * selection: a partial Fisher-Yates shuffle of idx = 0..n-1: for
#     j = 0..l-1, with (x1:x0) of the counter (j, 0, 2, 0) as a 64-bit u,
#     t = j + (u mod (n - j)) and idx[j], idx[t] are exchanged; S selects
#     the columns idx[0..l-1], in that order (l distinct indices).
# ---------------------------------------------------------------------------


def srft_signs(n: int, seed: int) -> np.ndarray:
    """d (length n) of D = diag(d), entries +1 / -1."""
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64((seed >> 32) & 0xFFFFFFFF)
    blocks = np.arange((n + 127) // 128, dtype=np.uint64)
    zero = np.zeros_like(blocks)
    words = philox4x32_10(blocks, zero, zero + np.uint64(1), zero, k0, k1)
    i = np.arange(n)
    b, t = i // 128, i % 128
    w = np.stack(words)[t // 32, b]
    bit = (w >> (t % 32).astype(np.uint64)) & np.uint64(1)
    return np.where(bit == 0, 1.0, -1.0)


def srft_selection(n: int, l: int, seed: int) -> np.ndarray:
    """The l distinct column indices of S, in draw order."""
    if not 0 <= l <= n:
        raise ValueError("need 0 <= l <= n")
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64((seed >> 32) & 0xFFFFFFFF)
    j = np.arange(l, dtype=np.uint64)
    zero = np.zeros_like(j)
    x0, x1, _, _ = philox4x32_10(j, zero, zero + np.uint64(2), zero, k0, k1)
    idx = np.arange(n, dtype=np.int64)
    for jj in range(l):
        u = (int(x1[jj]) << 32) | int(x0[jj])
        t = jj + u % (n - jj)
        idx[jj], idx[t] = idx[t], idx[jj]
    return idx[:l].copy()
