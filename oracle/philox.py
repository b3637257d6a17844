"""Counter-based Gaussian sampling matrices for the oracle (test infrastructure only).

The paper draws a fresh n-by-w Gaussian matrix Omega for the first t-block of
R3SVD (Alg 2) and for every Delta-t growth block of R3SVD/R4SVD (Alg 2, Alg 3).
It does not say which generator.  This module writes out the Philox4x64-10
generator from its published definition (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11) with plain Python integers, and the
Box-Muller transform, so that the oracle and the device path can draw the same
Omega without sharing code.

Stream layout (identical on both sides, documented in the C header):
  key      = (seed, 0)
  counter  = (j, q, b, i)  for row j of Omega, 4-column group q = c // 4,
             block b of SVT iteration i (b = 0 is the t-block of the first call,
             growth blocks count from 1 within each iteration).
  words w0..w3 -> u_l = ((w_l >> 11) + 0.5) * 2**-53
  columns 4q+0, 4q+1 = sqrt(-2 ln u0) * (cos, sin)(2 pi u1)
  columns 4q+2, 4q+3 = sqrt(-2 ln u2) * (cos, sin)(2 pi u3)
"""
import math

import numpy as np

_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1


def philox4x64_10(counter, key):
    """One Philox4x64 block with 10 rounds: 4 words out for a 4-word counter and 2-word key."""
    c0, c1, c2, c3 = (int(v) & _MASK for v in counter)
    k0, k1 = (int(v) & _MASK for v in key)
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & _MASK, (p0 >> 64) ^ c3 ^ k1, p0 & _MASK)
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return (c0, c1, c2, c3)


def word_to_uniform(w):
    """Map a 64-bit word to the open interval (0, 1) on the 2**-53 grid (never 0 or 1)."""
    return ((int(w) >> 11) + 0.5) * (2.0 ** -53)


def _mulhilo(a, b):
    """64x64 -> 128-bit product of uint64 arrays, returned as (hi, lo) words."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo, a_hi = a & m32, a >> s32
    b_lo, b_hi = np.uint64(b & 0xFFFFFFFF), np.uint64(b >> 32)
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> s32) + (lh & m32) + (hl & m32)
    lo = (ll & m32) | (mid << s32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    return hi, lo


def philox4x64_10_array(c0, c1, c2, c3, k0, k1):
    """Philox4x64-10 over arrays of counters (same rounds as philox4x64_10)."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64).copy() for v in (c0, c1, c2, c3))
    k0 = np.uint64(k0 & _MASK)
    k1 = np.uint64(k1 & _MASK)
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo(c0, _M0)
            hi1, lo1 = _mulhilo(c2, _M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            k0 = np.uint64((int(k0) + _W0) & _MASK)
            k1 = np.uint64((int(k1) + _W1) & _MASK)
    return c0, c1, c2, c3


def omega_block(seed, it, blk, n, w):
    """The n-by-w Gaussian block Omega_{it,blk} as float64 (row j, column c)."""
    ngroups = (w + 3) // 4
    jj, qq = np.meshgrid(np.arange(n, dtype=np.uint64), np.arange(ngroups, dtype=np.uint64), indexing="ij")
    words = philox4x64_10_array(jj.ravel(), qq.ravel(), np.full(jj.size, blk, np.uint64),
                                np.full(jj.size, it, np.uint64), int(seed), 0)
    u = [((wd >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53) for wd in words]
    cols = []
    for pair in range(2):
        rad = np.sqrt(-2.0 * np.log(u[2 * pair]))
        ang = 2.0 * np.pi * u[2 * pair + 1]
        cols.append(rad * np.cos(ang))
        cols.append(rad * np.sin(ang))
    z = np.stack(cols, axis=1).reshape(n, ngroups * 4)
    return np.ascontiguousarray(z[:, :w])


def omega_block_scalar(seed, it, blk, n, w):
    """Element-by-element version of omega_block (plain Python, for small pins)."""
    out = np.empty((n, w), dtype=np.float64)
    for j in range(n):
        for c in range(w):
            words = philox4x64_10((j, c // 4, blk, it), (seed, 0))
            l = c % 4
            u_r = word_to_uniform(words[2 * (l // 2)])
            u_a = word_to_uniform(words[2 * (l // 2) + 1])
            rad = math.sqrt(-2.0 * math.log(u_r))
            ang = 2.0 * math.pi * u_a
            out[j, c] = rad * (math.cos(ang) if l % 2 == 0 else math.sin(ang))
    return out
