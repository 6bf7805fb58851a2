"""Philox4x64-10 counter-based generator and the uniforms drawn from it.

Follows the published definition (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 64x64->128
multiplications with key bumps by the Weyl constants.  Pure Python integers,
so every operation is exact.

Stream layout used by this project (both sides implement it independently):
  uniform(key, counter, s, i):
      words = philox4x64(ctr=(counter, s, i // 4, domain), key=(key, 0))
      u     = (words[i % 4] >> 11) * 2**-53          in [0, 1)
  domain 0 = sampling uniforms u[s, i] for sample s, path position i;
  domain 1 = parameter initialisation (s = 0, i = parameter index).
"""
import numpy as np

_MASK = (1 << 64) - 1
_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B


def philox4x64(ctr, key, rounds=10):
    """One Philox4x64 block: 4 counter words, 2 key words -> 4 words."""
    c0, c1, c2, c3 = (int(x) & _MASK for x in ctr)
    k0, k1 = (int(x) & _MASK for x in key)
    for _ in range(rounds):
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & _MASK,
                          (p0 >> 64) ^ c3 ^ k1, p0 & _MASK)
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def word_to_uniform(w):
    """Top 53 bits of a 64-bit word scaled to [0, 1); exact in float64."""
    return float(int(w) >> 11) * (2.0 ** -53)


def uniforms(key, counter, ns, n, domain=0):
    """u[s, i] for s < ns, i < n (float64 array, shape (ns, n))."""
    out = np.empty((ns, n), dtype=np.float64)
    nb = (n + 3) // 4
    for s in range(ns):
        for b in range(nb):
            w = philox4x64((counter, s, b, domain), (key, 0))
            for j in range(4):
                i = 4 * b + j
                if i < n:
                    out[s, i] = word_to_uniform(w[j])
    return out
