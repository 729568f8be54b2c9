"""Counter-based Gaussian numbers for the test matrix Omega of rSVD-BKI (Alg. 5).

Omega = randn(n, k+s) is the only random draw of the method.  To let the CPU
oracle and the GPU library draw the *same* Omega without passing it across,
each side implements the same counter-based generator from its published
definition:

* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): a 4 x 32-bit counter, a 2 x 32-bit key, ten
  rounds of two 32x32->64 multiplications (multipliers 0xD2511F53 and
  0xCD9E8D57) with the key bumped by the Weyl constants 0x9E3779B9 and
  0xBB67AE85 between rounds.
* Box-Muller (1958): two uniforms u1, u2 in (0, 1) give
  sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2).

Mapping used for Omega (n x b, row-major element index e = row*b + col):
  pair t = e // 2;  counter = (t mod 2^32, t div 2^32, step, attempt);
  key = (seed mod 2^32, seed div 2^32);
  u1 = (z1 + 0.5) * 2^-53 with z1 = ((x0 << 32) | x1) >> 11, the top 53 bits
       of the 64-bit word (x0:x1); u2 likewise from (x2:x3);
  element 2t gets the cosine branch and element 2t+1 the sine branch.
"""

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on arrays of counters.

    ctr: tuple of four uint32 arrays (or scalars); key: pair of uint32.
    Returns four uint32 arrays.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in ctr)
    k0 = np.uint64(key[0]) & _MASK
    k1 = np.uint64(key[1]) & _MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0                      # 32 x 32 -> 64 bit products
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def _unit53(hi, lo):
    z = ((hi.astype(np.uint64) << _S32) | lo.astype(np.uint64)) >> np.uint64(11)
    return (z.astype(np.float64) + 0.5) * (2.0 ** -53)


def gaussian_block(rows, cols, seed, step, attempt):
    """The rows x cols standard-normal matrix Omega for (seed, step, attempt)."""
    count = int(rows) * int(cols)
    npair = (count + 1) // 2
    t = np.arange(npair, dtype=np.uint64)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    x0, x1, x2, x3 = philox4x32_10(
        (t & _MASK, t >> _S32,
         np.full(npair, step & 0xFFFFFFFF, dtype=np.uint64),
         np.full(npair, attempt & 0xFFFFFFFF, dtype=np.uint64)),
        (seed & 0xFFFFFFFF, seed >> 32))
    u1 = _unit53(x0, x1)
    u2 = _unit53(x2, x3)
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    out = np.empty(2 * npair, dtype=np.float64)
    out[0::2] = rad * np.cos(ang)
    out[1::2] = rad * np.sin(ang)
    return out[:count].reshape(rows, cols)
