"""Counter-based random draw of the KLE coefficients xi (oracle side).

The paper puts the randomness of the model problem in omega (Sec. 2.1) and has
the coordinator hand out samples as contiguous index ranges (Sec. 4.2, batch
sampling); it does not name a generator.  Reading taken here: every
coefficient is a pure function of (seed, level, sample index), produced by the
Philox4x64-10 generator of Salmon, Moraes, Dror and Shaw (SC'11):

  key     = (seed, 0)
  counter = (sample index i, level l, block j, 0)
  one block -> four 64-bit words w0..w3
  uniform  u = ((w >> 12) + 1/2) * 2**-52        (exact, in (0, 1))
  normals  Box-Muller on (u0, u1) and (u2, u3):
           z_even = sqrt(-2 log u_a) * cos(2 pi u_b)
           z_odd  = sqrt(-2 log u_a) * sin(2 pi u_b)
  xi_m     = the m-th normal of the concatenated blocks j = 0, 1, ...

log, sin and cos are evaluated by this module's own fixed operation sequences
(no fused multiply-add), so the result is a well defined function of the bits
of u and can be reproduced bit for bit by an independent implementation that
follows the same published recipe.  Only IEEE-754 correctly rounded +, -, *,
/, sqrt and exact bit manipulations are used.

  log(u): u = m 2^e with m in [sqrt(1/2), sqrt(2)); s = (m-1)/(m+1);
          log m = 2 s sum_{k=0}^{K} s^{2k}/(2k+1)  (atanh series, K = 11,
          Horner in s^2, coefficients 1.0/(2k+1)); log u = e*ln2_hi +
          (log m + e*ln2_lo) with the fdlibm split of ln 2.
  sin(pi r), cos(pi r), |r| <= 1/4: Taylor series in r with coefficients
          c_0 = pi, c_k = -c_{k-1}*(pi*pi)/((2k)(2k+1)) (sin, k <= 10) and
          d_0 = 1, d_k = -d_{k-1}*(pi*pi)/((2k-1)(2k)) (cos, k <= 10), where
          pi is the double nearest to pi; Horner in r^2.
  2 pi u: t = 2u, q = rint(4u), r = t - q/2 (exact), quadrant q mod 4.
"""
from __future__ import annotations

import math
import struct

import numpy as np

MASK64 = (1 << 64) - 1
# Philox4x64 round multipliers and Weyl key increments (Salmon et al., SC'11).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
PHILOX_ROUNDS = 10


def philox4x64(counter, key, rounds: int = PHILOX_ROUNDS):
    """One Philox4x64 block: four 64-bit words for a 4-word counter, 2-word key.

    Round: (hi0, lo0) = M0 * x0, (hi1, lo1) = M1 * x2 (full 128-bit products),
    x <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0); the key is bumped by the
    Weyl increments before every round but the first.
    Pinned against numpy.random.Philox (an independent implementation).
    """
    x0, x1, x2, x3 = (int(c) & MASK64 for c in counter)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        x0, x1, x2, x3 = ((p1 >> 64) ^ x1 ^ k0, p1 & MASK64,
                          (p0 >> 64) ^ x3 ^ k1, p0 & MASK64)
    return x0, x1, x2, x3


def raw_words(seed: int, level: int, first: int, count: int, n_modes: int, stream: int = 0) -> np.ndarray:
    """Raw Philox words, uint64 [count, 4*ceil(n_modes/4)], for samples first.. .

    stream is counter word 3: 0 for xi, 2 for the random forcing's xi_f."""
    nblk = (n_modes + 3) // 4
    out = np.empty((count, 4 * nblk), dtype=np.uint64)
    for s in range(count):
        i = first + s
        for j in range(nblk):
            out[s, 4 * j:4 * j + 4] = philox4x64((i, level, j, stream), (seed, 0))
    return out


def uniforms(words: np.ndarray) -> np.ndarray:
    """u = ((w >> 12) + 0.5) * 2**-52: exact (53 significant bits), in (0, 1)."""
    w = np.asarray(words, dtype=np.uint64) >> np.uint64(12)
    return (w.astype(np.float64) + 0.5) * 2.0 ** -52


# --- the two elementary functions, as fixed operation sequences -------------

LN2_HI = float.fromhex("0x1.62e42fee00000p-1")   # fdlibm ln2_hi (low bits zero)
LN2_LO = float.fromhex("0x1.a39ef35793c76p-33")  # fdlibm ln2_lo
SQRT2 = math.sqrt(2.0)                            # correctly rounded sqrt(2)
LOG_TERMS = 12                                    # k = 0..11
TRIG_TERMS = 11                                   # k = 0..10


def _log_coeffs():
    return [1.0 / (2 * k + 1) for k in range(LOG_TERMS)]


def _sin_coeffs():
    pi2 = math.pi * math.pi
    c = [math.pi]
    for k in range(1, TRIG_TERMS):
        c.append(-c[-1] * pi2 / ((2 * k) * (2 * k + 1)))
    return c


def _cos_coeffs():
    pi2 = math.pi * math.pi
    d = [1.0]
    for k in range(1, TRIG_TERMS):
        d.append(-d[-1] * pi2 / ((2 * k - 1) * (2 * k)))
    return d


def fixed_log(u: np.ndarray) -> np.ndarray:
    """Natural log of positive normal doubles by the atanh series above."""
    u = np.asarray(u, dtype=np.float64)
    bits = u.view(np.uint64)
    e = ((bits >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) - 1023
    m = ((bits & np.uint64(0x000FFFFFFFFFFFFF)) | np.uint64(0x3FF0000000000000)).view(np.float64)
    big = m > SQRT2
    m = np.where(big, m * 0.5, m)
    e = np.where(big, e + 1, e)
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    c = _log_coeffs()
    p = np.full_like(s, c[-1])
    for k in range(LOG_TERMS - 2, -1, -1):
        p = p * z + c[k]
    logm = 2.0 * (s * p)
    ef = e.astype(np.float64)
    return ef * LN2_HI + (logm + ef * LN2_LO)


def fixed_sincos_2pi(u: np.ndarray):
    """(sin(2 pi u), cos(2 pi u)) for u in (0, 1) by quadrant reduction."""
    u = np.asarray(u, dtype=np.float64)
    t = 2.0 * u
    q = np.rint(4.0 * u)
    r = t - 0.5 * q
    r2 = r * r
    cs, cc = _sin_coeffs(), _cos_coeffs()
    ps = np.full_like(r, cs[-1])
    pc = np.full_like(r, cc[-1])
    for k in range(TRIG_TERMS - 2, -1, -1):
        ps = ps * r2 + cs[k]
        pc = pc * r2 + cc[k]
    sr = r * ps      # sin(pi r)
    cr = pc          # cos(pi r)
    quad = q.astype(np.int64) & 3
    sin_v = np.select([quad == 0, quad == 1, quad == 2], [sr, cr, -sr], -cr)
    cos_v = np.select([quad == 0, quad == 1, quad == 2], [cr, -sr, -cr], sr)
    return sin_v, cos_v


def box_muller(u: np.ndarray) -> np.ndarray:
    """Normals from uniforms taken in consecutive pairs (u_a, u_b)."""
    u = np.asarray(u, dtype=np.float64)
    ua = u[..., 0::2]
    ub = u[..., 1::2]
    rad = np.sqrt(-2.0 * fixed_log(ua))
    s, c = fixed_sincos_2pi(ub)
    z = np.empty(u.shape, dtype=np.float64)
    z[..., 0::2] = rad * c
    z[..., 1::2] = rad * s
    return z


def draw_xi(seed: int, level: int, first: int, count: int, n_modes: int, stream: int = 0) -> np.ndarray:
    """xi[count, n_modes] (fp64) for samples first..first+count-1 of a level (stream: counter word 3)."""
    w = raw_words(seed, level, first, count, n_modes, stream)
    return box_muller(uniforms(w))[:, :n_modes]


def float_bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]
