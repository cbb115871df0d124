"""Counter-based Gaussian noise: Philox4x64-10 and a Box-Muller transform.

The paper only says the Langevin white noise is drawn on the fly from a pseudo-random
generator (Sec. "adQTB", first paragraph; the O block of the TRPMD equations of motion).
Both sides of the parity test implement one counter-based generator from its published
definition (Salmon, Moraes, Dror & Shaw, SC'11: Philox-4x64 with 10 rounds) and the
Box-Muller transform (1958). To make the Gaussians reproducible bit for bit on any
machine, the logarithm and the sine/cosine are evaluated here with IEEE +,-,*,/ only,
in a fixed order:

* ln u: u = m 2^e with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s), s = (m-1)/(m+1),
  atanh by its Taylor series (12 terms, |s| <= 0.1716), ln u = e ln2 + ln m.
* sin/cos(2 pi u): q = rint(4u), r = u - q/4 is exact, theta = 2 pi r in [-pi/4, pi/4],
  Taylor series to theta^17 (sin) and theta^18 (cos), quadrant q mod 4.

Uniforms: u = ((x >> 11) + 0.5) * 2^-53, in (0, 1).
"""
import math

import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

LN2 = 0.6931471805599453
SQRT_HALF = 0.7071067811865476
TWO_PI = 6.283185307179586
_LOG_TERMS = 12
_SIN_TERMS = 9      # theta^1 .. theta^17
_COS_TERMS = 10     # theta^0 .. theta^18

# Streams (second key word) used by the method.
STREAM_RPMD_O = 5
STREAM_QTB_WHITE = 6


def _mulhilo(a, b):
    """Full 64x64 -> 128-bit product, returned as (hi, lo)."""
    al, ah = a & _LO32, a >> _S32
    bl, bh = b & _LO32, b >> _S32
    ll = al * bl
    hl = ah * bl
    lh = al * bh
    hh = ah * bh
    cross = (ll >> _S32) + (hl & _LO32) + (lh & _LO32)
    hi = hh + (hl >> _S32) + (lh >> _S32) + (cross >> _S32)
    return hi, a * b


def philox4x64_10(ctr, key):
    """Philox-4x64-10 block function. ctr: 4 arrays (uint64), key: 2 arrays/scalars."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.asarray(key[0], dtype=np.uint64)
    k1 = np.asarray(key[1], dtype=np.uint64)
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo(_M0, c0)
            hi1, lo1 = _mulhilo(_M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            k0 = k0 + _W0
            k1 = k1 + _W1
    return c0, c1, c2, c3


def uniform(x):
    """53-bit uniform in (0, 1) from a 64-bit word."""
    return ((x >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def own_log(u):
    """Natural log from IEEE basic operations only (see module docstring)."""
    u = np.asarray(u, dtype=np.float64)
    m, e = np.frexp(u)
    low = m < SQRT_HALF
    m = np.where(low, m * 2.0, m)
    e = np.where(low, e - 1, e).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    s2 = s * s
    p = np.full_like(s, 1.0 / (2 * _LOG_TERMS - 1))
    for k in range(_LOG_TERMS - 2, -1, -1):
        p = p * s2 + 1.0 / (2 * k + 1)
    r = (2.0 * s) * p
    return e * LN2 + r


def own_sincos_2pi(u):
    """(sin 2 pi u, cos 2 pi u) from IEEE basic operations only."""
    u = np.asarray(u, dtype=np.float64)
    q = np.rint(4.0 * u)
    r = u - q * 0.25
    th = TWO_PI * r
    t = th * th
    sp = np.full_like(t, (-1.0) ** (_SIN_TERMS - 1) / math.factorial(2 * _SIN_TERMS - 1))
    for k in range(_SIN_TERMS - 2, -1, -1):
        sp = sp * t + (-1.0) ** k / math.factorial(2 * k + 1)
    s = th * sp
    cp = np.full_like(t, (-1.0) ** (_COS_TERMS - 1) / math.factorial(2 * _COS_TERMS - 2))
    for k in range(_COS_TERMS - 2, -1, -1):
        cp = cp * t + (-1.0) ** k / math.factorial(2 * k)
    c = cp
    qi = q.astype(np.int64) & 3
    sin = np.select([qi == 0, qi == 1, qi == 2], [s, c, -s], -c)
    cos = np.select([qi == 0, qi == 1, qi == 2], [c, -s, -c], s)
    return sin, cos


def box_muller(x0, x1):
    """Two standard normals from two 64-bit words (Box & Muller 1958)."""
    u0 = uniform(x0)
    u1 = uniform(x1)
    rad = np.sqrt(-2.0 * own_log(u0))
    s, c = own_sincos_2pi(u1)
    return rad * c, rad * s


def gaussians4(seed, stream, c0, c1, c2, c3=0):
    """Four standard normals per counter (c0, c1, c2, c3) under key (seed, stream).

    Returns an array [..., 4]; the method uses components 0, 1, 2 for x, y, z.
    """
    w = philox4x64_10((c0, c1, c2, c3), (np.uint64(seed), np.uint64(stream)))
    g0, g1 = box_muller(w[0], w[1])
    g2, g3 = box_muller(w[2], w[3])
    return np.stack([g0, g1, g2, g3], axis=-1)


def rpmd_noise(seed, step, n_atoms, n_beads):
    """O-step noise xi[mode][atom][xyz] of step ``step``: counter (step, atom, mode, 0)."""
    atom = np.arange(n_atoms, dtype=np.uint64)[None, :]
    mode = np.arange(n_beads, dtype=np.uint64)[:, None]
    g = gaussians4(seed, STREAM_RPMD_O, np.uint64(step), atom, mode)
    return g[..., :3]


def qtb_white(seed, tau0, n_steps, n_atoms, nseg, atoms=None):
    """adQTB white noise w[t][atom][xyz] for global steps tau0 .. tau0+n_steps-1 (all atoms,
    or the given atom indices).

    Counter (tau + nseg, atom, 0, 0) so that the window of the first segment, which
    reaches back one segment before step 0, still has a non-negative counter.
    """
    tau = np.arange(tau0, tau0 + n_steps, dtype=np.int64) + nseg
    assert tau.min() >= 0
    idx = np.arange(n_atoms) if atoms is None else np.asarray(atoms)
    g = gaussians4(seed, STREAM_QTB_WHITE, tau.astype(np.uint64)[:, None],
                   idx.astype(np.uint64)[None, :], np.uint64(0))
    return g[..., :3]
