"""Smooth particle-mesh Ewald reciprocal sum and the classic Ewald k-sum that pins it.

The paper's long-range electrostatics are the force field's business; the workloads fix
Ewald summation with SPME. Written from Essmann, Perera, Berkowitz, Darden, Lee &
Pedersen, J. Chem. Phys. 103, 8577 (1995):

* cardinal B-splines M_n by their recursion, M_2(x) = 1 - |x - 1| on [0, 2];
  dM_n/dx = M_{n-1}(x) - M_{n-1}(x - 1);
* charge grid Q(k) = sum_i q_i prod_a M_n(u_ai - k_a) over periodic images, with
  u_ai = K_a times the fractional coordinate of atom i wrapped into [0, 1);
* E = 1/(2 pi V) sum_{m != 0} exp(-pi^2 |m|^2 / alpha^2) / |m|^2 B(m) |F(Q)(m)|^2 (times the
  Coulomb constant), B(m) = prod_a |b_a(m_a)|^2,
  |b(m)|^2 = 1 / |sum_{k=0}^{n-2} M_n(k+1) exp(2 pi i m k / K)|^2;
* forces are the exact gradient of that energy.

Reading for odd n and even K: the denominator of |b(K/2)|^2 vanishes; the neighbour
value |b(K/2 - 1)|^2 is used instead.
"""
import math

import numpy as np


def bspline(n, x):
    """Cardinal B-spline M_n(x) (Essmann eq. 4.1 recursion)."""
    x = np.asarray(x, dtype=np.float64)
    if n == 2:
        return np.where((x >= 0.0) & (x <= 2.0), 1.0 - np.abs(x - 1.0), 0.0)
    return x / (n - 1) * bspline(n - 1, x) + (n - x) / (n - 1) * bspline(n - 1, x - 1.0)


def bspline_deriv(n, x):
    return bspline(n - 1, x) - bspline(n - 1, np.asarray(x) - 1.0)


def bspline_moduli(K, n):
    """|b(m)|^2 for m = 0 .. K-1."""
    m = np.arange(K)
    k = np.arange(n - 1)
    den = (bspline(n, k + 1.0)[None, :] * np.exp(2j * math.pi * np.outer(m, k) / K)).sum(axis=1)
    mod = 1.0 / np.abs(den) ** 2
    bad = np.abs(den) ** 2 < 1e-10
    for mm in np.nonzero(bad)[0]:
        mod[mm] = mod[mm - 1]
    return mod


def influence(box, K, n, alpha, coulomb):
    """G(m) = C/(pi V) exp(-pi^2 m^2/alpha^2)/m^2 B(m), G(0) = 0, so E = 1/2 sum G |F(Q)|^2."""
    V = float(np.prod(box))
    axes = []
    for a in range(3):
        m = np.arange(K[a])
        ms = np.where(m <= K[a] // 2, m, m - K[a]) / box[a]
        axes.append(ms)
    m1, m2, m3 = np.meshgrid(*axes, indexing="ij")
    msq = m1 * m1 + m2 * m2 + m3 * m3
    B = np.multiply.outer(np.multiply.outer(bspline_moduli(K[0], n), bspline_moduli(K[1], n)),
                          bspline_moduli(K[2], n))
    G = np.zeros_like(msq)
    nz = msq > 0
    G[nz] = coulomb / (math.pi * V) * np.exp(-math.pi ** 2 * msq[nz] / alpha ** 2) / msq[nz] * B[nz]
    return G


def _stencil(x, box, K, n):
    """Grid indices [N][3][n] and weights / derivative weights of every atom."""
    s = x / box
    s = s - np.floor(s)
    u = s * np.asarray(K)
    fl = np.floor(u)
    frac = u - fl
    t = np.arange(n)
    idx = (fl.astype(np.int64)[:, :, None] - t[None, None, :]) % np.asarray(K)[None, :, None]
    w = bspline(n, frac[:, :, None] + t[None, None, :])
    dw = bspline_deriv(n, frac[:, :, None] + t[None, None, :])
    return idx, w, dw


def spme(x, q, box, K, n, alpha, coulomb):
    """Reciprocal-space energy and gradient [N][3] of one configuration."""
    K = tuple(int(k) for k in K)
    idx, w, dw = _stencil(x, box, K, n)
    N = len(x)
    # flat grid index and weight of each of the n^3 points of every atom
    f = ((idx[:, 0, :, None, None] * K[1] + idx[:, 1, None, :, None]) * K[2]
         + idx[:, 2, None, None, :]).reshape(N, -1)
    W = (w[:, 0, :, None, None] * w[:, 1, None, :, None] * w[:, 2, None, None, :]).reshape(N, -1)
    Qg = np.bincount(f.ravel(), weights=(q[:, None] * W).ravel(), minlength=K[0] * K[1] * K[2])
    Qg = Qg.reshape(K)
    FQ = np.fft.fftn(Qg)
    G = influence(box, K, n, alpha, coulomb)
    energy = 0.5 * float(np.sum(G * np.abs(FQ) ** 2))
    phi = (np.fft.ifftn(G * FQ).real * (K[0] * K[1] * K[2])).ravel()
    ph = phi[f]                                                 # [N][n^3]
    d0 = (dw[:, 0, :, None, None] * w[:, 1, None, :, None] * w[:, 2, None, None, :]).reshape(N, -1)
    d1 = (w[:, 0, :, None, None] * dw[:, 1, None, :, None] * w[:, 2, None, None, :]).reshape(N, -1)
    d2 = (w[:, 0, :, None, None] * w[:, 1, None, :, None] * dw[:, 2, None, None, :]).reshape(N, -1)
    grad = np.stack([(d0 * ph).sum(1) * K[0] / box[0],
                     (d1 * ph).sum(1) * K[1] / box[1],
                     (d2 * ph).sum(1) * K[2] / box[2]], axis=1) * q[:, None]
    return energy, grad


def ewald_recip_direct(x, q, box, alpha, kmax, coulomb):
    """Classic Ewald reciprocal energy and gradient by the direct sum over |m_a| <= kmax."""
    V = float(np.prod(box))
    r = np.arange(-kmax, kmax + 1)
    m = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    m = m[np.any(m != 0, axis=1)] / box
    msq = (m * m).sum(1)
    pref = np.exp(-math.pi ** 2 * msq / alpha ** 2) / msq
    keep = pref > 1e-300
    m, msq, pref = m[keep], msq[keep], pref[keep]
    E = 0.0
    grad = np.zeros_like(x)
    for c0 in range(0, len(m), 4096):
        mm, pp = m[c0:c0 + 4096], pref[c0:c0 + 4096]
        ph = 2.0 * math.pi * x @ mm.T                    # [N][M]
        c, s = np.cos(ph), np.sin(ph)
        Sr = q @ c
        Si = q @ s
        E += float((pp * (Sr * Sr + Si * Si)).sum())
        # d|S|^2/dx_j = 2 q_j 2 pi m (-sin Sr + cos Si)
        g = (q[:, None] * (-s * Sr[None, :] + c * Si[None, :]) * pp[None, :]) @ mm
        grad += 2.0 * 2.0 * math.pi * g
    scale = coulomb / (2.0 * math.pi * V)
    return E * scale, grad * scale
