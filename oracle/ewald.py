"""Converged classical Ewald sum (paper Sec. II, eqs. 6-10) -- TEST INFRASTRUCTURE ONLY.

Tin-foil boundary conditions (k = 0 dropped, eq. 4).  For a net charge Q the
standard uniform-background term -pi Q^2 / (2 V alpha^2) is added, so the
result is the k != 0 periodic Coulomb energy for any input.  With
alpha = 1 / (sqrt(2) sigma):

  E_real  = 1/2 sum_{i,j,n}' q_i q_j erfc(alpha r) / r        (eq. 6, near)
  E_recip = (2 pi / V) sum_{k != 0} exp(-k^2 / (4 alpha^2)) / k^2 |S(k)|^2   (eq. 10)
  E_self  = -alpha / sqrt(pi) sum q_i^2                        (eq. 10)

Both sums are taken until their terms fall below 1e-17 relative, so the
result is exact to rounding for the small cells it is used on.
"""
import math

import numpy as np
from scipy.special import erfc


def ewald(xyz, q, box, alpha=None, tol=1e-17):
    """Returns (energy, forces[n, 3]) in Gaussian units."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    box = np.asarray(box, dtype=np.float64).reshape(3)
    n = q.shape[0]
    V = float(np.prod(box))
    if alpha is None:
        alpha = 5.0 / float(np.min(box))
    # real space: erfc(alpha r) < tol beyond r_cut
    x = 1.0
    while erfc(x) > tol:
        x += 0.05
    rcut = x / alpha
    M = [int(math.ceil(rcut / L)) + 1 for L in box]
    d0 = xyz[:, None, :] - xyz[None, :, :]
    E = 0.0
    F = np.zeros((n, 3))
    for mx in range(-M[0], M[0] + 1):
        for my in range(-M[1], M[1] + 1):
            for mz in range(-M[2], M[2] + 1):
                d = d0 + np.array([mx * box[0], my * box[1], mz * box[2]])
                r = np.sqrt(np.sum(d * d, axis=2))
                if mx == 0 and my == 0 and mz == 0:
                    np.fill_diagonal(r, np.inf)
                mask = r < rcut
                rr = np.where(mask, r, 1.0)
                qq = q[:, None] * q[None, :]
                e = np.where(mask, qq * erfc(alpha * rr) / rr, 0.0)
                E += 0.5 * np.sum(e)
                # -dE/dr along d/r
                g = np.where(mask, qq * (erfc(alpha * rr) / rr ** 2
                                         + 2 * alpha / math.sqrt(math.pi)
                                         * np.exp(-(alpha * rr) ** 2) / rr) / rr, 0.0)
                F += np.sum(g[:, :, None] * d, axis=1)
    # reciprocal space: exp(-k^2/4alpha^2) < tol beyond k_cut
    kcut = 2.0 * alpha * math.sqrt(math.log(1.0 / tol))
    mm = [int(math.ceil(kcut * L / (2 * math.pi))) for L in box]
    grids = np.meshgrid(*[np.arange(-m, m + 1) for m in mm], indexing="ij")
    kv = np.stack([g.reshape(-1) * 2 * math.pi / L for g, L in zip(grids, box)], axis=1)
    k2 = np.sum(kv * kv, axis=1)
    keep = (k2 > 0) & (k2 <= kcut * kcut)
    kv, k2 = kv[keep], k2[keep]
    c = 4 * math.pi * np.exp(-k2 / (4 * alpha * alpha)) / k2
    ph = xyz @ kv.T                                  # [n, nk]
    cs, sn = np.cos(ph), np.sin(ph)
    sr = q @ cs
    si = q @ sn
    E += np.sum(c * (sr * sr + si * si)) / (2 * V)
    im = sn * sr[None, :] - cs * si[None, :]         # Im(exp(i k r_i) conj S)
    F += (q[:, None] / V) * ((im * c[None, :]) @ kv)
    # self and background
    E -= alpha / math.sqrt(math.pi) * np.sum(q * q)
    Q = np.sum(q)
    E -= math.pi * Q * Q / (2 * V * alpha * alpha)
    return E, F
