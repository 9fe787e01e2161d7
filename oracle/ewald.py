"""Classic Ewald summation and direct image sums (oracle ground truth).

Periodic 1/R potential of eq. potential / energy of eq. potentialenergy for a
neutral set of charges in the cube [0, L]^3, tin-foil (conducting) boundary,
k = 0 term omitted:

  Phi_i = sum_j sum'_n Q_j erfc(a r)/r                       (real space)
        + (4 pi / V) sum_{k != 0} exp(-k^2/4a^2)/k^2 Re[S(k) e^{-i k.x_i}]
        - 2 a Q_i / sqrt(pi)                                  (self)
  S(k) = sum_j Q_j e^{i k.x_j},  k = 2 pi m / L.

The paper compares against Ewald with a^2 = 6.25 (L = 1), two periodic images
in real space and four Fourier modes per direction (Section 4); those are
the defaults here, read as |n_d| <= 2 and |m_d| <= 4.

Forces are the analytic gradient F_i = -dU/dx_i.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc


def ewald(x, Q, L=1.0, alpha=None, nimg=2, mmax=4, forces=False, targets=None):
    x = np.asarray(x, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    N = len(Q)
    alpha = 2.5 / L if alpha is None else alpha
    V = L ** 3
    targets = np.arange(N) if targets is None else np.asarray(targets)
    xt = x[targets]
    phi = np.zeros(len(targets))
    F = np.zeros((len(targets), 3)) if forces else None
    rng = range(-nimg, nimg + 1)
    cells = np.array([(a, b, c) for a in rng for b in rng for c in rng], dtype=np.float64) * L
    for ci, sh in enumerate(cells):
        d = xt[:, None, :] - x[None, :, :] + sh[None, None, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        if not sh.any():
            r[np.arange(len(targets)), targets] = np.inf
        ar = alpha * r
        ec = erfc(ar)
        phi += np.sum(Q[None, :] * ec / r, axis=1)
        if forces:
            fac = (ec / r + 2.0 * alpha / math.sqrt(math.pi) * np.exp(-ar * ar)) / (r * r)
            F += np.einsum("ij,ijk->ik", Q[None, :] * fac, d)
    m = np.arange(-mmax, mmax + 1)
    M = np.array([(a, b, c) for a in m for b in m for c in m if (a, b, c) != (0, 0, 0)],
                 dtype=np.float64)
    K = 2.0 * math.pi * M / L
    k2 = np.sum(K * K, axis=1)
    A = np.exp(-k2 / (4 * alpha * alpha)) / k2
    S = np.exp(1j * (x @ K.T)).T @ Q                       # (nk,)
    et = np.exp(-1j * (xt @ K.T))                          # (nt, nk)
    phi += (4.0 * math.pi / V) * np.real(et * S[None, :]) @ A
    phi -= 2.0 * alpha * Q[targets] / math.sqrt(math.pi)
    out = {"Phi": phi}
    if len(targets) == N:
        out["U"] = 0.5 * float(np.sum(Q * phi))
    if forces:
        F *= Q[targets][:, None]
        # F_i = (4 pi / V) Q_i sum_k A_k k Im[conj(S_k) e^{i k.x_i}]
        im = np.imag(np.conj(S)[None, :] * np.conj(et))    # Im[S* e^{ikx}]
        F += (4.0 * math.pi / V) * Q[targets][:, None] * ((im * A[None, :]) @ K)
        out["F"] = F
    return out


def direct_image_energy(x, Q, L=1.0, R=20):
    """Energy by direct summation over whole periodic cells with |n| <= R
    (spherical order of cells), excluding i = j in the central cell."""
    x = np.asarray(x, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    r = np.arange(-R, R + 1)
    n = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    n = n[np.sum(n * n, axis=1) <= R * R].astype(np.float64) * L
    U = 0.0
    N = len(Q)
    for i in range(N):
        d = x[i][None, None, :] - x[None, :, :] + n[:, None, :]
        dist = np.sqrt(np.sum(d * d, axis=2))
        c0 = np.nonzero(np.all(n == 0, axis=1))[0][0]
        dist[c0, i] = np.inf
        U += 0.5 * Q[i] * np.sum(Q[None, :] / dist)
    return U


def surface_term(x, Q, L=1.0):
    """Spherical-vacuum minus tin-foil energy: (2 pi / 3 V) |sum_j Q_j x_j|^2."""
    D = np.sum(np.asarray(Q)[:, None] * np.asarray(x), axis=0)
    return 2.0 * math.pi / (3.0 * L ** 3) * float(D @ D)
