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


def ewald_sampled(x, Q, targets, L=1.0, alpha=None, rcut=None, mmax=None, forces=False, chunk=4):
    """Tin-foil Ewald potential (and forces) at a few target charges of a
    large system, the same sum as ewald() with the splitting moved so that
    the real-space part does most of the work: real space over every pair
    closer than rcut (images n in {-1, 0, 1}^3 cover rcut <= L), reciprocal
    space over the cube |m_d| <= mmax, the structure factor of all charges
    formed from separable per-axis exponentials (one product per m_x and
    m_y, then a matrix product over m_z).  Defaults alpha = 6/L, rcut = L,
    mmax = 12: erfc(6) ~ 2e-17 and exp(-k^2 / 4 alpha^2) ~ 7e-18 at the
    first omitted shell, so the truncation is below float64 rounding."""
    x = np.asarray(x, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    targets = np.asarray(targets)
    alpha = 6.0 / L if alpha is None else alpha
    rcut = L if rcut is None else rcut
    mmax = 12 if mmax is None else mmax
    if rcut > L:
        raise ValueError("rcut must not exceed L (images beyond the first shell are not visited)")
    V = L ** 3
    nt = len(targets)
    xt = x[targets]
    phi = np.zeros(nt)
    F = np.zeros((nt, 3)) if forces else None
    shifts = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)], float) * L
    for s0 in range(0, nt, chunk):
        sl = slice(s0, min(nt, s0 + chunk))
        for sh in shifts:
            d = xt[sl, None, :] - x[None, :, :] + sh[None, None, :]
            r2 = np.sum(d * d, axis=2)
            mask = r2 < rcut * rcut
            if not sh.any():
                mask[np.arange(sl.stop - sl.start), targets[sl]] = False
            ti, jj = np.nonzero(mask)
            r = np.sqrt(r2[ti, jj])
            ar = alpha * r
            ec = erfc(ar)
            cnt = sl.stop - sl.start
            phi[sl] += np.bincount(ti, weights=Q[jj] * ec / r, minlength=cnt)
            if forces:
                fac = Q[jj] * (ec / r + 2.0 * alpha / math.sqrt(math.pi) * np.exp(-ar * ar)) / (r * r)
                for k in range(3):
                    F[sl, k] += np.bincount(ti, weights=fac * d[ti, jj, k], minlength=cnt)
    m = np.arange(-mmax, mmax + 1)
    tw = 2.0 * math.pi / L
    Ex = np.exp(1j * tw * np.outer(x[:, 0], m))
    Ey = np.exp(1j * tw * np.outer(x[:, 1], m))
    Ez = np.exp(1j * tw * np.outer(x[:, 2], m))
    S = np.empty((len(m), len(m), len(m)), dtype=np.complex128)     # [mx, my, mz]
    for ix in range(len(m)):
        A = (Q * Ex[:, ix])[:, None] * Ey
        S[ix] = A.T @ Ez
    del Ex, Ey, Ez
    kx, ky, kz = np.meshgrid(tw * m, tw * m, tw * m, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    k2[mmax, mmax, mmax] = np.inf
    W = np.exp(-k2 / (4 * alpha * alpha)) / k2                     # zero at m = 0
    et = (np.exp(-1j * tw * np.outer(xt[:, 0], m))[:, :, None, None]
          * np.exp(-1j * tw * np.outer(xt[:, 1], m))[:, None, :, None]
          * np.exp(-1j * tw * np.outer(xt[:, 2], m))[:, None, None, :])   # (nt, mx, my, mz)
    z = et * S[None]
    phi += (4.0 * math.pi / V) * np.einsum("tabc,abc->t", np.real(z), W)
    phi -= 2.0 * alpha * Q[targets] / math.sqrt(math.pi)
    out = {"Phi": phi}
    if forces:
        F *= Q[targets][:, None]
        # F_t = -Q_t grad Phi(x_t), grad Phi = (4 pi / V) sum_k W_k k Im[S_k e^{-i k.x}]
        im = np.imag(z) * W[None]
        g = np.stack([np.einsum("tabc,abc->t", im, kk) for kk in (kx, ky, kz)], axis=1)
        F -= (4.0 * math.pi / V) * Q[targets][:, None] * g
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
