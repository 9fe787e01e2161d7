"""1-D finite element ingredients (oracle).

Order-p Lagrange elements on Gauss-Lobatto-Legendre nodes, written in
element units: one element is the interval [-1/2, 1/2] (h = 1).  The 3-D
operators of the mesh solve (Section 2.2, "Solution of the mesh potential")
are Kronecker sums of these 1-D matrices on a uniform tensor mesh:

    K = K1 (x) M1 (x) M1 + M1 (x) K1 (x) M1 + M1 (x) M1 (x) K1,

which is exactly the Galerkin stiffness matrix of the tensor-product Q_p
space.  Integrals use Gauss-Legendre quadrature with p+1 points, exact for
every integrand used here (degree <= 2p+1).  The choice of nodes does not
change the FE space (only its basis), so GLL nodes are used for conditioning.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_legendre(m):
    """m-point Gauss-Legendre rule on [-1/2, 1/2]."""
    t, w = npleg.leggauss(m)
    return 0.5 * t, 0.5 * w


def gll_nodes(p):
    """p+1 Gauss-Lobatto-Legendre nodes on [-1/2, 1/2]: the end points and
    the roots of P_p'."""
    if p == 1:
        return np.array([-0.5, 0.5])
    c = np.zeros(p + 1)
    c[p] = 1.0
    inner = np.sort(np.real(npleg.legroots(npleg.legder(c))))
    return 0.5 * np.concatenate([[-1.0], inner, [1.0]])


def lagrange(nodes, x):
    """Values of the Lagrange basis on `nodes` at points x: shape (len(x), n)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.ones((len(x), n))
    for k in range(n):
        for j in range(n):
            if j != k:
                out[:, k] *= (x - nodes[j]) / (nodes[k] - nodes[j])
    return out


def lagrange_deriv(nodes, x):
    """Derivatives of the Lagrange basis at x (product rule, valid at nodes)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.zeros((len(x), n))
    for k in range(n):
        for j in range(n):
            if j == k:
                continue
            term = np.full(len(x), 1.0 / (nodes[k] - nodes[j]))
            for m in range(n):
                if m != k and m != j:
                    term *= (x - nodes[m]) / (nodes[k] - nodes[m])
            out[:, k] += term
    return out


def element_matrices(p):
    """Element stiffness k_e[a,b] = int l_a' l_b' and mass m_e[a,b] = int l_a l_b
    on one element of unit size."""
    nodes = gll_nodes(p)
    xq, wq = gauss_legendre(p + 1)
    L = lagrange(nodes, xq)
    D = lagrange_deriv(nodes, xq)
    ke = (D * wq[:, None]).T @ D
    me = (L * wq[:, None]).T @ L
    return ke, me


def periodic_matrices(p, n):
    """Periodic assembly of K1, M1 over n unit elements: p*n DOFs, global
    node index p*e + k (mod p*n)."""
    ke, me = element_matrices(p)
    N = p * n
    K = np.zeros((N, N))
    M = np.zeros((N, N))
    for e in range(n):
        idx = (p * e + np.arange(p + 1)) % N
        K[np.ix_(idx, idx)] += ke
        M[np.ix_(idx, idx)] += me
    return K, M


def dirichlet_matrices(p, n):
    """Non-periodic assembly over n unit elements: p*n+1 DOFs (all nodes,
    boundary rows included; the caller restricts to the interior)."""
    ke, me = element_matrices(p)
    N = p * n + 1
    K = np.zeros((N, N))
    M = np.zeros((N, N))
    for e in range(n):
        idx = p * e + np.arange(p + 1)
        K[np.ix_(idx, idx)] += ke
        M[np.ix_(idx, idx)] += me
    return K, M


def kron_apply(A, B, C, X):
    """(A (x) B (x) C) applied to a 3-D array X indexed [z, y, x]
    (A acts on z, B on y, C on x)."""
    Y = np.einsum("ij,jkl->ikl", A, X, optimize=True)
    Y = np.einsum("ij,kjl->kil", B, Y, optimize=True)
    Y = np.einsum("ij,klj->kli", C, Y, optimize=True)
    return Y


def stiffness_apply(K1, M1, X):
    """3-D periodic stiffness K applied to X[z, y, x]."""
    return (kron_apply(K1, M1, M1, X) + kron_apply(M1, K1, M1, X)
            + kron_apply(M1, M1, K1, X))
