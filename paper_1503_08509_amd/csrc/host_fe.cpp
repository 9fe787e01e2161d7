// Host-side finite element and screen ingredients (see host_fe.hpp).
#include "host_fe.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <stdexcept>

namespace fep3m {

static void legendre_pair(int n, double x, double &pn, double &pnm1) {
  // Three-term recurrence: (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}.
  double p0 = 1.0, p1 = x;
  if (n == 0) { pn = 1.0; pnm1 = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pnm1 = p0;
}

void gauss_legendre(int m, Vec &x, Vec &w) {
  // Newton iteration on P_m from the classical cosine initial guesses;
  // weights 2 / ((1 - t^2) P_m'(t)^2) on [-1, 1], halved for [-1/2, 1/2].
  x.assign(m, 0.0);
  w.assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (m + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double pn, pm;
      legendre_pair(m, t, pn, pm);
      dp = m * (t * pn - pm) / (t * t - 1.0);
      double dt = pn / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double pn, pm;
    legendre_pair(m, t, pn, pm);
    dp = m * (t * pn - pm) / (t * t - 1.0);
    x[m - 1 - i] = 0.5 * t;
    w[m - 1 - i] = 0.5 * 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

Vec gll_nodes(int p) {
  // Interior nodes are the roots of P_p'; Newton on f = t P_p - P_{p-1}
  // (proportional to (1 - t^2) P_p') with f' = (p + 1) P_p, started from
  // the Chebyshev-Gauss-Lobatto points.
  Vec out(p + 1);
  for (int k = 0; k <= p; ++k) {
    double t = -std::cos(M_PI * k / p);
    if (k > 0 && k < p) {
      for (int it = 0; it < 100; ++it) {
        double pn, pm;
        legendre_pair(p, t, pn, pm);
        double dt = (t * pn - pm) / ((p + 1.0) * pn);
        t -= dt;
        if (std::fabs(dt) < 1e-16) break;
      }
    }
    out[k] = 0.5 * t;
  }
  out[0] = -0.5;
  out[p] = 0.5;
  return out;
}

void lagrange(const Vec &nodes, double x, double *out, double *dout) {
  const int n = int(nodes.size());
  for (int k = 0; k < n; ++k) {
    double v = 1.0;
    for (int j = 0; j < n; ++j)
      if (j != k) v *= (x - nodes[j]) / (nodes[k] - nodes[j]);
    out[k] = v;
    if (dout) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) {
        if (j == k) continue;
        double t = 1.0 / (nodes[k] - nodes[j]);
        for (int m = 0; m < n; ++m)
          if (m != k && m != j) t *= (x - nodes[m]) / (nodes[k] - nodes[m]);
        s += t;
      }
      dout[k] = s;
    }
  }
}

void element_matrices(int p, Mat &ke, Mat &me) {
  Vec nodes = gll_nodes(p), xq, wq;
  gauss_legendre(p + 1, xq, wq);  // exact for degree <= 2p + 1
  ke = Mat(p + 1, p + 1);
  me = Mat(p + 1, p + 1);
  Vec l(p + 1), dl(p + 1);
  for (size_t iq = 0; iq < xq.size(); ++iq) {
    lagrange(nodes, xq[iq], l.data(), dl.data());
    for (int a = 0; a <= p; ++a)
      for (int b = 0; b <= p; ++b) {
        ke(a, b) += wq[iq] * dl[a] * dl[b];
        me(a, b) += wq[iq] * l[a] * l[b];
      }
  }
}

void sym_eig(const Mat &A0, Vec &w, Mat &V) {
  const int n = A0.r;
  Mat A = A0;
  V = Mat(n, n);
  for (int i = 0; i < n; ++i) V(i, i) = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += A(i, i) * A(i, i);
      for (int j = i + 1; j < n; ++j) off += A(i, j) * A(i, j);
    }
    if (off <= 1e-34 * diag || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J
          double akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * akq;
          A(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A
          double apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * aqk;
          A(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V(k, p), vkq = V(k, q);
          V(k, p) = c * vkp - s * vkq;
          V(k, q) = s * vkp + c * vkq;
        }
      }
    }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A(a, a) < A(b, b); });
  w.assign(n, 0.0);
  Mat Vs(n, n);
  for (int j = 0; j < n; ++j) {
    w[j] = A(idx[j], idx[j]);
    for (int i = 0; i < n; ++i) Vs(i, j) = V(i, idx[j]);
  }
  V = Vs;
}

void sym_gen_eig(const Mat &K, const Mat &M, Vec &w, Mat &V) {
  // Cholesky M = L L^T, then A = L^-1 K L^-T, A = W diag(w) W^T, V = L^-T W.
  const int n = M.r;
  Mat L(n, n);
  for (int j = 0; j < n; ++j) {
    double s = M(j, j);
    for (int k = 0; k < j; ++k) s -= L(j, k) * L(j, k);
    if (s <= 0) throw std::runtime_error("mass matrix not positive definite");
    L(j, j) = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = M(i, j);
      for (int k = 0; k < j; ++k) t -= L(i, k) * L(j, k);
      L(i, j) = t / L(j, j);
    }
  }
  // Y = L^-1 K  (forward substitution per column)
  Mat Y(n, n);
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double t = K(i, c);
      for (int k = 0; k < i; ++k) t -= L(i, k) * Y(k, c);
      Y(i, c) = t / L(i, i);
    }
  // A = Y L^-T, i.e. A^T = L^-1 Y^T
  Mat A(n, n);
  for (int r = 0; r < n; ++r)
    for (int i = 0; i < n; ++i) {
      double t = Y(r, i);
      for (int k = 0; k < i; ++k) t -= L(i, k) * A(r, k);
      A(r, i) = t / L(i, i);
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double s = 0.5 * (A(i, j) + A(j, i));
      A(i, j) = A(j, i) = s;
    }
  Mat W;
  sym_eig(A, w, W);
  // V = L^-T W: back substitution with L^T
  V = Mat(n, n);
  for (int c = 0; c < n; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double t = W(i, c);
      for (int k = i + 1; k < n; ++k) t -= L(k, i) * V(k, c);
      V(i, c) = t / L(i, i);
    }
}

Mat inverse(const Mat &A0) {
  const int n = A0.r;
  Mat A = A0, I(n, n);
  for (int i = 0; i < n; ++i) I(i, i) = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A(r, col)) > std::fabs(A(piv, col))) piv = r;
    if (A(piv, col) == 0.0) throw std::runtime_error("singular matrix");
    for (int k = 0; k < n; ++k) {
      std::swap(A(col, k), A(piv, k));
      std::swap(I(col, k), I(piv, k));
    }
    double pv = A(col, col);
    for (int k = 0; k < n; ++k) { A(col, k) /= pv; I(col, k) /= pv; }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double f = A(r, col);
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { A(r, k) -= f * A(col, k); I(r, k) -= f * I(col, k); }
    }
  }
  return I;
}

namespace {

// int_{-1/2}^{1/2} (t + o)^m c(t) dt for the polynomial c of degree deg
// (ascending coefficients): (t + o)^m expanded binomially, t^k integrated
// exactly.
double moment_exact(const double *c, int deg, int m, double o) {
  auto tint = [](int k) { return (k % 2) ? 0.0 : 2.0 * std::pow(0.5, k + 1) / (k + 1); };
  double s = 0.0, binom = 1.0;
  for (int j = 0; j <= m; ++j) {   // (t + o)^m = sum_j C(m, j) t^j o^(m - j)
    double tj = 0.0;
    for (int k = 0; k <= deg; ++k) tj += c[k] * tint(j + k);
    s += binom * std::pow(o, m - j) * tj;
    binom = binom * (m - j) / (j + 1);
  }
  return s;
}

// Monomial coefficients of the Lagrange polynomial of nodes[k].
Vec lagrange_monomial(const Vec &nodes, int k) {
  Vec c(1, 1.0);
  for (size_t j = 0; j < nodes.size(); ++j) {
    if (int(j) == k) continue;
    const double den = nodes[k] - nodes[j];
    Vec nc(c.size() + 1, 0.0);
    for (size_t i = 0; i < c.size(); ++i) {
      nc[i] -= c[i] * nodes[j] / den;
      nc[i + 1] += c[i] / den;
    }
    c = nc;
  }
  return c;
}

}  // namespace

double Screen1D::eval_piece(int s, int l, double t) const {
  const double *c = piece(s, l);
  double v = 0.0;
  for (int k = q; k >= 0; --k) v = v * t + c[k];
  return v;
}

double Screen1D::eval(int l, double x) const {
  const int h = (span - 1) / 2;
  const double lo = -0.5 - h, hi = 0.5 + h;
  if (x < lo || x > hi) return 0.0;
  int s = int(std::floor(x + 0.5)) + h;
  if (s >= span) s = span - 1;
  return eval_piece(s, l, x - (s - h));
}

Screen1D make_screen(int q, int support) {
  // The screen basis functions as monomial pieces, their moment matrix of
  // eq. moment1d by exact monomial integrals, and the dual functions from
  // its inverse.
  Screen1D s;
  s.q = q;
  s.support = support;
  s.span = support ? 3 : 1;
  s.d = support ? q : q - 2;
  const int nb = s.d + 1, nk = q + 1;
  // basis[i][piece] coefficients (degree q), piece 0..span-1
  std::vector<std::vector<Vec>> basis(nb, std::vector<Vec>(s.span, Vec(nk, 0.0)));
  if (!support) {
    for (int j = 0; j < nb; ++j) {       // bubble * t^j = (1/4 - t^2) t^j
      basis[j][0][j] += 0.25;
      basis[j][0][j + 2] -= 1.0;
    }
  } else {
    Vec nodes(q + 1);
    for (int k = 0; k <= q; ++k) nodes[k] = -0.5 + double(k) / q;
    for (int i = 0; i <= q; ++i) {
      basis[i][1] = lagrange_monomial(nodes, i);
      if (i == 0) basis[i][0] = lagrange_monomial(nodes, q);   // the node is the upper end of the element below
      if (i == q) basis[i][2] = lagrange_monomial(nodes, 0);   // ... and the lower end of the element above
    }
  }
  const int h = (s.span - 1) / 2;
  Mat W(nb, nb);
  for (int m = 0; m < nb; ++m)
    for (int i = 0; i < nb; ++i) {
      double t = 0.0;
      for (int pz = 0; pz < s.span; ++pz) t += moment_exact(basis[i][pz].data(), q, m, double(pz - h));
      W(m, i) = t;
    }
  Mat Wi = inverse(W);   // r_l = sum_i Wi(i, l) basis_i
  s.pc.assign(size_t(s.span) * nb * nk, 0.0);
  for (int pz = 0; pz < s.span; ++pz)
    for (int l = 0; l < nb; ++l)
      for (int i = 0; i < nb; ++i)
        for (int k = 0; k < nk; ++k) s.pc[(size_t(pz) * nb + l) * nk + k] += Wi(i, l) * basis[i][pz][k];
  return s;
}

Mat load_weights(int p, const Screen1D &s) {
  Vec nodes = gll_nodes(p), xq, wq, l(p + 1);
  gauss_legendre(p + 1, xq, wq);  // degree p + q <= 2p + 1 per element
  Mat g(s.d + 1, s.span * p + 1);
  for (int pz = 0; pz < s.span; ++pz)
    for (size_t iq = 0; iq < xq.size(); ++iq) {
      lagrange(nodes, xq[iq], l.data(), nullptr);
      for (int ll = 0; ll <= s.d; ++ll) {
        const double r = s.eval_piece(pz, ll, xq[iq]);
        for (int k = 0; k <= p; ++k) g(ll, pz * p + k) += wq[iq] * r * l[k];
      }
    }
  return g;
}

void periodic_fourier_eigen(int p, int n, Vec &Wre, Vec &Wim, Vec &lam) {
  using C = std::complex<double>;
  Mat ke, me;
  element_matrices(p, ke, me);
  Wre.assign(size_t(n) * p * p, 0.0);
  Wim.assign(size_t(n) * p * p, 0.0);
  lam.assign(size_t(n) * p, 0.0);
  for (int f = 0; f < n; ++f) {
    const double th = 2.0 * M_PI * double(f) / double(n), c = std::cos(th), sn = std::sin(th);
    std::vector<C> Kc(size_t(p) * p), Mc(size_t(p) * p);
    auto block = [&](const Mat &e, std::vector<C> &out) {
      for (int k = 0; k < p; ++k)
        for (int l = 0; l < p; ++l) out[size_t(k) * p + l] = e(k, l);
      out[0] += e(p, p);                                    // the vertex shared with the element below
      for (int k = 0; k < p; ++k) {
        out[size_t(k) * p] += e(k, p) * C(c, sn);           // owned node k -> vertex of the element above
        out[k] += e(p, k) * C(c, -sn);                      // vertex -> owned node k of the element below
      }
    };
    block(ke, Kc);
    block(me, Mc);
    // real symmetric embedding [[Re, -Im], [Im, Re]] of both Hermitian blocks
    Mat KR(2 * p, 2 * p), MR(2 * p, 2 * p);
    for (int k = 0; k < p; ++k)
      for (int l = 0; l < p; ++l) {
        const C a = Kc[size_t(k) * p + l], b = Mc[size_t(k) * p + l];
        KR(k, l) = KR(k + p, l + p) = a.real();
        KR(k, l + p) = -a.imag();
        KR(k + p, l) = a.imag();
        MR(k, l) = MR(k + p, l + p) = b.real();
        MR(k, l + p) = -b.imag();
        MR(k + p, l) = b.imag();
      }
    Vec w;
    Mat V;
    sym_gen_eig(KR, MR, w, V);
    // every eigenvalue appears twice (z and i z); keep one M^-orthonormal
    // complex vector per complex dimension, in ascending order
    auto mdot = [&](const std::vector<C> &a, const std::vector<C> &b) {
      C s = 0.0;
      for (int k = 0; k < p; ++k) {
        C t = 0.0;
        for (int l = 0; l < p; ++l) t += Mc[size_t(k) * p + l] * b[l];
        s += std::conj(a[k]) * t;
      }
      return s;
    };
    std::vector<std::vector<C>> acc;
    std::vector<double> accl;
    for (int col = 0; col < 2 * p && int(acc.size()) < p; ++col) {
      std::vector<C> z(p);
      for (int k = 0; k < p; ++k) z[k] = C(V(k, col), V(k + p, col));
      for (const auto &a : acc) {
        const C pr = mdot(a, z);
        for (int k = 0; k < p; ++k) z[k] -= pr * a[k];
      }
      const double nrm = mdot(z, z).real();
      if (nrm < 0.25) continue;
      const double sc = 1.0 / std::sqrt(nrm);
      for (C &v : z) v *= sc;
      acc.push_back(z);
      accl.push_back(w[col]);
    }
    if (int(acc.size()) != p) throw std::runtime_error("Fourier block eigenvectors");
    if (f == 0) {   // constants: the mode of smallest eigenvalue
      int i0 = 0;
      for (int i = 1; i < p; ++i)
        if (std::fabs(accl[i]) < std::fabs(accl[i0])) i0 = i;
      accl[i0] = 0.0;
    }
    for (int i = 0; i < p; ++i) {
      lam[size_t(f) * p + i] = accl[i];
      for (int k = 0; k < p; ++k) {
        Wre[(size_t(f) * p + k) * p + i] = acc[i][k].real();
        Wim[(size_t(f) * p + k) * p + i] = acc[i][k].imag();
      }
    }
  }
}

void assemble_1d(int p, int ne, bool periodic, Mat &K, Mat &M) {
  Mat ke, me;
  element_matrices(p, ke, me);
  const int N = periodic ? p * ne : p * ne + 1;
  K = Mat(N, N);
  M = Mat(N, N);
  for (int e = 0; e < ne; ++e)
    for (int a = 0; a <= p; ++a)
      for (int b = 0; b <= p; ++b) {
        int ia = p * e + a, ib = p * e + b;
        if (periodic) { ia %= N; ib %= N; }
        K(ia, ib) += ke(a, b);
        M(ia, ib) += me(a, b);
      }
}

}  // namespace fep3m
