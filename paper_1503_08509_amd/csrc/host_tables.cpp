// Create-time near-field tables: order-p Dirichlet FE solutions for the
// basis screens R_a = r_ax (x) r_ay (x) r_az on a B^3-element box centred on
// the source element (Remark of Section 4), stored by their nodal values on
// the (2 n_sr + 1)^3 near block.  Dirichlet data: exact free-space potential
// of R_a, evaluated through 1/r = (2/sqrt(pi)) int_0^inf exp(-r^2 t^2) dt,
// which separates into 1-D factors for a tensor-product density.
#include "host_tables.hpp"

#include <cmath>
#include <stdexcept>
#include <thread>

namespace fep3m {
namespace {

// J_k = int_A^B s^k exp(-s^2) ds, k = 0..kmax.
void gauss_moments(double A, double B, int kmax, double *J) {
  const double sp = std::sqrt(M_PI);
  double j0;
  if (A >= 0) j0 = 0.5 * sp * (std::erfc(A) - std::erfc(B));
  else if (B <= 0) j0 = 0.5 * sp * (std::erfc(-B) - std::erfc(-A));
  else j0 = 0.5 * sp * (std::erf(B) - std::erf(A));
  J[0] = j0;
  double eA = std::exp(-A * A), eB = std::exp(-B * B);
  if (kmax >= 1) J[1] = 0.5 * (eA - eB);
  for (int k = 2; k <= kmax; ++k)
    J[k] = 0.5 * (k - 1) * J[k - 2] + 0.5 * (std::pow(A, k - 1) * eA - std::pow(B, k - 1) * eB);
}

// F(t; x) = int_{-1/2}^{1/2} f(s) exp(-t^2 (x - s)^2) ds for the polynomial f
// with ascending monomial coefficients c.
struct GaussFactor {
  Vec sq, sw;
  GaussFactor() { gauss_legendre(48, sq, sw); }
  double operator()(const Vec &c, double t, double x) const {
    const int deg = int(c.size()) - 1;
    if (t <= 4.0) {  // wide Gaussian: Gauss-Legendre in s
      double s = 0.0;
      for (size_t i = 0; i < sq.size(); ++i) {
        double f = 0.0;
        for (int k = deg; k >= 0; --k) f = f * sq[i] + c[k];
        double dx = x - sq[i];
        s += sw[i] * f * std::exp(-t * t * dx * dx);
      }
      return s;
    }
    double dist = std::max(std::max(-0.5 - x, x - 0.5), 0.0);
    if (t * dist > 10.0) return 0.0;
    // s = t (xi - x): F = (1/t) sum_j f^(j)(x)/j! t^-j J_j(A, B)
    double A = t * (-0.5 - x), B = t * (0.5 - x);
    double J[16];
    gauss_moments(A, B, deg, J);
    Vec dc = c;
    double fact = 1.0, val = 0.0, tp = t;
    for (int j = 0; j <= deg; ++j) {
      double dj = 0.0;
      for (int k = int(dc.size()) - 1; k >= 0; --k) dj = dj * x + dc[k];
      val += dj / fact * J[j] / tp;
      // derivative of dc
      Vec nd(std::max<size_t>(1, dc.size() - 1), 0.0);
      for (size_t k = 1; k < dc.size(); ++k) nd[k - 1] = dc[k] * double(k);
      dc = nd;
      fact *= (j + 1);
      tp *= t;
    }
    return val;
  }
};

// Composite Gauss-Legendre rule in tau = ln t, weights including dt/dtau
// and the 2/sqrt(pi) of the Gaussian identity.
void tau_rule(Vec &t, Vec &w) {
  Vec gx, gw;
  gauss_legendre(16, gx, gw);  // on [-1/2, 1/2]
  t.clear();
  w.clear();
  for (double a = -36.0; a < 22.0 - 1e-12; a += 0.5) {
    for (size_t i = 0; i < gx.size(); ++i) {
      double tau = a + 0.25 + 0.5 * gx[i];
      double tt = std::exp(tau);
      t.push_back(tt);
      w.push_back(0.5 * gw[i] * tt * 2.0 / std::sqrt(M_PI));
    }
  }
}

// Y = A applied along one axis of a 3-D array X[nz][ny][nx] (x fastest).
// A maps the axis extent A.c -> A.r.  Dims of X given; returns dims of Y.
void apply_axis(const Mat &A, const Vec &X, int nz, int ny, int nx, int axis, Vec &Y) {
  int oz = nz, oy = ny, ox = nx;
  if (axis == 0) ox = A.r; else if (axis == 1) oy = A.r; else oz = A.r;
  Y.assign(size_t(oz) * oy * ox, 0.0);
  for (int k = 0; k < oz; ++k)
    for (int j = 0; j < oy; ++j)
      for (int i = 0; i < ox; ++i) {
        double s = 0.0;
        if (axis == 0) {
          const double *row = &A.a[size_t(i) * A.c];
          const double *xr = &X[(size_t(k) * ny + j) * nx];
          for (int c = 0; c < A.c; ++c) s += row[c] * xr[c];
        } else if (axis == 1) {
          const double *row = &A.a[size_t(j) * A.c];
          for (int c = 0; c < A.c; ++c) s += row[c] * X[(size_t(k) * ny + c) * nx + i];
        } else {
          const double *row = &A.a[size_t(k) * A.c];
          for (int c = 0; c < A.c; ++c) s += row[c] * X[(size_t(c) * ny + j) * nx + i];
        }
        Y[(size_t(k) * oy + j) * ox + i] = s;
      }
}

Mat transpose(const Mat &A) {
  Mat T(A.c, A.r);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
  return T;
}

}  // namespace

void compute_tables(int p, const Screen1D &scr, int n_sr, int B, Vec &T) {
  if (B % 2 == 0 || B < 2 * n_sr + 3) throw std::runtime_error("table box must be odd and exceed the near block");
  const int d = scr.d, nb1 = d + 1, nb = nb1 * nb1 * nb1;
  const int S = 2 * n_sr + 1, np1 = p + 1;
  const int c = (B - 1) / 2;
  const int nn = B * p + 1, ni = nn - 2;
  Vec g1 = gll_nodes(p);
  Vec coord(nn);
  for (int e = 0; e < B; ++e)
    for (int k = 0; k < p; ++k) coord[p * e + k] = (e - c) + g1[k];
  coord[nn - 1] = (B - c) - 0.5;

  Mat K1, M1;
  assemble_1d(p, B, false, K1, M1);
  Mat Ki(ni, ni), Mi(ni, ni);
  for (int i = 0; i < ni; ++i)
    for (int j = 0; j < ni; ++j) { Ki(i, j) = K1(i + 1, j + 1); Mi(i, j) = M1(i + 1, j + 1); }
  Vec lam;
  Mat V;
  sym_gen_eig(Ki, Mi, lam, V);
  Mat Vt = transpose(V);
  // rows of V for the near-block nodes (global p(c - n_sr) .. p(c + n_sr + 1))
  const int g0 = p * (c - n_sr), nblk = S * p + 1;
  Mat Vs(nblk, ni);
  for (int r = 0; r < nblk; ++r)
    for (int j = 0; j < ni; ++j) Vs(r, j) = V(g0 + r - 1, j);

  Mat G = load_weights(p, scr);
  Vec tq, tw;
  tau_rule(tq, tw);
  const int NT = int(tq.size());
  GaussFactor gf;
  // F_l(t, coord_i) for each l: [l][i][t]
  std::vector<Vec> F(nb1, Vec(size_t(nn) * NT));
  for (int l = 0; l < nb1; ++l) {
    Vec mono = scr.monomial(l);
    for (int i = 0; i < nn; ++i)
      for (int it = 0; it < NT; ++it) F[l][size_t(i) * NT + it] = gf(mono, tq[it], coord[i]);
  }

  T.assign(size_t(nb) * S * S * S * np1 * np1 * np1, 0.0);
  auto work = [&](int ia) {
    const int ax = ia % nb1, ay = (ia / nb1) % nb1, az = ia / (nb1 * nb1);
    // exact potential on the boundary nodes (Dirichlet data)
    Vec gext(size_t(nn) * nn * nn, 0.0);
    for (int k = 0; k < nn; ++k)
      for (int j = 0; j < nn; ++j)
        for (int i = 0; i < nn; ++i) {
          bool bnd = (i == 0 || j == 0 || k == 0 || i == nn - 1 || j == nn - 1 || k == nn - 1);
          if (!bnd) continue;
          const double *fx = &F[ax][size_t(i) * NT];
          const double *fy = &F[ay][size_t(j) * NT];
          const double *fz = &F[az][size_t(k) * NT];
          double s = 0.0;
          for (int it = 0; it < NT; ++it) s += tw[it] * fx[it] * fy[it] * fz[it];
          gext[(size_t(k) * nn + j) * nn + i] = s;
        }
    // rhs = 4 pi G_a (source element) - K g_ext
    Vec t1, t2, t3, Kg(gext.size(), 0.0);
    apply_axis(M1, gext, nn, nn, nn, 2, t1);      // Mz
    apply_axis(M1, t1, nn, nn, nn, 1, t2);        // My Mz
    apply_axis(K1, t2, nn, nn, nn, 0, t3);        // Kx My Mz
    for (size_t i = 0; i < Kg.size(); ++i) Kg[i] += t3[i];
    apply_axis(M1, t1, nn, nn, nn, 0, t2);        // Mx Mz
    apply_axis(K1, t2, nn, nn, nn, 1, t3);        // Ky Mx Mz
    for (size_t i = 0; i < Kg.size(); ++i) Kg[i] += t3[i];
    apply_axis(K1, gext, nn, nn, nn, 2, t1);      // Kz
    apply_axis(M1, t1, nn, nn, nn, 1, t2);
    apply_axis(M1, t2, nn, nn, nn, 0, t3);        // Mx My Kz
    for (size_t i = 0; i < Kg.size(); ++i) Kg[i] += t3[i];
    Vec r(size_t(ni) * ni * ni);
    for (int k = 0; k < ni; ++k)
      for (int j = 0; j < ni; ++j)
        for (int i = 0; i < ni; ++i) {
          size_t gi = (size_t(k + 1) * nn + (j + 1)) * nn + (i + 1);
          double b = 0.0;
          int mk = k + 1 - p * c, mj = j + 1 - p * c, mi = i + 1 - p * c;
          if (mk >= 0 && mk <= p && mj >= 0 && mj <= p && mi >= 0 && mi <= p)
            b = 4.0 * M_PI * G(az, mk) * G(ay, mj) * G(ax, mi);
          r[(size_t(k) * ni + j) * ni + i] = b - Kg[gi];
        }
    apply_axis(Vt, r, ni, ni, ni, 0, t1);
    apply_axis(Vt, t1, ni, ni, ni, 1, t2);
    apply_axis(Vt, t2, ni, ni, ni, 2, t1);
    for (int k = 0; k < ni; ++k)
      for (int j = 0; j < ni; ++j)
        for (int i = 0; i < ni; ++i) t1[(size_t(k) * ni + j) * ni + i] /= (lam[i] + lam[j] + lam[k]);
    apply_axis(Vs, t1, ni, ni, ni, 0, t2);
    apply_axis(Vs, t2, ni, ni, nblk, 1, t3);
    apply_axis(Vs, t3, ni, nblk, nblk, 2, t2);   // w on the block nodes [nblk]^3
    for (int Dz = 0; Dz < S; ++Dz)
      for (int Dy = 0; Dy < S; ++Dy)
        for (int Dx = 0; Dx < S; ++Dx) {
          size_t iD = (size_t(Dz) * S + Dy) * S + Dx;
          for (int mz = 0; mz <= p; ++mz)
            for (int my = 0; my <= p; ++my)
              for (int mx = 0; mx <= p; ++mx) {
                size_t src = (size_t(p * Dz + mz) * nblk + (p * Dy + my)) * nblk + (p * Dx + mx);
                size_t m = (size_t(mz) * np1 + my) * np1 + mx;
                T[(size_t(ia) * S * S * S + iD) * np1 * np1 * np1 + m] = t2[src];
              }
        }
  };
  std::vector<std::thread> th;
  for (int ia = 0; ia < nb; ++ia) th.emplace_back(work, ia);
  for (auto &t : th) t.join();
}

}  // namespace fep3m
