// Create-time near-field tables (Remark of Section 4): for every basis
// screen R_a = r_ax (x) r_ay (x) r_az the order-p finite element solution of
// -lap w = 4 pi R_a on a box of B^3 elements centred on the source element,
// with the free-space potential of R_a as Dirichlet data, kept at the nodes
// of the (2 n_sr + 1)^3 near block.
//
// Dirichlet data.  The box boundary lies at least (B - 1)/2 - (span - 1)/2
// elements from every part of the screen (span = 1 or 3 elements per axis),
// so 1/|x - xi| is analytic over each source element and a tensor
// Gauss-Legendre rule per element converges geometrically; the screen
// pieces are polynomials of degree q, which the rule integrates exactly.
// kBoundaryRule points per axis and element leave an error far below 1e-15
// at the smallest admitted box (B = 2 n_sr + 3).
//
// Interior solve.  Interior unknowns only: K_ii w = 4 pi G_a - K_ib g.  The
// coupling K_ib g is assembled element by element over the outer shell of
// elements (the only ones holding boundary nodes); K_ii is the Kronecker sum
// of the interior 1-D pencil, diagonalised once (K v = lam M v, V^T M V = I).
#include "host_tables.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <stdexcept>
#include <thread>

namespace fep3m {
namespace {

constexpr int kBoundaryRule = 14;

int worker_count(int jobs) {
  const unsigned hc = std::thread::hardware_concurrency();
  return std::max(1, std::min(jobs, int(hc ? hc : 4)));
}

template <class F>
void parallel_for(int jobs, F &&f) {
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  const int nw = worker_count(jobs);
  for (int w = 0; w < nw; ++w)
    th.emplace_back([&]() {
      for (int j = next.fetch_add(1); j < jobs; j = next.fetch_add(1)) f(j);
    });
  for (auto &t : th) t.join();
}

// Free-space potential of every basis screen at the boundary nodes:
// out[b * nb + a] for boundary node b (coordinates bx, by, bz relative to
// the source element's centre).
void boundary_potentials(const Screen1D &scr, const std::vector<double> &bx, const std::vector<double> &by,
                         const std::vector<double> &bz, Vec &out) {
  const int m = kBoundaryRule, nl = scr.d + 1, nb = nl * nl * nl, sp = scr.span, h = (sp - 1) / 2;
  Vec gx, gw;
  gauss_legendre(m, gx, gw);
  // per piece: quadrature point positions (source-centre units) and the
  // weighted dual-function values wr[piece][l][i] = w_i r_l(x_i)
  Vec pos(size_t(sp) * m), wr(size_t(sp) * nl * m);
  for (int s = 0; s < sp; ++s)
    for (int i = 0; i < m; ++i) {
      pos[s * m + i] = (s - h) + gx[i];
      for (int l = 0; l < nl; ++l) wr[(size_t(s) * nl + l) * m + i] = gw[i] * scr.eval_piece(s, l, gx[i]);
    }
  const int nbnd = int(bx.size());
  out.assign(size_t(nbnd) * nb, 0.0);
  parallel_for((nbnd + 63) / 64, [&](int chunk) {
    Vec kx(m), A(nl), Bv(size_t(nl) * nl), acc(nb);
    for (int b = chunk * 64; b < std::min(nbnd, chunk * 64 + 64); ++b) {
      std::fill(acc.begin(), acc.end(), 0.0);
      for (int sz = 0; sz < sp; ++sz)
        for (int iz = 0; iz < m; ++iz) {
          const double dz = bz[b] - pos[sz * m + iz];
          std::fill(Bv.begin(), Bv.end(), 0.0);
          for (int sy = 0; sy < sp; ++sy)
            for (int iy = 0; iy < m; ++iy) {
              const double dy = by[b] - pos[sy * m + iy];
              const double dyz = dy * dy + dz * dz;
              std::fill(A.begin(), A.end(), 0.0);
              for (int sx = 0; sx < sp; ++sx) {
                for (int ix = 0; ix < m; ++ix) {
                  const double dx = bx[b] - pos[sx * m + ix];
                  kx[ix] = 1.0 / std::sqrt(dx * dx + dyz);
                }
                for (int l = 0; l < nl; ++l) {
                  const double *w = &wr[(size_t(sx) * nl + l) * m];
                  double s = 0.0;
                  for (int ix = 0; ix < m; ++ix) s += w[ix] * kx[ix];
                  A[l] += s;
                }
              }
              for (int ly = 0; ly < nl; ++ly) {
                const double wy = wr[(size_t(sy) * nl + ly) * m + iy];
                for (int lx = 0; lx < nl; ++lx) Bv[ly * nl + lx] += wy * A[lx];
              }
            }
          for (int lz = 0; lz < nl; ++lz) {
            const double wz = wr[(size_t(sz) * nl + lz) * m + iz];
            for (int j = 0; j < nl * nl; ++j) acc[lz * nl * nl + j] += wz * Bv[j];
          }
        }
      for (int a = 0; a < nb; ++a) out[size_t(b) * nb + a] = acc[a];
    }
  });
}

}  // namespace

void compute_tables(int p, const Screen1D &scr, int n_sr, int B, Vec &T) {
  if (B % 2 == 0 || B < 2 * n_sr + 3) throw std::runtime_error("table box must be odd and exceed the near block");
  const int nl = scr.d + 1, nb = nl * nl * nl, sp = scr.span;
  const int S = 2 * n_sr + 1, np1 = p + 1;
  const int c = (B - 1) / 2;
  const int nn = B * p + 1, ni = nn - 2;
  Vec g1 = gll_nodes(p);
  Vec coord(nn);   // node coordinates relative to the source element's centre
  for (int e = 0; e < B; ++e)
    for (int k = 0; k < p; ++k) coord[p * e + k] = (e - c) + g1[k];
  coord[nn - 1] = (B - c) - 0.5;

  // boundary nodes in a fixed order and their potentials
  std::vector<int> bidx;
  std::vector<double> bx, by, bz;
  for (int k = 0; k < nn; ++k)
    for (int j = 0; j < nn; ++j)
      for (int i = 0; i < nn; ++i)
        if (i == 0 || j == 0 || k == 0 || i == nn - 1 || j == nn - 1 || k == nn - 1) {
          bidx.push_back((k * nn + j) * nn + i);
          bx.push_back(coord[i]);
          by.push_back(coord[j]);
          bz.push_back(coord[k]);
        }
  Vec bpot;
  boundary_potentials(scr, bx, by, bz, bpot);

  // interior 1-D pencil
  Mat ke, me;
  element_matrices(p, ke, me);
  Mat Ki(ni, ni), Mi(ni, ni);
  for (int e = 0; e < B; ++e)
    for (int a = 0; a <= p; ++a)
      for (int b = 0; b <= p; ++b) {
        const int ia = p * e + a - 1, ib = p * e + b - 1;
        if (ia < 0 || ib < 0 || ia >= ni || ib >= ni) continue;
        Ki(ia, ib) += ke(a, b);
        Mi(ia, ib) += me(a, b);
      }
  Vec lam;
  Mat V;
  sym_gen_eig(Ki, Mi, lam, V);
  const int g0 = p * (c - n_sr), nblk = S * p + 1;   // near-block nodes: global g0 .. g0 + nblk - 1

  Mat G = load_weights(p, scr);                     // (d + 1) x (sp p + 1)
  const int s0 = p * (c - (sp - 1) / 2);            // global node of the support's lower end
  T.assign(size_t(nb) * S * S * S * np1 * np1 * np1, 0.0);

  parallel_for(nb, [&](int ia) {
    const int ax = ia % nl, ay = (ia / nl) % nl, az = ia / (nl * nl);
    const size_t ni3 = size_t(ni) * ni * ni;
    Vec r(ni3, 0.0);
    // source: 4 pi G_a on the support's nodes (all interior)
    for (int kz = 0; kz <= sp * p; ++kz)
      for (int ky = 0; ky <= sp * p; ++ky)
        for (int kx = 0; kx <= sp * p; ++kx)
          r[(size_t(s0 + kz - 1) * ni + (s0 + ky - 1)) * ni + (s0 + kx - 1)] =
              4.0 * M_PI * G(az, kz) * G(ay, ky) * G(ax, kx);
    // boundary data on a full grid (zero inside), read per shell element
    Vec gb(size_t(nn) * nn * nn, 0.0);
    for (size_t b = 0; b < bidx.size(); ++b) gb[bidx[b]] = bpot[b * nb + ia];
    // r -= K_ib g: element stiffness (ke me me + me ke me + me me ke) on the
    // shell elements' boundary values, added to their interior nodes
    const int q1 = p + 1;
    Vec loc(size_t(q1) * q1 * q1), t1(loc.size()), t2(loc.size()), y(loc.size());
    for (int ez = 0; ez < B; ++ez)
      for (int ey = 0; ey < B; ++ey)
        for (int ex = 0; ex < B; ++ex) {
          if (ex > 0 && ey > 0 && ez > 0 && ex < B - 1 && ey < B - 1 && ez < B - 1) continue;
          for (int a = 0; a < q1; ++a)
            for (int b2 = 0; b2 < q1; ++b2)
              for (int c2 = 0; c2 < q1; ++c2)
                loc[(a * q1 + b2) * q1 + c2] = gb[(size_t(p * ez + a) * nn + (p * ey + b2)) * nn + (p * ex + c2)];
          std::fill(y.begin(), y.end(), 0.0);
          // three terms, each a product of 1-D element matrices along z, y, x
          for (int term = 0; term < 3; ++term) {
            const Mat &Az = term == 2 ? ke : me, &Ay = term == 1 ? ke : me, &Ax = term == 0 ? ke : me;
            for (int a = 0; a < q1; ++a)   // along x
              for (int b2 = 0; b2 < q1; ++b2)
                for (int c2 = 0; c2 < q1; ++c2) {
                  double s = 0.0;
                  for (int k = 0; k < q1; ++k) s += Ax(c2, k) * loc[(a * q1 + b2) * q1 + k];
                  t1[(a * q1 + b2) * q1 + c2] = s;
                }
            for (int a = 0; a < q1; ++a)   // along y
              for (int b2 = 0; b2 < q1; ++b2)
                for (int c2 = 0; c2 < q1; ++c2) {
                  double s = 0.0;
                  for (int k = 0; k < q1; ++k) s += Ay(b2, k) * t1[(a * q1 + k) * q1 + c2];
                  t2[(a * q1 + b2) * q1 + c2] = s;
                }
            for (int a = 0; a < q1; ++a)   // along z
              for (int b2 = 0; b2 < q1; ++b2)
                for (int c2 = 0; c2 < q1; ++c2) {
                  double s = 0.0;
                  for (int k = 0; k < q1; ++k) s += Az(a, k) * t2[(k * q1 + b2) * q1 + c2];
                  y[(a * q1 + b2) * q1 + c2] += s;
                }
          }
          for (int a = 0; a < q1; ++a)
            for (int b2 = 0; b2 < q1; ++b2)
              for (int c2 = 0; c2 < q1; ++c2) {
                const int gz = p * ez + a - 1, gy = p * ey + b2 - 1, gx = p * ex + c2 - 1;
                if (gz < 0 || gy < 0 || gx < 0 || gz >= ni || gy >= ni || gx >= ni) continue;
                r[(size_t(gz) * ni + gy) * ni + gx] -= y[(a * q1 + b2) * q1 + c2];
              }
        }
    // w = V^(3) diag(1 / (lam_i + lam_j + lam_k)) V^(3)T r, back-transformed
    // only on the near block's rows
    Vec u(ni3, 0.0), v(ni3, 0.0);
    for (int k = 0; k < ni; ++k)   // x: u[k][j][i'] = sum_i V(i, i') r[k][j][i]
      for (int j = 0; j < ni; ++j) {
        const double *rr = &r[(size_t(k) * ni + j) * ni];
        double *uu = &u[(size_t(k) * ni + j) * ni];
        for (int i = 0; i < ni; ++i) {
          const double ri = rr[i];
          if (ri == 0.0) continue;
          const double *vr = &V.a[size_t(i) * ni];
          for (int ip = 0; ip < ni; ++ip) uu[ip] += vr[ip] * ri;
        }
      }
    for (int k = 0; k < ni; ++k)   // y
      for (int j = 0; j < ni; ++j) {
        const double *uu = &u[(size_t(k) * ni + j) * ni];
        const double *vr = &V.a[size_t(j) * ni];
        for (int jp = 0; jp < ni; ++jp) {
          const double w = vr[jp];
          double *vv = &v[(size_t(k) * ni + jp) * ni];
          for (int i = 0; i < ni; ++i) vv[i] += w * uu[i];
        }
      }
    std::fill(u.begin(), u.end(), 0.0);
    for (int k = 0; k < ni; ++k) {   // z
      const double *vr = &V.a[size_t(k) * ni];
      const double *vv = &v[size_t(k) * ni * ni];
      for (int kp = 0; kp < ni; ++kp) {
        const double w = vr[kp];
        double *uu = &u[size_t(kp) * ni * ni];
        for (size_t t = 0; t < size_t(ni) * ni; ++t) uu[t] += w * vv[t];
      }
    }
    for (int k = 0; k < ni; ++k)
      for (int j = 0; j < ni; ++j)
        for (int i = 0; i < ni; ++i) u[(size_t(k) * ni + j) * ni + i] /= (lam[i] + lam[j] + lam[k]);
    // back along z, y, x onto the block rows (block node r is global g0 + r,
    // interior index g0 + r - 1)
    Vec bz_(size_t(nblk) * ni * ni, 0.0);
    for (int rz = 0; rz < nblk; ++rz) {
      const double *vr = &V.a[size_t(g0 + rz - 1) * ni];
      double *o = &bz_[size_t(rz) * ni * ni];
      for (int kp = 0; kp < ni; ++kp) {
        const double w = vr[kp];
        const double *uu = &u[size_t(kp) * ni * ni];
        for (size_t t = 0; t < size_t(ni) * ni; ++t) o[t] += w * uu[t];
      }
    }
    Vec byy(size_t(nblk) * nblk * ni, 0.0);
    for (int rz = 0; rz < nblk; ++rz)
      for (int ry = 0; ry < nblk; ++ry) {
        const double *vr = &V.a[size_t(g0 + ry - 1) * ni];
        double *o = &byy[(size_t(rz) * nblk + ry) * ni];
        for (int jp = 0; jp < ni; ++jp) {
          const double w = vr[jp];
          const double *src = &bz_[(size_t(rz) * ni + jp) * ni];
          for (int i = 0; i < ni; ++i) o[i] += w * src[i];
        }
      }
    for (int Dz = 0; Dz < S; ++Dz)
      for (int Dy = 0; Dy < S; ++Dy)
        for (int Dx = 0; Dx < S; ++Dx) {
          const size_t iD = (size_t(Dz) * S + Dy) * S + Dx;
          for (int mz = 0; mz <= p; ++mz)
            for (int my = 0; my <= p; ++my)
              for (int mx = 0; mx <= p; ++mx) {
                const double *src = &byy[(size_t(p * Dz + mz) * nblk + (p * Dy + my)) * ni];
                const double *vr = &V.a[size_t(g0 + p * Dx + mx - 1) * ni];
                double s = 0.0;
                for (int ip = 0; ip < ni; ++ip) s += vr[ip] * src[ip];
                T[(size_t(ia) * S * S * S + iD) * np1 * np1 * np1 + (size_t(mz) * np1 + my) * np1 + mx] = s;
              }
        }
  });
}

}  // namespace fep3m
