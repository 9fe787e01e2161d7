// The boxes of Section 2.6.  Grounded (eq. bcadjust with g = 0): the mesh
// potential of the box [0, n]^3 (element units) takes on the boundary the
// values -Phi_sr, the short-range potential of the charges of the near
// block; its interior solves K_II phi_I = b_I - K_IB phi_B.  Mesh vectors of
// the box are nb consecutive (p n + 1)^3 blocks [z][y][x], global node
// g = p e + k along each axis, no wrap.
//
//   boundary values   one thread per (configuration, face node): the node's
//                     element e = min(g / p, n - 1) per axis, its local node
//                     m; Phi_sr = sum over the charges of e's near block (cut
//                     at the faces) of Q_j / |x_B - x_j| minus the block's
//                     screen potential Psi_e[m] (read as W = -Psi from the
//                     near-field kernel run without phi)
//   interior          gather of the interior nodes into a contiguous
//                     (p n - 1)^3 block and the scatter back
//   element field     W_E[m] += phi at node (p e + k) of the box
//   residual          block partials of sum_I (b - K phi)^2 and sum_I b^2
//                     over the interior nodes
//   operator          y = K v on every node by three banded 1-D passes
//                     (class-row band tables in LDS)
//   reverse pass      box assembly of the deposit, the boundary terms of the
//                     moment adjoint (mu = G - K lambda in the deposit's
//                     boundary slots) and of the per-charge gradients (one
//                     wave per charge)
//   insulating box    (zero normal field) the surface load of -dPhi_sr/dn by
//                     a Gauss rule per boundary element face, the
//                     compatibility projection, and the reverse pass's face
//                     weights and per-charge face terms
#include <algorithm>

#include "kernels.hpp"

namespace fep3m {
namespace {

__device__ __forceinline__ int node_elem(int g, int PO, int n) { return min(g / PO, n - 1); }

template <int PO>
__global__ __launch_bounds__(256) void k_box_bvals(int n, int nsr, int nb, int64_t N, BoxNodes nodes,
                                                   const int *__restrict__ start, const double *__restrict__ sg,
                                                   const double *__restrict__ sQ, const double *__restrict__ Wneg,
                                                   double *__restrict__ phiB) {
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1;
  const int P = PO * n + 1;
  const size_t P2 = size_t(P) * P, per = P2 * P, M = size_t(n) * n * n;
  const size_t total = size_t(nb) * 6 * P2;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += size_t(gridDim.x) * blockDim.x) {
    const int cfg = int(t / (6 * P2));
    const size_t r = t % (6 * P2);
    const int face = int(r / P2), a = int((r % P2) % P), b = int((r % P2) / P);
    const int ax = face >> 1, side = face & 1;
    int g[3];
    g[ax] = side ? P - 1 : 0;
    g[ax == 0 ? 1 : 0] = a;
    g[ax == 2 ? 1 : 2] = b;
    int e[3], k[3];
    double xb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      e[c] = node_elem(g[c], PO, n);
      k[c] = g[c] - PO * e[c];
      xb[c] = e[c] + 0.5 + nodes.x[k[c]];
    }
    const size_t cbase = size_t(cfg) * M;
    double pairs = 0.0;
    for (int dz = -nsr; dz <= nsr; ++dz) {
      const int sz = e[2] + dz;
      if (sz < 0 || sz >= n) continue;
      for (int dy = -nsr; dy <= nsr; ++dy) {
        const int sy = e[1] + dy;
        if (sy < 0 || sy >= n) continue;
        const int sx0 = max(e[0] - nsr, 0), sx1 = min(e[0] + nsr, n - 1);
        const size_t row = cbase + size_t(n) * (sy + size_t(n) * sz);
        // the elements sx0 .. sx1 of one row are consecutive in the sorted order
        for (int s = start[row + sx0]; s < start[row + sx1 + 1]; ++s) {
          const double dx = sg[s] - xb[0], dyv = sg[N + s] - xb[1], dzv = sg[2 * N + s] - xb[2];
          pairs += sQ[s] / sqrt(dx * dx + dyv * dyv + dzv * dzv);
        }
      }
    }
    const size_t E = cbase + e[0] + size_t(n) * (e[1] + size_t(n) * e[2]);
    const int m = k[0] + Q1 * (k[1] + Q1 * k[2]);
    // Phi_sr = pairs - Psi = pairs + Wneg; the mesh takes -Phi_sr
    phiB[size_t(cfg) * per + (size_t(g[2]) * P + g[1]) * P + g[0]] = -(pairs + Wneg[E * NM + m]);
  }
}

// dst[interior block] = src[box] (to_interior) or the reverse on the
// interior nodes only (the boundary nodes of dst keep their values).
__global__ __launch_bounds__(256) void k_box_interior(int P, int nb, bool to_interior, const double *__restrict__ src,
                                                      double *__restrict__ dst) {
  const int Pi = P - 2;
  const size_t per = size_t(P) * P * P, peri = size_t(Pi) * Pi * Pi, total = peri * nb;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += size_t(gridDim.x) * blockDim.x) {
    const int cfg = int(t / peri);
    const size_t l = t % peri;
    const int i = int(l % Pi), j = int((l / Pi) % Pi), k = int(l / (size_t(Pi) * Pi));
    const size_t gb = size_t(cfg) * per + (size_t(k + 1) * P + (j + 1)) * P + (i + 1);
    if (to_interior) dst[t] = src[gb];
    else dst[gb] = src[t];
  }
}

// y = c y + a x (c = 0: y is not read)
__global__ __launch_bounds__(256) void k_box_axpby(size_t total, double a, const double *__restrict__ x, double c,
                                                   double *__restrict__ y) {
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += size_t(gridDim.x) * blockDim.x)
    y[t] = (c == 0.0 ? 0.0 : c * y[t]) + a * x[t];
}

__global__ __launch_bounds__(256) void k_box_fill(size_t total, double v, double *__restrict__ y) {
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += size_t(gridDim.x) * blockDim.x)
    y[t] = v;
}

template <int PO>
__global__ __launch_bounds__(256) void k_box_addphi(int n, int nb, const double *__restrict__ phi,
                                                    double *__restrict__ W) {
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1;
  const int P = PO * n + 1;
  const size_t M = size_t(n) * n * n, per = size_t(P) * P * P, total = size_t(nb) * M * NM;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += size_t(gridDim.x) * blockDim.x) {
    const size_t E = t / NM;
    const int m = int(t % NM);
    const int cfg = int(E / M);
    const size_t El = E % M;
    const int ex = int(El % n), ey = int((El / n) % n), ez = int(El / (size_t(n) * n));
    const int mx = m % Q1, my = (m / Q1) % Q1, mz = m / (Q1 * Q1);
    W[t] += phi[size_t(cfg) * per + (size_t(PO * ez + mz) * P + (PO * ey + my)) * P + (PO * ex + mx)];
  }
}

// K blocks per configuration; partial[cfg K + kb] = sum (b - y)^2 and
// partial[nb K + cfg K + kb] = sum b (plain = 1) or sum b^2 over this
// block's nodes: the interior ones (off = 1) or all (off = 0).  A null y
// reads as zero.
__global__ __launch_bounds__(256) void k_box_resid(int P, int off, int plain, int K, int nb,
                                                   const double *__restrict__ ball, const double *__restrict__ yall,
                                                   double *__restrict__ partial) {
  __shared__ double red[2][4];
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const int Pi = P - 2 * off;
  const size_t per = size_t(P) * P * P, peri = size_t(Pi) * Pi * Pi;
  double sr = 0.0, sb = 0.0;
  for (size_t l = size_t(kb) * blockDim.x + threadIdx.x; l < peri; l += size_t(K) * blockDim.x) {
    const int i = int(l % Pi), j = int((l / Pi) % Pi), k = int(l / (size_t(Pi) * Pi));
    const size_t g = size_t(cfg) * per + (size_t(k + off) * P + (j + off)) * P + (i + off);
    const double bv = ball[g], rv = bv - (yall ? yall[g] : 0.0);
    sr += rv * rv;
    sb += plain ? bv : bv * bv;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sr += __shfl_down(sr, o, 64);
    sb += __shfl_down(sb, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = sr;
    red[1][w] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int i = 0; i < 4; ++i) {
      a += red[0][i];
      c += red[1][i];
    }
    partial[blockIdx.x] = a;
    partial[size_t(nb) * K + blockIdx.x] = c;
  }
}

// The boundary nodes B whose element e(B) lies within nsr elements of Ec
// along every axis, each visited once (x faces whole, y faces without the
// x edges, z faces without the x and y edges): f(g, e, k) per node.
template <int PO, class Fn>
__device__ __forceinline__ void for_near_boundary(const int (&Ec)[3], int n, int nsr, Fn f) {
  const int P = PO * n + 1;
  int lo[3], hi[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int el = max(Ec[c] - nsr, 0), eh = min(Ec[c] + nsr, n - 1);
    lo[c] = PO * el;
    hi[c] = eh == n - 1 ? P - 1 : PO * eh + PO - 1;
  }
  for (int face = 0; face < 6; ++face) {
    const int ax = face >> 1, side = face & 1;
    if (side == 0 ? Ec[ax] > nsr : (n - 1 - Ec[ax]) > nsr) continue;
    int g[3], a0[3], a1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a0[c] = lo[c];
      a1[c] = hi[c];
      if (c < ax) {   // nodes on the faces of a lower axis were visited there
        a0[c] = max(a0[c], 1);
        a1[c] = min(a1[c], P - 2);
      }
    }
    a0[ax] = a1[ax] = side ? P - 1 : 0;
    for (g[2] = a0[2]; g[2] <= a1[2]; ++g[2])
      for (g[1] = a0[1]; g[1] <= a1[1]; ++g[1])
        for (g[0] = a0[0]; g[0] <= a1[0]; ++g[0]) {
          int e[3], k[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            e[c] = node_elem(g[c], PO, n);
            k[c] = g[c] - PO * e[c];
          }
          f(g, e, k);
        }
  }
}

// Box assembly of element-local nodal values: G[node] = sum over the
// elements holding the node of gE[E][m] (gather form, no wrap).
template <int PO>
__global__ __launch_bounds__(256) void k_box_assemble(int n, int nb, const double *__restrict__ gE,
                                                      double *__restrict__ G) {
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1;
  const int P = PO * n + 1;
  const size_t per = size_t(P) * P * P, M = size_t(n) * n * n;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < per * nb; t += size_t(gridDim.x) * blockDim.x) {
    const int cfg = int(t / per);
    const size_t l = t % per;
    const int g[3] = {int(l % P), int((l / P) % P), int(l / (size_t(P) * P))};
    int es[3][2], ks[3][2], cnt[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int e = g[c] / PO, k = g[c] - PO * e;
      cnt[c] = 0;
      if (k == 0 && e > 0) { es[c][cnt[c]] = e - 1; ks[c][cnt[c]] = PO; ++cnt[c]; }
      if (e < n) { es[c][cnt[c]] = e; ks[c][cnt[c]] = k; ++cnt[c]; }
    }
    double v = 0.0;
    for (int iz = 0; iz < cnt[2]; ++iz)
      for (int iy = 0; iy < cnt[1]; ++iy)
        for (int ix = 0; ix < cnt[0]; ++ix) {
          const size_t E = size_t(cfg) * M + es[0][ix] + size_t(n) * (es[1][iy] + size_t(n) * es[2][iz]);
          v += gE[E * NM + ks[0][ix] + Q1 * (ks[1][iy] + Q1 * ks[2][iz])];
        }
    G[t] = v;
  }
}

// The boundary part of the moment adjoint, sum_B mu_B T[a][e(B) - E][m_B],
// is the transposed near-field sum of mu placed at each boundary node's
// canonical slot (e(B), m_B): so g[e(B)][m_B] -= mu_B turns the near part
// of the adjoint, -sum_D <g_{E+D}, T_a[D]>, into the sum of both.  One
// thread per boundary node, each node once (x faces whole, y faces without
// the x edges, z faces without the x and y edges); the slots are distinct.
template <int PO>
__global__ __launch_bounds__(256) void k_box_mu_slots(int n, int nb, const double *__restrict__ mu,
                                                      double *__restrict__ gE) {
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1;
  const int P = PO * n + 1;
  const size_t P2 = size_t(P) * P, per = P2 * P, M = size_t(n) * n * n;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < size_t(nb) * 6 * P2;
       t += size_t(gridDim.x) * blockDim.x) {
    const int cfg = int(t / (6 * P2));
    const size_t r = t % (6 * P2);
    const int face = int(r / P2), a = int((r % P2) % P), b = int((r % P2) / P);
    const int ax = face >> 1, side = face & 1;
    int g[3];
    g[ax] = side ? P - 1 : 0;
    g[ax == 0 ? 1 : 0] = a;
    g[ax == 2 ? 1 : 2] = b;
    bool dup = false;
    for (int c = 0; c < ax; ++c) dup = dup || g[c] == 0 || g[c] == P - 1;
    if (dup) continue;
    int e[3], k[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      e[c] = node_elem(g[c], PO, n);
      k[c] = g[c] - PO * e[c];
    }
    const size_t E = size_t(cfg) * M + e[0] + size_t(n) * (e[1] + size_t(n) * e[2]);
    gE[E * NM + k[0] + Q1 * (k[1] + Q1 * k[2])] -= mu[size_t(cfg) * per + (size_t(g[2]) * P + g[1]) * P + g[0]];
  }
}

// Sum of four values over the 64 lanes of a wave (every lane gets the sum).
__device__ __forceinline__ void wave_sum4(double &a, double &b, double &c, double &d) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c += __shfl_xor(c, o, 64);
    d += __shfl_xor(d, o, 64);
  }
}

// True for an element within nsr elements of no face (no boundary term).
__device__ __forceinline__ bool far_from_faces(const int (&Ec)[3], int n, int nsr) {
  return Ec[0] > nsr && Ec[1] > nsr && Ec[2] > nsr && n - 1 - Ec[0] > nsr && n - 1 - Ec[1] > nsr &&
         n - 1 - Ec[2] > nsr;
}

// Boundary part of the per-charge gradients: for a sorted charge s near a
// face, bp = sum_B mu_B (x_B - x_s) / r^3 and bq = sum_B mu_B / r over the
// boundary nodes whose element's near block holds it (each visited once, as
// in for_near_boundary); F += s2 Q bp / 2 and dU/dQ -= inv_h bq / 2 (physical
// units), in caller order.  One wave per charge: the lanes split the nodes
// of each face's range and the wave sums them.
template <int PO>
__global__ __launch_bounds__(256) void k_box_charge_bnd(int n, int nsr, int nb, int64_t N, const int *__restrict__ off,
                                                        double inv_h, BoxNodes nodes, const double *__restrict__ sg,
                                                        const double *__restrict__ sQ, const double *__restrict__ mu,
                                                        const int *__restrict__ perm, double *__restrict__ F,
                                                        double *__restrict__ dUdQ) {
  const int P = PO * n + 1;
  const size_t per = size_t(P) * P * P;
  const int lane = threadIdx.x & 63;
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
  for (int64_t s = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); s < N; s += waves) {
    const double xs[3] = {sg[s], sg[N + s], sg[2 * N + s]};
    int Ec[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) Ec[c] = min(int(floor(xs[c])), n - 1);
    if (far_from_faces(Ec, n, nsr)) continue;
    const double *muc = mu + size_t(cfg_of(off, nb, s)) * per;
    int lo[3], hi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int el = max(Ec[c] - nsr, 0), eh = min(Ec[c] + nsr, n - 1);
      lo[c] = PO * el;
      hi[c] = eh == n - 1 ? P - 1 : PO * eh + PO - 1;
    }
    double bx = 0.0, by = 0.0, bz = 0.0, bq = 0.0;
    for (int face = 0; face < 6; ++face) {
      const int ax = face >> 1, side = face & 1;
      if (side == 0 ? Ec[ax] > nsr : (n - 1 - Ec[ax]) > nsr) continue;
      int a0[3], len[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        int u0 = lo[c], u1 = hi[c];
        if (c < ax) {   // nodes on the faces of a lower axis were visited there
          u0 = max(u0, 1);
          u1 = min(u1, P - 2);
        }
        if (c == ax) u0 = u1 = side ? P - 1 : 0;
        a0[c] = u0;
        len[c] = u1 - u0 + 1;
      }
      const int count = len[0] * len[1] * len[2];
      for (int idx = lane; idx < count; idx += 64) {
        const int g[3] = {a0[0] + idx % len[0], a0[1] + (idx / len[0]) % len[1], a0[2] + idx / (len[0] * len[1])};
        double d[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int e = node_elem(g[c], PO, n);
          d[c] = e + 0.5 + nodes.x[g[c] - PO * e] - xs[c];
        }
        const double mv = muc[(size_t(g[2]) * P + g[1]) * P + g[0]];
        const double ri = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double w = mv * ri * ri * ri;
        bx += w * d[0];
        by += w * d[1];
        bz += w * d[2];
        bq += mv * ri;
      }
    }
    wave_sum4(bx, by, bz, bq);
    if (lane == 0) {
      const int i = perm[s];
      const double q = sQ[s], c = 0.5 * inv_h * inv_h * q;
      if (F) {
        F[3 * size_t(i) + 0] += c * bx;
        F[3 * size_t(i) + 1] += c * by;
        F[3 * size_t(i) + 2] += c * bz;
      }
      if (dUdQ) dUdQ[i] -= 0.5 * inv_h * bq;
    }
  }
}

// Surface load of the insulating box, per boundary element face (one block
// each): at the NQ x NQ Gauss points of the face, the outward normal
// derivative of Phi_sr (near pairs of the face's element, cut at the
// faces, minus the element's screen field Psi = -Wneg, differentiated from
// its nodal values); then the face's (PO + 1)^2 nodal contributions
// -sum_q w_q dPhi_sr/dn(x_q) u_m(x_q) into tF[cfg][face][kb][kc] (kb along
// the higher tangential axis, kc along the lower).  Faces: f = a 2 n^2 +
// s n^2 + j n + i (axis a, side s, tangential element indices i lower, j
// higher).
template <int PO>
__global__ __launch_bounds__(128) void k_box_flux(int n, int nsr, int64_t N, BoxQuad qd, const int *__restrict__ start,
                                                  const double *__restrict__ sg, const double *__restrict__ sQ,
                                                  const double *__restrict__ Wneg, double *__restrict__ tF) {
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1, NQ = kBoxNQ;
  __shared__ double fl[NQ * NQ];
  const int nf = 6 * n * n;
  const int cfg = blockIdx.x / nf, f = blockIdx.x % nf;
  const int a = f / (2 * n * n), side = (f / (n * n)) % 2, i = f % n, j = (f / n) % n;
  const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
  int e[3];
  e[a] = side ? n - 1 : 0;
  e[t0] = i;
  e[t1] = j;
  const size_t M = size_t(n) * n * n;
  const size_t cbase = size_t(cfg) * M;
  const size_t E = cbase + e[0] + size_t(n) * (e[1] + size_t(n) * e[2]);
  const double sgn = side ? 1.0 : -1.0;
  const int q = threadIdx.x;
  if (q < NQ * NQ) {
    const int qi = q / NQ, qj = q % NQ;   // qi along t1, qj along t0
    double X[3];
    X[a] = side ? double(n) : 0.0;
    X[t0] = e[t0] + 0.5 + qd.xq[qj];
    X[t1] = e[t1] + 0.5 + qd.xq[qi];
    double dn = 0.0;   // n . grad of sum_j Q_j / |x - y_j|
    for (int dz = -nsr; dz <= nsr; ++dz) {
      const int sz = e[2] + dz;
      if (sz < 0 || sz >= n) continue;
      for (int dy = -nsr; dy <= nsr; ++dy) {
        const int sy = e[1] + dy;
        if (sy < 0 || sy >= n) continue;
        const int sx0 = max(e[0] - nsr, 0), sx1 = min(e[0] + nsr, n - 1);
        const size_t row = cbase + size_t(n) * (sy + size_t(n) * sz);
        for (int s = start[row + sx0]; s < start[row + sx1 + 1]; ++s) {
          const double d0 = X[0] - sg[s], d1 = X[1] - sg[N + s], d2 = X[2] - sg[2 * N + s];
          const double ri = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
          const double da = a == 0 ? d0 : (a == 1 ? d1 : d2);
          dn -= sQ[s] * da * ri * ri * ri;
        }
      }
    }
    dn *= sgn;
    // n . grad Psi = -n . grad Wneg from the element's nodal values
    const double *w = Wneg + E * NM;
    double dpsi = 0.0;
    for (int m = 0; m < NM; ++m) {
      const int k[3] = {m % Q1, (m / Q1) % Q1, m / (Q1 * Q1)};
      dpsi -= w[m] * qd.dend[side][k[a]] * qd.lq[qi][k[t1]] * qd.lq[qj][k[t0]];
    }
    dpsi *= sgn;
    fl[q] = (dn - dpsi) * qd.wq[qi] * qd.wq[qj];
  }
  __syncthreads();
  if (q < Q1 * Q1) {
    const int kb = q / Q1, kc = q % Q1;
    double v = 0.0;
    for (int qi = 0; qi < NQ; ++qi)
      for (int qj = 0; qj < NQ; ++qj) v += fl[qi * NQ + qj] * qd.lq[qi][kb] * qd.lq[qj][kc];
    tF[(size_t(blockIdx.x) * Q1 + kb) * Q1 + kc] = -v;
  }
}

// Reverse pass of the insulating box, per boundary face (one block each):
// Lw[q] = w_q lambda(x_q) at the face's Gauss points (lambda interpolated
// from the face's nodes) and hF[m] = sum_q Lw[q] dn u_m(x_q) over the
// element's nodes m (x fastest), the face's weight on the moment adjoint.
template <int PO>
__global__ __launch_bounds__(128) void k_box_flux_adj(int n, BoxQuad qd, const double *__restrict__ lam,
                                                      double *__restrict__ Lw, double *__restrict__ hF) {
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1, NQ = kBoxNQ;
  __shared__ double lw[NQ * NQ];
  const int P = PO * n + 1;
  const int nf = 6 * n * n;
  const int cfg = blockIdx.x / nf, f = blockIdx.x % nf;
  const int a = f / (2 * n * n), side = (f / (n * n)) % 2, i = f % n, j = (f / n) % n;
  const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
  const double *lc = lam + size_t(cfg) * P * P * P;
  const double sgn = side ? 1.0 : -1.0;
  const int q = threadIdx.x;
  if (q < NQ * NQ) {
    const int qi = q / NQ, qj = q % NQ;
    int g[3];
    g[a] = side ? P - 1 : 0;
    double v = 0.0;
    for (int kb = 0; kb < Q1; ++kb) {
      g[t1] = PO * j + kb;
      double r = 0.0;
      for (int kc = 0; kc < Q1; ++kc) {
        g[t0] = PO * i + kc;
        r += lc[(size_t(g[2]) * P + g[1]) * P + g[0]] * qd.lq[qj][kc];
      }
      v += r * qd.lq[qi][kb];
    }
    v *= qd.wq[qi] * qd.wq[qj];
    lw[q] = v;
    Lw[size_t(blockIdx.x) * NQ * NQ + q] = v;
  }
  __syncthreads();
  for (int m = threadIdx.x; m < NM; m += blockDim.x) {
    const int k[3] = {m % Q1, (m / Q1) % Q1, m / (Q1 * Q1)};
    double v = 0.0;
    for (int qi = 0; qi < NQ; ++qi) {
      double r = 0.0;
      for (int qj = 0; qj < NQ; ++qj) r += lw[qi * NQ + qj] * qd.lq[qj][k[t0]];
      v += r * qd.lq[qi][k[t1]];
    }
    hF[size_t(blockIdx.x) * NM + m] = sgn * qd.dend[side][k[a]] * v;
  }
}

// gE[E][m] -= sum of hF over E's boundary faces (axes in order), so that the
// near part of the moment adjoint carries the surface load's table term.
template <int PO>
__global__ __launch_bounds__(256) void k_box_h_slots(int n, int nb, const double *__restrict__ hF,
                                                     double *__restrict__ gE) {
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1;
  const size_t M = size_t(n) * n * n, nf = size_t(6) * n * n;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < size_t(nb) * M * NM;
       t += size_t(gridDim.x) * blockDim.x) {
    const size_t E = t / NM;
    const int m = int(t % NM), cfg = int(E / M);
    const size_t El = E % M;
    const int e[3] = {int(El % n), int((El / n) % n), int(El / (size_t(n) * n))};
    double v = 0.0;
    for (int a = 0; a < 3; ++a) {
      const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
      for (int side = 0; side < 2; ++side) {
        if (e[a] != (side ? n - 1 : 0)) continue;
        const size_t face = size_t(a) * 2 * n * n + size_t(side) * n * n + size_t(e[t1]) * n + e[t0];
        v += hF[(size_t(cfg) * nf + face) * NM + m];
      }
    }
    if (v != 0.0) gE[t] -= v;
  }
}

// Per-charge face terms of the insulating box's gradients: for a sorted
// charge whose element lies in the near block of a boundary face's element,
// sum over the face's Gauss points of Lw (-n / r^3 + 3 (n.d) d / r^5) and of
// Lw (n.d) / r^3 (d = x_q - x_s); F -= Q s2 / 2 times the first, dU/dQ +=
// inv_h / 2 times the second (physical units, caller order).  One wave per
// charge: the lanes split the (face element, Gauss point) pairs of each
// near face and the wave sums them.
template <int PO>
__global__ __launch_bounds__(256) void k_box_flux_charge(int n, int nsr, int nb, int64_t N,
                                                         const int *__restrict__ off, double inv_h, BoxQuad qd,
                                                         const double *__restrict__ sg, const double *__restrict__ sQ,
                                                         const double *__restrict__ Lw, const int *__restrict__ perm,
                                                         double *__restrict__ F, double *__restrict__ dUdQ) {
  constexpr int NQ = kBoxNQ, NQ2 = NQ * NQ;
  const size_t nf = size_t(6) * n * n;
  const int lane = threadIdx.x & 63;
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
  for (int64_t s = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); s < N; s += waves) {
    const double xs[3] = {sg[s], sg[N + s], sg[2 * N + s]};
    int Ec[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) Ec[c] = min(int(floor(xs[c])), n - 1);
    if (far_from_faces(Ec, n, nsr)) continue;
    const int cfg = cfg_of(off, nb, s);
    double gx = 0.0, gy = 0.0, gz = 0.0, dq = 0.0;
    for (int a = 0; a < 3; ++a) {
      const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
      for (int side = 0; side < 2; ++side) {
        if (side == 0 ? Ec[a] > nsr : (n - 1 - Ec[a]) > nsr) continue;
        const double sgn = side ? 1.0 : -1.0;
        const double da = (side ? double(n) : 0.0) - xs[a];   // normal offset, the same at every point
        const int i0 = max(Ec[t0] - nsr, 0), i1 = min(Ec[t0] + nsr, n - 1);
        const int j0 = max(Ec[t1] - nsr, 0), j1 = min(Ec[t1] + nsr, n - 1);
        const int ni = i1 - i0 + 1, count = ni * (j1 - j0 + 1) * NQ2;
        const double *lwp = Lw + (size_t(cfg) * nf + size_t(a) * 2 * n * n + size_t(side) * n * n) * NQ2;
        for (int idx = lane; idx < count; idx += 64) {
          const int q = idx % NQ2, el = idx / NQ2;
          const int i = i0 + el % ni, j = j0 + el / ni;
          const int qi = q / NQ, qj = q % NQ;
          double d[3];
          d[a] = da;
          d[t0] = i + 0.5 + qd.xq[qj] - xs[t0];
          d[t1] = j + 0.5 + qd.xq[qi] - xs[t1];
          const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          const double ri = 1.0 / sqrt(r2), ri3 = ri * ri * ri;
          const double w = lwp[(size_t(j) * n + i) * NQ2 + q];
          const double nd = sgn * da;
          const double c5 = 3.0 * nd * ri3 * ri * ri;
          gx += w * (c5 * d[0] - (a == 0 ? sgn : 0.0) * ri3);
          gy += w * (c5 * d[1] - (a == 1 ? sgn : 0.0) * ri3);
          gz += w * (c5 * d[2] - (a == 2 ? sgn : 0.0) * ri3);
          dq += w * nd * ri3;
        }
      }
    }
    wave_sum4(gx, gy, gz, dq);
    if (lane == 0) {
      const int idx = perm[s];
      const double qv = sQ[s], c = 0.5 * inv_h * inv_h * qv;
      if (F) {
        F[3 * size_t(idx) + 0] -= c * gx;
        F[3 * size_t(idx) + 1] -= c * gy;
        F[3 * size_t(idx) + 2] -= c * gz;
      }
      if (dUdQ) dUdQ[idx] += 0.5 * inv_h * dq;
    }
  }
}

// f[node] += the contributions of the boundary faces holding the node (in
// a fixed order: planes by axis and side, then faces by element).
template <int PO>
__global__ __launch_bounds__(256) void k_box_flux_add(int n, int nb, const double *__restrict__ tF,
                                                      double *__restrict__ f) {
  constexpr int Q1 = PO + 1;
  const int P = PO * n + 1;
  const size_t per = size_t(P) * P * P, nf = size_t(6) * n * n;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < per * nb; t += size_t(gridDim.x) * blockDim.x) {
    const int cfg = int(t / per);
    const size_t l = t % per;
    const int g[3] = {int(l % P), int((l / P) % P), int(l / (size_t(P) * P))};
    if (g[0] != 0 && g[0] != P - 1 && g[1] != 0 && g[1] != P - 1 && g[2] != 0 && g[2] != P - 1) continue;
    double v = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int side = 0; side < 2; ++side) {
        if (g[a] != (side ? P - 1 : 0)) continue;
        const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
        int e0[2], k0[2], c0 = 0, e1[2], k1[2], c1 = 0;
        {
          const int ee = g[t0] / PO, kk = g[t0] - PO * ee;
          if (kk == 0 && ee > 0) { e0[c0] = ee - 1; k0[c0] = PO; ++c0; }
          if (ee < n) { e0[c0] = ee; k0[c0] = kk; ++c0; }
        }
        {
          const int ee = g[t1] / PO, kk = g[t1] - PO * ee;
          if (kk == 0 && ee > 0) { e1[c1] = ee - 1; k1[c1] = PO; ++c1; }
          if (ee < n) { e1[c1] = ee; k1[c1] = kk; ++c1; }
        }
        for (int u1 = 0; u1 < c1; ++u1)
          for (int u0 = 0; u0 < c0; ++u0) {
            const size_t face = size_t(a) * 2 * n * n + size_t(side) * n * n + size_t(e1[u1]) * n + e0[u0];
            v += tF[((size_t(cfg) * nf + face) * Q1 + k1[u1]) * Q1 + k0[u0]];
          }
      }
    f[t] += v;
  }
}

// f -= (s_cfg / V) w1 (x) w1 (x) w1 on every node (the compatibility
// projection: s the sum of f, V = n^3, w1 the row sums of the 1-D mass).
__global__ __launch_bounds__(256) void k_box_sub_mass(int P, int nb, double invV, const double *__restrict__ w1,
                                                      const double *__restrict__ sums, double *__restrict__ f) {
  const size_t per = size_t(P) * P * P;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < per * nb; t += size_t(gridDim.x) * blockDim.x) {
    const int cfg = int(t / per);
    const size_t l = t % per;
    const int i = int(l % P), j = int((l / P) % P), k = int(l / (size_t(P) * P));
    f[t] -= sums[cfg] * invV * w1[i] * w1[j] * w1[k];
  }
}

// Passes of the box operator K = Kx My Mz + Mx Ky Mz + Mx My Kz along one
// axis of nb P^3 blocks.  The 1-D element-assembled matrices are banded (node
// o couples to nodes o - HB .. o + HB, HB = p) and, on the uniform mesh, row o
// depends only on its class: o mod p inside, p for o = 0, p + 1 for
// o = P - 1.  They come as compact tables of p + 2 class rows,
// row[c (2 HB + 1) + d] = A(o, o - HB + d), staged in LDS.
template <int HB>
__device__ __forceinline__ int band_class(int o, int P) {
  return o == 0 ? HB : (o == P - 1 ? HB + 1 : o % HB);
}

// Along y (axis 1) or z (axis 2): out0 = A in0 (+ B in1 when in1 is given),
// out1 = C in0 when out1 is given.  A thread owns R consecutive outputs of
// one line with the R + 2 HB inputs they need in registers; the lanes run
// over x, so every load and store of a wave covers consecutive x.
template <int HB, int R>
__global__ __launch_bounds__(256) void k_box_band(int P, int axis, int nb, const double *__restrict__ Ac,
                                                  const double *__restrict__ Bc, const double *__restrict__ Cc,
                                                  const double *__restrict__ in0, const double *__restrict__ in1,
                                                  double *__restrict__ out0, double *__restrict__ out1) {
  constexpr int W = 2 * HB + 1, NV = R + 2 * HB, NC = HB + 2;
  __shared__ double tab[3][NC * W];
  for (int i = threadIdx.x; i < NC * W; i += blockDim.x) {
    tab[0][i] = Ac[i];
    tab[1][i] = Bc[i];
    tab[2][i] = Cc[i];
  }
  __syncthreads();
  const size_t P2 = size_t(P) * P, per = P2 * P;
  const int nrun = (P + R - 1) / R;
  const size_t total = size_t(nb) * P2 * nrun;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += size_t(gridDim.x) * blockDim.x) {
    size_t base, stride;
    int o0;
    if (axis == 1) {            // t = ((sys, z), run, x)
      const int x = int(t % P);
      const size_t r = t / P;
      o0 = int(r % nrun) * R;
      const size_t sz = r / nrun;   // sys * P + z
      base = (sz / P) * per + (sz % P) * P2 + x;
      stride = P;
    } else {                    // t = (sys, run, y, x)
      const size_t xy = t % P2, r = t / P2;
      o0 = int(r % nrun) * R;
      base = (r / nrun) * per + xy;
      stride = P2;
    }
    double v0[NV], v1[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int k = o0 - HB + j;
      const bool ok = k >= 0 && k < P;
      v0[j] = ok ? in0[base + size_t(k) * stride] : 0.0;
      v1[j] = (ok && in1) ? in1[base + size_t(k) * stride] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int o = o0 + r;
      if (o >= P) break;
      const int c = band_class<HB>(o, P) * W;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int d = 0; d < W; ++d) s0 += tab[0][c + d] * v0[r + d];
      if (in1) {
#pragma unroll
        for (int d = 0; d < W; ++d) s0 += tab[1][c + d] * v1[r + d];
      }
      out0[base + size_t(o) * stride] = s0;
      if (out1) {
#pragma unroll
        for (int d = 0; d < W; ++d) s1 += tab[2][c + d] * v0[r + d];
        out1[base + size_t(o) * stride] = s1;
      }
    }
  }
}

// Along x: out = A in0 + B in1.  A block stages LPB whole x-lines of both
// inputs in LDS (zero padded by HB on each side) and writes the lines'
// outputs, one per thread, coalesced.
constexpr int kBandLines = 4;

template <int HB>
__global__ __launch_bounds__(256) void k_box_band_x(int P, size_t lines, const double *__restrict__ Ac,
                                                    const double *__restrict__ Bc, const double *__restrict__ in0,
                                                    const double *__restrict__ in1, double *__restrict__ out) {
  constexpr int W = 2 * HB + 1, NC = HB + 2, LPB = kBandLines;
  extern __shared__ double sh[];
  const int L = P + 2 * HB;
  double *s0 = sh, *s1 = sh + LPB * L, *ta = s1 + LPB * L, *tb = ta + NC * W;
  for (int i = threadIdx.x; i < NC * W; i += blockDim.x) {
    ta[i] = Ac[i];
    tb[i] = Bc[i];
  }
  for (size_t lb = size_t(blockIdx.x) * LPB; lb < lines; lb += size_t(gridDim.x) * LPB) {
    __syncthreads();
    for (int i = threadIdx.x; i < LPB * L; i += blockDim.x) {
      const int li = i / L, x = i % L - HB;
      const size_t l = lb + li;
      const bool ok = l < lines && x >= 0 && x < P;
      s0[i] = ok ? in0[l * P + x] : 0.0;
      s1[i] = ok ? in1[l * P + x] : 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < LPB * P; i += blockDim.x) {
      const int li = i / P, o = i % P;
      const size_t l = lb + li;
      if (l >= lines) break;
      const int c = band_class<HB>(o, P) * W;
      const double *v0 = s0 + li * L + o, *v1 = s1 + li * L + o;   // v[d] = in[o - HB + d]
      double acc = 0.0;
#pragma unroll
      for (int d = 0; d < W; ++d) acc += ta[c + d] * v0[d];
#pragma unroll
      for (int d = 0; d < W; ++d) acc += tb[c + d] * v1[d];
      out[l * P + o] = acc;
    }
  }
}

inline int grid_of(size_t count) {
  size_t g = (count + 255) / 256;
  if (g < 1) g = 1;
  return int(g > 65536 ? 65536 : g);
}

template <int HB>
void box_apply_impl(hipStream_t s, int P, int nb, const double *Kc, const double *Mc, const double *v, double *t1,
                    double *t2, double *t3, double *t4, double *y) {
  constexpr int RYZ = 8;
  const size_t lines = size_t(nb) * P * P;
  const int gyz = grid_of(lines * ((P + RYZ - 1) / RYZ));
  const int gx = int(std::min<size_t>((lines + kBandLines - 1) / kBandLines, 65536));
  const size_t shx = (size_t(2) * kBandLines * (P + 2 * HB) + size_t(2) * (HB + 2) * (2 * HB + 1)) * sizeof(double);
  // t1 = Mz v, t3 = Kz v
  hipLaunchKernelGGL((k_box_band<HB, RYZ>), dim3(gyz), dim3(256), 0, s, P, 2, nb, Mc, Mc, Kc, v, nullptr, t1, t3);
  // t2 = Ky t1 + My t3, t4 = My t1
  hipLaunchKernelGGL((k_box_band<HB, RYZ>), dim3(gyz), dim3(256), 0, s, P, 1, nb, Kc, Mc, Mc, t1, t3, t2, t4);
  // y = Kx t4 + Mx t2
  hipLaunchKernelGGL((k_box_band_x<HB>), dim3(gx), dim3(256), shx, s, P, lines, Kc, Mc, t4, t2, y);
}

}  // namespace

int launch_box_apply(hipStream_t s, int P, int nb, int p, const double *Kc, const double *Mc, const double *v,
                     double *t1, double *t2, double *t3, double *t4, double *y) {
  if (P < 2 * p + 1) return -1;   // the class rows need two elements
  switch (p) {
    case 4: box_apply_impl<4>(s, P, nb, Kc, Mc, v, t1, t2, t3, t4, y); return 0;
    case 5: box_apply_impl<5>(s, P, nb, Kc, Mc, v, t1, t2, t3, t4, y); return 0;
    case 6: box_apply_impl<6>(s, P, nb, Kc, Mc, v, t1, t2, t3, t4, y); return 0;
    default: return -1;
  }
}

int launch_box_bvals(hipStream_t s, int nb, int n, int nsr, int p, int64_t N, const BoxNodes &nodes, const int *start,
                     const double *sg, const double *sQ, const double *Wneg, double *phiB) {
  const size_t P = size_t(p) * n + 1;
  const int g = grid_of(size_t(nb) * 6 * P * P);
  switch (p) {
    case 4: hipLaunchKernelGGL(k_box_bvals<4>, dim3(g), dim3(256), 0, s, n, nsr, nb, N, nodes, start, sg, sQ, Wneg, phiB); return 0;
    case 5: hipLaunchKernelGGL(k_box_bvals<5>, dim3(g), dim3(256), 0, s, n, nsr, nb, N, nodes, start, sg, sQ, Wneg, phiB); return 0;
    case 6: hipLaunchKernelGGL(k_box_bvals<6>, dim3(g), dim3(256), 0, s, n, nsr, nb, N, nodes, start, sg, sQ, Wneg, phiB); return 0;
    default: return -1;
  }
}

void launch_box_interior(hipStream_t s, int P, int nb, bool to_interior, const double *src, double *dst) {
  const size_t Pi = size_t(P) - 2;
  hipLaunchKernelGGL(k_box_interior, dim3(grid_of(Pi * Pi * Pi * nb)), dim3(256), 0, s, P, nb, to_interior, src, dst);
}

void launch_box_axpby(hipStream_t s, size_t total, double a, const double *x, double c, double *y) {
  hipLaunchKernelGGL(k_box_axpby, dim3(grid_of(total)), dim3(256), 0, s, total, a, x, c, y);
}

void launch_box_fill(hipStream_t s, size_t total, double v, double *y) {
  hipLaunchKernelGGL(k_box_fill, dim3(grid_of(total)), dim3(256), 0, s, total, v, y);
}

int launch_box_addphi(hipStream_t s, int nb, int n, int p, const double *phi, double *W) {
  const size_t total = size_t(nb) * n * n * n * (p + 1) * (p + 1) * (p + 1);
  switch (p) {
    case 4: hipLaunchKernelGGL(k_box_addphi<4>, dim3(grid_of(total)), dim3(256), 0, s, n, nb, phi, W); return 0;
    case 5: hipLaunchKernelGGL(k_box_addphi<5>, dim3(grid_of(total)), dim3(256), 0, s, n, nb, phi, W); return 0;
    case 6: hipLaunchKernelGGL(k_box_addphi<6>, dim3(grid_of(total)), dim3(256), 0, s, n, nb, phi, W); return 0;
    default: return -1;
  }
}

int launch_box_resid(hipStream_t s, int P, int nb, bool interior, bool plain, const double *b, const double *y,
                     double *partial) {
  const int off = interior ? 1 : 0;
  const size_t Pi = size_t(P) - 2 * off;
  const size_t peri = Pi * Pi * Pi;
  int K = int(std::min<size_t>((peri + 255) / 256, size_t(1024) / size_t(nb > 0 ? nb : 1)));
  if (K < 1) K = 1;
  hipLaunchKernelGGL(k_box_resid, dim3(nb * K), dim3(256), 0, s, P, off, plain ? 1 : 0, K, nb, b, y, partial);
  return K;
}

int launch_box_assemble(hipStream_t s, int nb, int n, int p, const double *gE, double *G) {
  const size_t P = size_t(p) * n + 1;
  const int g = grid_of(P * P * P * nb);
  switch (p) {
    case 4: hipLaunchKernelGGL(k_box_assemble<4>, dim3(g), dim3(256), 0, s, n, nb, gE, G); return 0;
    case 5: hipLaunchKernelGGL(k_box_assemble<5>, dim3(g), dim3(256), 0, s, n, nb, gE, G); return 0;
    case 6: hipLaunchKernelGGL(k_box_assemble<6>, dim3(g), dim3(256), 0, s, n, nb, gE, G); return 0;
    default: return -1;
  }
}

int launch_box_charge_bnd(hipStream_t s, int nb, int n, int nsr, int p, int64_t N, const int *off, double inv_h,
                          const BoxNodes &nodes, const double *sg, const double *sQ, const double *mu, const int *perm,
                          double *F, double *dUdQ) {
  const int g = int(std::min<int64_t>((N + 3) / 4, 65535));   // one wave per charge, four per block
  switch (p) {
    case 4: hipLaunchKernelGGL(k_box_charge_bnd<4>, dim3(g), dim3(256), 0, s, n, nsr, nb, N, off, inv_h, nodes, sg, sQ, mu, perm, F, dUdQ); return 0;
    case 5: hipLaunchKernelGGL(k_box_charge_bnd<5>, dim3(g), dim3(256), 0, s, n, nsr, nb, N, off, inv_h, nodes, sg, sQ, mu, perm, F, dUdQ); return 0;
    case 6: hipLaunchKernelGGL(k_box_charge_bnd<6>, dim3(g), dim3(256), 0, s, n, nsr, nb, N, off, inv_h, nodes, sg, sQ, mu, perm, F, dUdQ); return 0;
    default: return -1;
  }
}

int launch_box_flux(hipStream_t s, int nb, int n, int nsr, int p, int64_t N, const BoxQuad &qd, const int *start,
                    const double *sg, const double *sQ, const double *Wneg, double *tF, double *f) {
  const int g = nb * 6 * n * n;
  const size_t P = size_t(p) * n + 1;
  switch (p) {
    case 4:
      hipLaunchKernelGGL(k_box_flux<4>, dim3(g), dim3(128), 0, s, n, nsr, N, qd, start, sg, sQ, Wneg, tF);
      hipLaunchKernelGGL(k_box_flux_add<4>, dim3(grid_of(P * P * P * nb)), dim3(256), 0, s, n, nb, tF, f);
      return 0;
    case 5:
      hipLaunchKernelGGL(k_box_flux<5>, dim3(g), dim3(128), 0, s, n, nsr, N, qd, start, sg, sQ, Wneg, tF);
      hipLaunchKernelGGL(k_box_flux_add<5>, dim3(grid_of(P * P * P * nb)), dim3(256), 0, s, n, nb, tF, f);
      return 0;
    case 6:
      hipLaunchKernelGGL(k_box_flux<6>, dim3(g), dim3(128), 0, s, n, nsr, N, qd, start, sg, sQ, Wneg, tF);
      hipLaunchKernelGGL(k_box_flux_add<6>, dim3(grid_of(P * P * P * nb)), dim3(256), 0, s, n, nb, tF, f);
      return 0;
    default: return -1;
  }
}

void launch_box_sub_mass(hipStream_t s, int P, int nb, double invV, const double *w1, const double *sums, double *f) {
  const size_t per = size_t(P) * P * P;
  hipLaunchKernelGGL(k_box_sub_mass, dim3(grid_of(per * nb)), dim3(256), 0, s, P, nb, invV, w1, sums, f);
}

int launch_box_mu_slots(hipStream_t s, int nb, int n, int p, const double *mu, double *gE) {
  const size_t P = size_t(p) * n + 1;
  const int g = grid_of(size_t(nb) * 6 * P * P);
  switch (p) {
    case 4: hipLaunchKernelGGL(k_box_mu_slots<4>, dim3(g), dim3(256), 0, s, n, nb, mu, gE); return 0;
    case 5: hipLaunchKernelGGL(k_box_mu_slots<5>, dim3(g), dim3(256), 0, s, n, nb, mu, gE); return 0;
    case 6: hipLaunchKernelGGL(k_box_mu_slots<6>, dim3(g), dim3(256), 0, s, n, nb, mu, gE); return 0;
    default: return -1;
  }
}

int launch_box_flux_adj(hipStream_t s, int nb, int n, int p, const BoxQuad &qd, const double *lam, double *Lw,
                        double *hF) {
  const int g = nb * 6 * n * n;
  switch (p) {
    case 4: hipLaunchKernelGGL(k_box_flux_adj<4>, dim3(g), dim3(128), 0, s, n, qd, lam, Lw, hF); return 0;
    case 5: hipLaunchKernelGGL(k_box_flux_adj<5>, dim3(g), dim3(128), 0, s, n, qd, lam, Lw, hF); return 0;
    case 6: hipLaunchKernelGGL(k_box_flux_adj<6>, dim3(g), dim3(128), 0, s, n, qd, lam, Lw, hF); return 0;
    default: return -1;
  }
}

int launch_box_h_slots(hipStream_t s, int nb, int n, int p, const double *hF, double *gE) {
  const int g = grid_of(size_t(nb) * n * n * n * (p + 1) * (p + 1) * (p + 1));
  switch (p) {
    case 4: hipLaunchKernelGGL(k_box_h_slots<4>, dim3(g), dim3(256), 0, s, n, nb, hF, gE); return 0;
    case 5: hipLaunchKernelGGL(k_box_h_slots<5>, dim3(g), dim3(256), 0, s, n, nb, hF, gE); return 0;
    case 6: hipLaunchKernelGGL(k_box_h_slots<6>, dim3(g), dim3(256), 0, s, n, nb, hF, gE); return 0;
    default: return -1;
  }
}

int launch_box_flux_charge(hipStream_t s, int nb, int n, int nsr, int p, int64_t N, const int *off, double inv_h,
                           const BoxQuad &qd, const double *sg, const double *sQ, const double *Lw, const int *perm,
                           double *F, double *dUdQ) {
  const int g = int(std::min<int64_t>((N + 3) / 4, 65535));   // one wave per charge, four per block
  switch (p) {
    case 4: hipLaunchKernelGGL(k_box_flux_charge<4>, dim3(g), dim3(256), 0, s, n, nsr, nb, N, off, inv_h, qd, sg, sQ, Lw, perm, F, dUdQ); return 0;
    case 5: hipLaunchKernelGGL(k_box_flux_charge<5>, dim3(g), dim3(256), 0, s, n, nsr, nb, N, off, inv_h, qd, sg, sQ, Lw, perm, F, dUdQ); return 0;
    case 6: hipLaunchKernelGGL(k_box_flux_charge<6>, dim3(g), dim3(256), 0, s, n, nsr, nb, N, off, inv_h, qd, sg, sQ, Lw, perm, F, dUdQ); return 0;
    default: return -1;
  }
}

}  // namespace fep3m
