// Kernels of the screen families other than the one-element q = 3 screen
// (Section 2.1: 27-element screens of degree q = 1..4; Section 5:
// one-element screens of degree q != 3).  They differ from it in the number
// of moments per axis (NL = d + 1), the element order (PO = q + 2) and the
// support of an element's screens (SPAN = 1 or 3 elements per axis), so the
// stages that touch the screens have their own float64 kernels here:
//   moments      C[E][a] = sum_{i in E} Q_i u_i^a, a = ax + NL ay + NL^2 az
//   load         b_g = 4 pi sum over the source elements whose support holds
//                node g of sum_a C[s][a] gw[ax][jx] gw[ay][jy] gw[az][jz],
//                j the node's index in the source's support (gather form)
//   near field   W_E[m] = phi_E[m] - sum_D sum_a T[a][D][m] C[E - D][a]
//   adjoint      A[E][a] = 4 pi <lambda on the support of E, G_a>
//                          - sum_D <g_{E + D}, T_a[D]>
// The pair sum, the interpolation, the deposit, the assembly, the mesh
// operator and the forces are shared with the q = 3 path (templated on the
// order and the moment count).
//
// Element ids are configuration-major (b n^3 + e); mesh vectors are nb
// consecutive (PO n)^3 blocks [z][y][x].
#include <algorithm>

#include "kernels.hpp"

namespace fep3m {
namespace {

__device__ __forceinline__ int wrapn(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Fixed-order block sum (shuffle tree in each wave, then the waves in
// order); valid in thread 0.  blockDim a multiple of 64, at most 1024.
__device__ double block_sum_s(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

// One thread per (element, moment).
template <int NL>
__global__ __launch_bounds__(256) void k_moments_g(int n, int MT, int64_t N, const int *__restrict__ start,
                                                   const double *__restrict__ sg, const double *__restrict__ sQ,
                                                   double *__restrict__ C) {
  constexpr int NA = NL * NL * NL;
  const int M = n * n * n;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < int64_t(MT) * NA;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int E = int(t / NA), a = int(t % NA);
    const int ax = a % NL, ay = (a / NL) % NL, az = a / (NL * NL);
    const int El = E % M;
    const int ex = El % n, ey = (El / n) % n, ez = El / (n * n);
    double c = 0.0;
    auto add = [&](double q, double gx, double gy, double gz) {
      const double ux = gx - ex - 0.5, uy = gy - ey - 0.5, uz = gz - ez - 0.5;
      double m = q;
      for (int k = 0; k < ax; ++k) m *= ux;
      for (int k = 0; k < ay; ++k) m *= uy;
      for (int k = 0; k < az; ++k) m *= uz;
      c += m;
    };
    // four charges' loads in flight before they are summed, in order
    const int s1 = start[E + 1];
    int s = start[E];
    for (; s + 4 <= s1; s += 4) {
      double q[4], gx[4], gy[4], gz[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        q[u] = sQ[s + u];
        gx[u] = sg[s + u];
        gy[u] = sg[N + s + u];
        gz[u] = sg[2 * N + s + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) add(q[u], gx[u], gy[u], gz[u]);
    }
    for (; s < s1; ++s) add(sQ[s], sg[s], sg[N + s], sg[2 * N + s]);
    C[t] = c;
  }
}

// Sources along one axis whose support holds global node g: SPAN of them
// (SPAN + 1 at an element vertex), with the node's index j in each support.
// In a box (no wrap) a source outside [0, n) gets j = -1.
template <int PO, int SPAN>
__device__ __forceinline__ int axis_sources(int g, int n, bool box, int (&s)[SPAN + 1], int (&j)[SPAN + 1]) {
  constexpr int H = (SPAN - 1) / 2;
  const int e = g / PO, k = g - e * PO;
  const int lo = e - SPAN + (k > 0 ? 1 : 0);   // lowest s - H
  const int cnt = e - lo + 1;
#pragma unroll
  for (int c = 0; c < SPAN + 1; ++c) {
    const int sh = lo + c;
    s[c] = box ? sh + H : ((sh + H) % n + n) % n;
    j[c] = (box && (s[c] < 0 || s[c] >= n)) ? -1 : g - PO * sh;
  }
  return cnt;
}

// b (per configuration, K blocks strided over its nodes) and block partials
// of sum b for the compatibility projection.  box: the (PO n + 1)^3 nodes of
// the box [0, n]^3, elements outside it contribute nothing.
template <int PO, int SPAN, int NL>
__global__ __launch_bounds__(256) void k_load_g(int n, int K, int box, const double *__restrict__ Call,
                                                const double *__restrict__ gw, double *__restrict__ ball,
                                                double *__restrict__ partial) {
  constexpr int NA = NL * NL * NL, KS = SPAN * PO + 1;
  __shared__ double red[8];
  const int P = PO * n + (box ? 1 : 0);
  const size_t per = size_t(P) * P * P;
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const double *C = Call + size_t(cfg) * n * n * n * NA;
  double *b = ball + size_t(cfg) * per;
  double acc = 0.0;
  for (size_t g = size_t(kb) * blockDim.x + threadIdx.x; g < per; g += size_t(K) * blockDim.x) {
    const int gx = int(g % P), gy = int((g / P) % P), gz = int(g / (size_t(P) * P));
    int sx[SPAN + 1], jx[SPAN + 1], sy[SPAN + 1], jy[SPAN + 1], sz[SPAN + 1], jz[SPAN + 1];
    const int cx = axis_sources<PO, SPAN>(gx, n, box, sx, jx);
    const int cy = axis_sources<PO, SPAN>(gy, n, box, sy, jy);
    const int cz = axis_sources<PO, SPAN>(gz, n, box, sz, jz);
    double v = 0.0;
#pragma unroll
    for (int iz = 0; iz < SPAN + 1; ++iz) {
      if (iz >= cz || jz[iz] < 0) continue;
#pragma unroll
      for (int iy = 0; iy < SPAN + 1; ++iy) {
        if (iy >= cy || jy[iy] < 0) continue;
#pragma unroll
        for (int ix = 0; ix < SPAN + 1; ++ix) {
          if (ix >= cx || jx[ix] < 0) continue;
          const double *c = C + (size_t(sx[ix]) + size_t(n) * (sy[iy] + size_t(n) * sz[iz])) * NA;
          double tz = 0.0;
          for (int az = 0; az < NL; ++az) {
            double ty = 0.0;
            for (int ay = 0; ay < NL; ++ay) {
              double tx = 0.0;
              for (int ax = 0; ax < NL; ++ax) tx += gw[ax * KS + jx[ix]] * c[(az * NL + ay) * NL + ax];
              ty += gw[ay * KS + jy[iy]] * tx;
            }
            tz += gw[az * KS + jz[iz]] * ty;
          }
          v += tz;
        }
      }
    }
    v *= 4.0 * M_PI;
    b[g] = v;
    acc += v;
  }
  const double s = block_sum_s(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Near-screen field, Psi_E[m] = sum_D sum_a T[a][D][m] C[E - D][a].  A block
// takes a brick of 4 x 4 x 4 target elements and NG groups of MG nodes
// (NM = NG MG); thread (group, target) accumulates its group's nodes of its
// target.  The moments of the brick's source halo (the brick widened by
// n_sr <= 3 elements on every side) are staged in LDS AC moments at a time;
// per (offset D, moment a) a thread reads the one moment of its target's
// source E - D from LDS and multiplies it into MG table values that are the
// same for the whole wave (a wave lies inside one group), read through
// scalar loads.  Sums run over moment chunks, then D, then the chunk's
// moments.  box: sources outside [0, n)^3 are absent and phi is the
// (PO n + 1)^3 nodal field of the box; a null phi gives W = -Psi.
template <int PO, int NL>
struct PsiShape {
  static constexpr int NM = (PO + 1) * (PO + 1) * (PO + 1), NA = NL * NL * NL;
  static constexpr int MG = NM == 64 ? 16 : (NM == 125 ? 25 : (NM == 216 ? 27 : 49));
  static constexpr int NG = NM / MG;
  // TT targets per thread, 4 elements apart along x: with many moments the
  // table values (read once per thread) dominate, and a second target
  // halves their reads per result
  static constexpr int TT = (NA >= 27 && MG <= 27) ? 2 : 1;
  static constexpr int BX = 4 * TT, BY = 4, BZ = 4, TB = 64;   // TB threads per node group: one wave
  static constexpr int AC = NA < 8 ? NA : (TT == 2 ? 4 : 8);   // moments per LDS stage
  static constexpr int HX = BX + 6, HY = BY + 6, HZ = BZ + 6, NH = HX * HY * HZ;
  static constexpr int THREADS = NG * TB;
  static_assert(NG * MG == NM && THREADS <= 1024, "near-field brick shape");
};

template <int PO, int NL>
__global__ __launch_bounds__((PsiShape<PO, NL>::THREADS)) void k_psi_g(int n, int nsr, int box,
                                                                     const double *__restrict__ Call,
                                                                     const double *__restrict__ T,
                                                                     const double *__restrict__ phiall,
                                                                     double *__restrict__ Wall) {
  using S = PsiShape<PO, NL>;
  constexpr int Q1 = PO + 1, NM = S::NM, NA = S::NA, MG = S::MG, AC = S::AC, HX = S::HX, HY = S::HY, NH = S::NH;
  __shared__ double Cs[AC * NH];
  const int bxn = (n + S::BX - 1) / S::BX, byn = (n + S::BY - 1) / S::BY, bzn = (n + S::BZ - 1) / S::BZ;
  const int per_cfg = bxn * byn * bzn;
  const int cfg = blockIdx.x / per_cfg;
  const int br = blockIdx.x % per_cfg;
  const int bx = br % bxn, by = (br / bxn) % byn, bz = br / (bxn * byn);
  const size_t M = size_t(n) * n * n;
  const int P = PO * n + (box ? 1 : 0);
  const double *C = Call + size_t(cfg) * M * NA;
  const double *phi = phiall ? phiall + size_t(cfg) * P * P * P : nullptr;
  double *W = Wall + size_t(cfg) * M * NM;
  const int S1 = 2 * nsr + 1, ND = S1 * S1 * S1;
  constexpr int TT = S::TT;
  const int tid = threadIdx.x, t = tid % S::TB;
  const int g = __builtin_amdgcn_readfirstlane(tid / S::TB);
  const int tx = t % 4, ty = (t / 4) % S::BY, tz = t / (4 * S::BY);   // targets tx + 4 u, u < TT
  const int hx0 = bx * S::BX - nsr, hy0 = by * S::BY - nsr, hz0 = bz * S::BZ - nsr;
  const int LX = S::BX + 2 * nsr, LY = S::BY + 2 * nsr, LZ = S::BZ + 2 * nsr;   // halo in use
  // the source of offset D sits at halo (t + nsr - D): index hbase - (D + nsr) . (1, HX, HX HY)
  const int hbase = ((tz + 2 * nsr) * HY + ty + 2 * nsr) * HX + tx + 2 * nsr;
  double acc[TT][MG];
#pragma unroll
  for (int u = 0; u < TT; ++u)
#pragma unroll
    for (int j = 0; j < MG; ++j) acc[u][j] = 0.0;
  for (int a0 = 0; a0 < NA; a0 += AC) {
    __syncthreads();
    for (int i = tid; i < AC * LX * LY * LZ; i += S::THREADS) {
      const int aa = i % AC, h = i / AC;
      const int lx = h % LX, ly = (h / LX) % LY, lz = h / (LX * LY);
      int sx = hx0 + lx, sy = hy0 + ly, sz = hz0 + lz;
      const bool in = sx >= 0 && sx < n && sy >= 0 && sy < n && sz >= 0 && sz < n;
      if (!box) {
        sx = wrapn(sx, n);
        sy = wrapn(sy, n);
        sz = wrapn(sz, n);
      }
      double v = 0.0;
      if ((!box || in) && a0 + aa < NA) v = C[(size_t(sx) + size_t(n) * (sy + size_t(n) * sz)) * NA + a0 + aa];
      Cs[aa * NH + (lz * HY + ly) * HX + lx] = v;
    }
    __syncthreads();
    for (int dz = 0; dz < S1; ++dz)
      for (int dy = 0; dy < S1; ++dy) {
        const int hrow = hbase - (dz * HY + dy) * HX;
        const int iD0 = (dz * S1 + dy) * S1;
        for (int dx = 0; dx < S1; ++dx) {
          const double *Td = T + (size_t(a0) * ND + iD0 + dx) * NM + g * MG;
#pragma unroll
          for (int aa = 0; aa < AC; ++aa) {
            if (a0 + aa >= NA) break;
            double cv[TT];
#pragma unroll
            for (int u = 0; u < TT; ++u) cv[u] = Cs[aa * NH + hrow - dx + 4 * u];
            const double *Ta = Td + size_t(aa) * ND * NM;
#pragma unroll
            for (int j = 0; j < MG; ++j) {
              const double tv = Ta[j];
#pragma unroll
              for (int u = 0; u < TT; ++u) acc[u][j] += cv[u] * tv;
            }
          }
        }
      }
  }
#pragma unroll
  for (int u = 0; u < TT; ++u) {
    const int ex = bx * S::BX + tx + 4 * u, ey = by * S::BY + ty, ez = bz * S::BZ + tz;
    if (ex >= n || ey >= n || ez >= n) continue;
    const size_t E = size_t(ex) + size_t(n) * (ey + size_t(n) * ez);
    double *dst = W + E * NM + g * MG;
#pragma unroll
    for (int j = 0; j < MG; ++j) {
      const int m = g * MG + j;
      const int mx = m % Q1, my = (m / Q1) % Q1, mz = m / (Q1 * Q1);
      double ph = 0.0;
      if (phi) {
        const int gx = wrapn(PO * ex + mx, P), gy = wrapn(PO * ey + my, P), gz = wrapn(PO * ez + mz, P);
        ph = phi[(size_t(gz) * P + gy) * P + gx];
      }
      dst[j] = ph - acc[u][j];
    }
  }
}

// Near part of the moment adjoint, A[E][a] = -sum_D sum_m g_{E+D}[m] T[a][D][m].
// A block takes a brick of TB target elements and NG groups of AG moments
// (NA = NG AG); thread (group, target) accumulates its group's moments of its
// target.  The deposits of the brick's source halo (the brick widened by
// n_sr <= 3 elements on every side) are staged in LDS MC nodes at a time;
// per (offset D, node m) a thread reads the one deposit of its target's
// source E + D from LDS and multiplies it into AG table values that are the
// same for the whole wave (a wave lies inside one group), read from the
// transposed tables Tt[D][m][a] through scalar loads.  Sums run over m
// chunks, then D, then the chunk's nodes.
template <int NA>
struct AdjNearShape {
  static constexpr int AG = NA == 27 ? 9 : (NA == 125 ? 25 : (NA >= 8 ? 8 : NA));
  static constexpr int NG = NA / AG;
  static constexpr int TB = NG == 1 ? 256 : 64;   // threads per moment group (a multiple of the wave)
  // targets per thread, XT elements apart along x: with several groups each
  // thread takes two targets, halving the table reads per result
  static constexpr int TPT = NG == 1 ? 1 : 2;
  static constexpr int BX = 8, BY = TB == 256 ? 8 : 4, BZ = 4, XT = BX / TPT;
  static constexpr int MC = 2;                    // deposit nodes per LDS stage
  static constexpr int HX = BX + 6, HY = BY + 6, HZ = BZ + 6;
  static constexpr int NH = HX * HY * HZ;
  static constexpr int THREADS = NG * TB;
  static_assert(NG * AG == NA && BX * BY * BZ == TB * TPT && TB % 64 == 0, "adjoint brick shape");
};

template <int PO, int NL>
__global__ __launch_bounds__(AdjNearShape<NL * NL * NL>::THREADS) void k_adj_near_g(
    int n, int nsr, int box, const double *__restrict__ gEall, const double *__restrict__ Tt,
    double *__restrict__ Aall) {
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1, NA = NL * NL * NL;
  using S = AdjNearShape<NA>;
  constexpr int AG = S::AG, TB = S::TB, MC = S::MC, HX = S::HX, HY = S::HY, NH = S::NH;
  __shared__ double Gs[MC * NH];
  const int bxn = (n + S::BX - 1) / S::BX, byn = (n + S::BY - 1) / S::BY, bzn = (n + S::BZ - 1) / S::BZ;
  const int per_cfg = bxn * byn * bzn;
  const int cfg = blockIdx.x / per_cfg;
  const int br = blockIdx.x % per_cfg;
  const int bx = br % bxn, by = (br / bxn) % byn, bz = br / (bxn * byn);
  const size_t M = size_t(n) * n * n;
  const double *gE = gEall + size_t(cfg) * M * NM;
  double *A = Aall + size_t(cfg) * M * NA;
  const int S1 = 2 * nsr + 1, ND = S1 * S1 * S1;
  const int tid = threadIdx.x, t = tid % TB;
  const int g = __builtin_amdgcn_readfirstlane(tid / TB);
  constexpr int TPT = S::TPT, XT = S::XT;
  const int tx = t % XT, ty = (t / XT) % S::BY, tz = t / (XT * S::BY);   // targets tx + XT u, u < TPT
  const int hx0 = bx * S::BX - nsr, hy0 = by * S::BY - nsr, hz0 = bz * S::BZ - nsr;
  const int LX = S::BX + 2 * nsr, LY = S::BY + 2 * nsr, LZ = S::BZ + 2 * nsr;   // halo in use
  const int hbase = (tz * HY + ty) * HX + tx;   // halo index of the source at D = (-nsr, -nsr, -nsr)
  double acc[TPT][AG];
#pragma unroll
  for (int u = 0; u < TPT; ++u)
#pragma unroll
    for (int j = 0; j < AG; ++j) acc[u][j] = 0.0;
  for (int m0 = 0; m0 < NM; m0 += MC) {
    __syncthreads();
    for (int i = tid; i < MC * LX * LY * LZ; i += S::THREADS) {
      const int mm = i % MC, h = i / MC;
      const int lx = h % LX, ly = (h / LX) % LY, lz = h / (LX * LY);
      int sx = hx0 + lx, sy = hy0 + ly, sz = hz0 + lz;
      const bool in = sx >= 0 && sx < n && sy >= 0 && sy < n && sz >= 0 && sz < n;
      if (!box) {
        sx = wrapn(sx, n);
        sy = wrapn(sy, n);
        sz = wrapn(sz, n);
      }
      double v = 0.0;
      if ((!box || in) && m0 + mm < NM) v = gE[(size_t(sx) + size_t(n) * (sy + size_t(n) * sz)) * NM + m0 + mm];
      Gs[mm * NH + (lz * HY + ly) * HX + lx] = v;
    }
    __syncthreads();
    for (int dz = 0; dz < S1; ++dz)
      for (int dy = 0; dy < S1; ++dy) {
        const int hrow = hbase + (dz * HY + dy) * HX;
        const double *Trow = Tt + (size_t((dz * S1 + dy) * S1) * NM + m0) * NA + g * AG;
        if constexpr (TPT > 1) {
          for (int dx = 0; dx < S1; ++dx) {
            const double *Td = Trow + size_t(dx) * NM * NA;
#pragma unroll
            for (int mm = 0; mm < MC; ++mm) {
              if (m0 + mm >= NM) break;
              double gv[TPT];
#pragma unroll
              for (int u = 0; u < TPT; ++u) gv[u] = Gs[mm * NH + hrow + dx + XT * u];
#pragma unroll
              for (int j = 0; j < AG; ++j) {
                const double tv = Td[mm * NA + j];
#pragma unroll
                for (int u = 0; u < TPT; ++u) acc[u][j] += gv[u] * tv;
              }
            }
          }
          continue;
        }
        // offsets two at a time: both offsets' table values are requested
        // before the first is used (S1 is odd: the last offset alone)
        int dx = 0;
        for (; dx + 1 < S1; dx += 2) {
          const double *Td = Trow + size_t(dx) * NM * NA;
          double tv[2][MC][AG], gv[2][MC];
#pragma unroll
          for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int mm = 0; mm < MC; ++mm) {
              const bool ok = m0 + mm < NM;
              gv[u][mm] = ok ? Gs[mm * NH + hrow + dx + u] : 0.0;
#pragma unroll
              for (int j = 0; j < AG; ++j) tv[u][mm][j] = ok ? Td[size_t(u) * NM * NA + mm * NA + j] : 0.0;
            }
#pragma unroll
          for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int mm = 0; mm < MC; ++mm)
#pragma unroll
              for (int j = 0; j < AG; ++j) acc[0][j] += gv[u][mm] * tv[u][mm][j];
        }
        {
          const double *Td = Trow + size_t(dx) * NM * NA;
#pragma unroll
          for (int mm = 0; mm < MC; ++mm) {
            if (m0 + mm >= NM) break;
            const double gv = Gs[mm * NH + hrow + dx];
#pragma unroll
            for (int j = 0; j < AG; ++j) acc[0][j] += gv * Td[mm * NA + j];
          }
        }
      }
  }
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    const int ex = bx * S::BX + tx + XT * u, ey = by * S::BY + ty, ez = bz * S::BZ + tz;
    if (ex >= n || ey >= n || ez >= n) continue;
    double *dst = A + (size_t(ex) + size_t(n) * (ey + size_t(n) * ez)) * NA + g * AG;
#pragma unroll
    for (int j = 0; j < AG; ++j) dst[j] = -acc[u][j];
  }
}

// Mesh part of the moment adjoint: A[E][a] += 4 pi sum over the support's
// nodes of lambda * gw[ax][jx] gw[ay][jy] gw[az][jz], one thread per
// (element, moment), contracted along x, then y, then z.  box: lambda on the
// (PO n + 1)^3 nodes of the box (SPAN 1, so no index leaves it).
// The same load separably (periodic; SPAN 3: the 27-element screens, SPAN
// 1: the one-element screens): b = 4 pi (W_z (x) W_y (x) W_x) C, W mapping
// (source element s, moment index a) of one axis to the nodes g of the
// source's support with weight gw[a][g - p (s - H)], H = (SPAN - 1) / 2.
// Three passes, each a 1-D gather over the SPAN or SPAN + 1 sources of a
// node (every moment of a source element is read once per pass instead of
// once per node of its support):
//   x:  T1[c][sz][sy][az][ay][gx] = sum_{sx, ax} W_x C[c][sz][sy][sx][az][ay][ax]
//   y:  T2[c][sz][az][gy][gx]     = sum_{sy, ay} W_y T1
//   z:  b[c][gz][gy][gx]          = 4 pi sum_{sz, az} W_z T2  (with block partials of b)
template <int PO, int SPAN, int NL>
__global__ __launch_bounds__(256) void k_load_sx(int nb, int n, const double *__restrict__ C,
                                                 const double *__restrict__ gw, double *__restrict__ T1) {
  constexpr int NA = NL * NL * NL, NL2 = NL * NL, KS = SPAN * PO + 1;
  const int P = PO * n;
  const size_t rows = size_t(nb) * n * n;   // (c, sz, sy)
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < rows * P; t += size_t(gridDim.x) * blockDim.x) {
    const int gx = int(t % P);
    const size_t row = t / P;
    int sx[SPAN + 1], jx[SPAN + 1];
    const int cx = axis_sources<PO, SPAN>(gx, n, false, sx, jx);
    double acc[NL2];
#pragma unroll
    for (int q = 0; q < NL2; ++q) acc[q] = 0.0;
#pragma unroll
    for (int i = 0; i < SPAN + 1; ++i) {
      if (i >= cx) break;
      double w[NL];
#pragma unroll
      for (int ax = 0; ax < NL; ++ax) w[ax] = gw[ax * KS + jx[i]];
      const double *c = C + (row * n + sx[i]) * NA;
#pragma unroll
      for (int q = 0; q < NL2; ++q) {
        double v = 0.0;
#pragma unroll
        for (int ax = 0; ax < NL; ++ax) v += w[ax] * c[q * NL + ax];
        acc[q] += v;
      }
    }
#pragma unroll
    for (int q = 0; q < NL2; ++q) T1[(row * NL2 + q) * P + gx] = acc[q];
  }
}

template <int PO, int SPAN, int NL>
__global__ __launch_bounds__(256) void k_load_sy(int nb, int n, const double *__restrict__ gw,
                                                 const double *__restrict__ T1, double *__restrict__ T2) {
  constexpr int NL2 = NL * NL, KS = SPAN * PO + 1;
  const int P = PO * n;
  const size_t P2 = size_t(P) * P;
  const size_t total = size_t(nb) * n * P2;   // (c, sz, gy, gx)
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += size_t(gridDim.x) * blockDim.x) {
    const int gx = int(t % P), gy = int((t / P) % P);
    const size_t csz = t / P2;   // c n + sz
    int sy[SPAN + 1], jy[SPAN + 1];
    const int cy = axis_sources<PO, SPAN>(gy, n, false, sy, jy);
    double acc[NL];
#pragma unroll
    for (int az = 0; az < NL; ++az) acc[az] = 0.0;
#pragma unroll
    for (int i = 0; i < SPAN + 1; ++i) {
      if (i >= cy) break;
      const double *r = T1 + ((csz * n + sy[i]) * NL2) * P + gx;
#pragma unroll
      for (int az = 0; az < NL; ++az) {
        double v = 0.0;
#pragma unroll
        for (int ay = 0; ay < NL; ++ay) v += gw[ay * KS + jy[i]] * r[size_t(az * NL + ay) * P];
        acc[az] += v;
      }
    }
#pragma unroll
    for (int az = 0; az < NL; ++az) T2[((csz * NL + az) * P + gy) * P + gx] = acc[az];
  }
}

template <int PO, int SPAN, int NL>
__global__ __launch_bounds__(256) void k_load_sz(int n, int K, const double *__restrict__ gw,
                                                 const double *__restrict__ T2all, double *__restrict__ ball,
                                                 double *__restrict__ partial) {
  constexpr int KS = SPAN * PO + 1;
  __shared__ double red[8];
  const int P = PO * n;
  const size_t P2 = size_t(P) * P, per = P2 * P;
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const double *T2 = T2all + size_t(cfg) * n * NL * P2;
  double *b = ball + size_t(cfg) * per;
  double acc = 0.0;
  for (size_t g = size_t(kb) * blockDim.x + threadIdx.x; g < per; g += size_t(K) * blockDim.x) {
    const size_t gxy = g % P2;
    const int gz = int(g / P2);
    int sz[SPAN + 1], jz[SPAN + 1];
    const int cz = axis_sources<PO, SPAN>(gz, n, false, sz, jz);
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < SPAN + 1; ++i) {
      if (i >= cz) break;
#pragma unroll
      for (int az = 0; az < NL; ++az) v += gw[az * KS + jz[i]] * T2[(size_t(sz[i]) * NL + az) * P2 + gxy];
    }
    v *= 4.0 * M_PI;
    b[g] = v;
    acc += v;
  }
  const double s = block_sum_s(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <int PO, int SPAN, int NL>
__global__ __launch_bounds__(256) void k_adj_lam_g(int n, int MT, int box, const double *__restrict__ lamall,
                                                   const double *__restrict__ gw, double *__restrict__ A) {
  constexpr int NA = NL * NL * NL, KS = SPAN * PO + 1, H = (SPAN - 1) / 2;
  const int M = n * n * n, P = PO * n + (box ? 1 : 0);
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < int64_t(MT) * NA;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int E = int(t / NA), a = int(t % NA);
    const int ax = a % NL, ay = (a / NL) % NL, az = a / (NL * NL);
    const int cfg = E / M, El = E % M;
    const int ex = El % n, ey = (El / n) % n, ez = El / (n * n);
    const double *lam = lamall + size_t(cfg) * P * P * P;
    const int x0 = PO * (ex - H), y0 = PO * (ey - H), z0 = PO * (ez - H);
    double sz = 0.0;
    for (int kz = 0; kz < KS; ++kz) {
      const size_t rz = size_t(wrapn(((z0 + kz) % P + P) % P, P)) * P;
      double sy = 0.0;
      for (int ky = 0; ky < KS; ++ky) {
        const double *row = lam + (rz + size_t(wrapn(((y0 + ky) % P + P) % P, P))) * P;
        double sx = 0.0;
        for (int kx = 0; kx < KS; ++kx) sx += gw[ax * KS + kx] * row[wrapn(((x0 + kx) % P + P) % P, P)];
        sy += gw[ay * KS + ky] * sx;
      }
      sz += gw[az * KS + kz] * sy;
    }
    A[t] += 4.0 * M_PI * sz;
  }
}

// The lambda part of the moment adjoint, the transpose of the separable
// load (periodic): A += 4 pi (W_z (x) W_y (x) W_x)^T lam, one axis at a time
// through the load's scratch:
//   z:  U1[c][sz][az][gy][gx]     = sum_kz gw[az][kz] lam[p (sz - H) + kz][gy][gx]
//   y:  U2[c][sz][sy][az][ay][gx] = sum_ky gw[ay][ky] U1[c][sz][az][p (sy - H) + ky][gx]
//   x:  A[c][sz][sy][sx][az][ay][ax] += 4 pi sum_kx gw[ax][kx] U2[c][sz][sy][az][ay][p (sx - H) + kx]
// (node indices wrap modulo P = p n).
template <int PO, int SPAN, int NL>
__global__ __launch_bounds__(256) void k_adjl_z(int nb, int n, const double *__restrict__ lamall,
                                                const double *__restrict__ gw, double *__restrict__ U1) {
  constexpr int KS = SPAN * PO + 1;
  const int P = PO * n;
  const size_t P2 = size_t(P) * P;
  const size_t total = size_t(nb) * n * P2;   // (c, sz, gy, gx)
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += size_t(gridDim.x) * blockDim.x) {
    const size_t gxy = t % P2, csz = t / P2;
    const int sz = int(csz % n);
    const size_t c = csz / n;
    const double *lam = lamall + c * P2 * P + gxy;
    const int z0 = PO * (sz - (SPAN - 1) / 2);
    double acc[NL];
#pragma unroll
    for (int az = 0; az < NL; ++az) acc[az] = 0.0;
#pragma unroll
    for (int kz = 0; kz < KS; ++kz) {
      const double v = lam[size_t(((z0 + kz) % P + P) % P) * P2];
#pragma unroll
      for (int az = 0; az < NL; ++az) acc[az] += gw[az * KS + kz] * v;
    }
#pragma unroll
    for (int az = 0; az < NL; ++az) U1[(csz * NL + az) * P2 + gxy] = acc[az];
  }
}

template <int PO, int SPAN, int NL>
__global__ __launch_bounds__(256) void k_adjl_y(int nb, int n, const double *__restrict__ gw,
                                                const double *__restrict__ U1, double *__restrict__ U2) {
  constexpr int KS = SPAN * PO + 1, NL2 = NL * NL;
  const int P = PO * n;
  const size_t P2 = size_t(P) * P;
  const size_t total = size_t(nb) * n * n * P;   // (c, sz, sy, gx)
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += size_t(gridDim.x) * blockDim.x) {
    const int gx = int(t % P);
    const size_t row = t / P;   // (c n + sz) n + sy
    const int sy = int(row % n);
    const size_t csz = row / n;
    const int y0 = PO * (sy - (SPAN - 1) / 2);
#pragma unroll
    for (int az = 0; az < NL; ++az) {
      const double *u = U1 + (csz * NL + az) * P2 + gx;
      double acc[NL];
#pragma unroll
      for (int ay = 0; ay < NL; ++ay) acc[ay] = 0.0;
#pragma unroll
      for (int ky = 0; ky < KS; ++ky) {
        const double v = u[size_t(((y0 + ky) % P + P) % P) * P];
#pragma unroll
        for (int ay = 0; ay < NL; ++ay) acc[ay] += gw[ay * KS + ky] * v;
      }
#pragma unroll
      for (int ay = 0; ay < NL; ++ay) U2[(row * NL2 + az * NL + ay) * P + gx] = acc[ay];
    }
  }
}

template <int PO, int SPAN, int NL>
__global__ __launch_bounds__(256) void k_adjl_x(int nb, int n, const double *__restrict__ gw,
                                                const double *__restrict__ U2, double *__restrict__ A) {
  constexpr int KS = SPAN * PO + 1, NL2 = NL * NL, NA = NL2 * NL;
  const int P = PO * n;
  const size_t total = size_t(nb) * n * n * n * NL2;   // (c, sz, sy, q = (az, ay), sx)
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += size_t(gridDim.x) * blockDim.x) {
    const int sx = int(t % n);
    const size_t rq = t / n;   // row NL2 + q
    const int q = int(rq % NL2);
    const size_t row = rq / NL2;
    const double *u = U2 + rq * P;
    const int x0 = PO * (sx - (SPAN - 1) / 2);
    double acc[NL];
#pragma unroll
    for (int ax = 0; ax < NL; ++ax) acc[ax] = 0.0;
#pragma unroll
    for (int kx = 0; kx < KS; ++kx) {
      const double v = u[((x0 + kx) % P + P) % P];
#pragma unroll
      for (int ax = 0; ax < NL; ++ax) acc[ax] += gw[ax * KS + kx] * v;
    }
    double *a = A + (row * n + sx) * NA + q * NL;
#pragma unroll
    for (int ax = 0; ax < NL; ++ax) a[ax] += 4.0 * M_PI * acc[ax];
  }
}

inline int grid_for_count(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g < 1) g = 1;
  return int(g > 65536 ? 65536 : g);
}

}  // namespace

// ----------------------------------------------------------------- launchers

#define FEP3M_NL_SWITCH(NLV, CALL) \
  switch (NLV) {                   \
    case 1: CALL(1); break;        \
    case 2: CALL(2); break;        \
    case 3: CALL(3); break;        \
    case 4: CALL(4); break;        \
    case 5: CALL(5); break;        \
    default: return -1;            \
  }

int launch_moments_g(hipStream_t s, int nb, int n, int nl, int64_t N, const int *start, const double *sg,
                     const double *sQ, double *C) {
  const int MT = nb * n * n * n;
  const int g = grid_for_count(int64_t(MT) * nl * nl * nl);
#define CALL(NL) hipLaunchKernelGGL(k_moments_g<NL>, dim3(g), dim3(256), 0, s, n, MT, N, start, sg, sQ, C)
  FEP3M_NL_SWITCH(nl, CALL)
#undef CALL
  return 0;
}

template <int PO, int SPAN>
static int load_g_nl(hipStream_t s, int nb, int n, int nl, int K, int box, const double *C, const double *gw,
                     double *b, double *partial) {
#define CALL(NL) \
  hipLaunchKernelGGL((k_load_g<PO, SPAN, NL>), dim3(nb * K), dim3(256), 0, s, n, K, box, C, gw, b, partial)
  FEP3M_NL_SWITCH(nl, CALL)
#undef CALL
  return 0;
}

template <int PO, int SPAN>
static int load_sep_nl(hipStream_t s, int nb, int n, int nl, int K, const double *C, const double *gw, double *t1,
                       double *t2, double *b, double *partial) {
  const size_t P = size_t(PO) * n;
  auto grid = [](size_t count) { return int(std::min<size_t>((count + 255) / 256, 65536)); };
  const int g1 = grid(size_t(nb) * n * n * P), g2 = grid(size_t(nb) * n * P * P);
#define CALL(NL)                                                                                         \
  hipLaunchKernelGGL((k_load_sx<PO, SPAN, NL>), dim3(g1), dim3(256), 0, s, nb, n, C, gw, t1);          \
  hipLaunchKernelGGL((k_load_sy<PO, SPAN, NL>), dim3(g2), dim3(256), 0, s, nb, n, gw, t1, t2);         \
  hipLaunchKernelGGL((k_load_sz<PO, SPAN, NL>), dim3(nb * K), dim3(256), 0, s, n, K, gw, t2, b, partial)
  FEP3M_NL_SWITCH(nl, CALL)
#undef CALL
  return 0;
}

size_t load_sep_scratch(int nb, int n, int p, int nl) {
  const size_t P = size_t(p) * n;
  return size_t(nb) * n * n * P * nl * nl + size_t(nb) * n * P * P * nl;   // T1, then T2
}

int launch_load_g(hipStream_t s, int nb, int n, int p, int span, int nl, int box, const double *C, const double *gw,
                  double *b, double *partial, double *sep) {
  if (box && span != 1) return -1;   // a box holds the one-element screens only
  const int P = p * n + (box ? 1 : 0);
  const int K = seg_blocks(nb, size_t(P) * P * P);
  // separable passes through the scratch T1, T2 (one moment per element: the gather reads one value per source)
  if ((span == 3 || (span == 1 && nl > 1)) && sep && !box) {
    double *t1 = sep, *t2 = sep + size_t(nb) * n * n * size_t(P) * nl * nl;
    int r = -1;
    switch (10 * p + span) {
      case 31: r = load_sep_nl<3, 1>(s, nb, n, nl, K, C, gw, t1, t2, b, partial); break;
      case 41: r = load_sep_nl<4, 1>(s, nb, n, nl, K, C, gw, t1, t2, b, partial); break;
      case 51: r = load_sep_nl<5, 1>(s, nb, n, nl, K, C, gw, t1, t2, b, partial); break;
      case 61: r = load_sep_nl<6, 1>(s, nb, n, nl, K, C, gw, t1, t2, b, partial); break;
      case 33: r = load_sep_nl<3, 3>(s, nb, n, nl, K, C, gw, t1, t2, b, partial); break;
      case 43: r = load_sep_nl<4, 3>(s, nb, n, nl, K, C, gw, t1, t2, b, partial); break;
      case 53: r = load_sep_nl<5, 3>(s, nb, n, nl, K, C, gw, t1, t2, b, partial); break;
      case 63: r = load_sep_nl<6, 3>(s, nb, n, nl, K, C, gw, t1, t2, b, partial); break;
      default: return -1;
    }
    return r < 0 ? -1 : K;
  }
  int r = -1;
  if (span == 1) {
    switch (p) {
      case 4: r = load_g_nl<4, 1>(s, nb, n, nl, K, box, C, gw, b, partial); break;
      case 5: r = load_g_nl<5, 1>(s, nb, n, nl, K, box, C, gw, b, partial); break;
      case 6: r = load_g_nl<6, 1>(s, nb, n, nl, K, box, C, gw, b, partial); break;
      default: return -1;
    }
  } else if (span == 3) {
    switch (p) {
      case 3: r = load_g_nl<3, 3>(s, nb, n, nl, K, box, C, gw, b, partial); break;
      case 4: r = load_g_nl<4, 3>(s, nb, n, nl, K, box, C, gw, b, partial); break;
      case 5: r = load_g_nl<5, 3>(s, nb, n, nl, K, box, C, gw, b, partial); break;
      case 6: r = load_g_nl<6, 3>(s, nb, n, nl, K, box, C, gw, b, partial); break;
      default: return -1;
    }
  }
  return r < 0 ? -1 : K;
}

template <int PO>
static int psi_g_nl(hipStream_t s, int nb, int n, int nsr, int nl, int box, const double *C, const double *T,
                    const double *phi, double *W) {
  if (nsr < 1 || nsr > 3) return -1;
#define CALL(NL)                                                                                            \
  {                                                                                                         \
    using S = PsiShape<PO, NL>;                                                                             \
    const int bricks = ((n + S::BX - 1) / S::BX) * ((n + S::BY - 1) / S::BY) * ((n + S::BZ - 1) / S::BZ); \
    hipLaunchKernelGGL((k_psi_g<PO, NL>), dim3(nb * bricks), dim3(S::THREADS), 0, s, n, nsr, box, C, T,  \
                       phi, W);                                                                             \
  }
  FEP3M_NL_SWITCH(nl, CALL)
#undef CALL
  return 0;
}

int launch_psi_g(hipStream_t s, int nb, int n, int nsr, int p, int nl, int box, const double *C, const double *T,
                 const double *phi, double *W) {
  switch (p) {
    case 3: return psi_g_nl<3>(s, nb, n, nsr, nl, box, C, T, phi, W);
    case 4: return psi_g_nl<4>(s, nb, n, nsr, nl, box, C, T, phi, W);
    case 5: return psi_g_nl<5>(s, nb, n, nsr, nl, box, C, T, phi, W);
    case 6: return psi_g_nl<6>(s, nb, n, nsr, nl, box, C, T, phi, W);
    default: return -1;
  }
}

template <int PO, int NL>
static void adj_near_launch(hipStream_t s, int nb, int n, int nsr, int box, const double *gE, const double *Tt,
                            double *A) {
  if (launch_adj_near_mfma(s, nb, n, nsr, PO, NL, box, gE, Tt, A) == 0) return;   // matrix cores
  if (NL == 2 && launch_adj_moments(s, nb, PO, n, nsr, box, gE, Tt, nullptr, nullptr, A) == 0) return;   // 8 moments
  using S = AdjNearShape<NL * NL * NL>;
  const int bricks = ((n + S::BX - 1) / S::BX) * ((n + S::BY - 1) / S::BY) * ((n + S::BZ - 1) / S::BZ);
  hipLaunchKernelGGL((k_adj_near_g<PO, NL>), dim3(nb * bricks), dim3(S::THREADS), 0, s, n, nsr, box, gE, Tt, A);
}

template <int PO, int SPAN>
static int adj_g_nl(hipStream_t s, int nb, int n, int nsr, int nl, int box, const double *gE, const double *Tt,
                    const double *lam, const double *gw, double *A, double *sep) {
  if (nsr < 1 || nsr > 3) return -1;
  const int MT = nb * n * n * n;
  if (sep && !box && (SPAN == 3 || nl > 1)) {   // separable lambda part through the load's scratch
    const size_t P = size_t(PO) * n;
    double *u2 = sep, *u1 = sep + size_t(nb) * n * n * P * nl * nl;
    const int gz = grid_for_count(int64_t(nb) * n * P * P), gy = grid_for_count(int64_t(nb) * n * n * P);
    const int gx = grid_for_count(int64_t(MT) * nl * nl);
#define CALL(NL)                                                                                  \
  adj_near_launch<PO, NL>(s, nb, n, nsr, box, gE, Tt, A);                                         \
  hipLaunchKernelGGL((k_adjl_z<PO, SPAN, NL>), dim3(gz), dim3(256), 0, s, nb, n, lam, gw, u1);   \
  hipLaunchKernelGGL((k_adjl_y<PO, SPAN, NL>), dim3(gy), dim3(256), 0, s, nb, n, gw, u1, u2);    \
  hipLaunchKernelGGL((k_adjl_x<PO, SPAN, NL>), dim3(gx), dim3(256), 0, s, nb, n, gw, u2, A)
    FEP3M_NL_SWITCH(nl, CALL)
#undef CALL
    return 0;
  }
  const int g = grid_for_count(int64_t(MT) * nl * nl * nl);
#define CALL(NL)                                             \
  adj_near_launch<PO, NL>(s, nb, n, nsr, box, gE, Tt, A); \
  hipLaunchKernelGGL((k_adj_lam_g<PO, SPAN, NL>), dim3(g), dim3(256), 0, s, n, MT, box, lam, gw, A)
  FEP3M_NL_SWITCH(nl, CALL)
#undef CALL
  return 0;
}

int launch_adj_g(hipStream_t s, int nb, int n, int nsr, int p, int span, int nl, int box, const double *gE,
                 const double *T, const double *lam, const double *gw, double *A, double *sep) {
  if (box && span != 1) return -1;
  if (span == 1) {
    switch (p) {
      case 4: return adj_g_nl<4, 1>(s, nb, n, nsr, nl, box, gE, T, lam, gw, A, sep);
      case 5: return adj_g_nl<5, 1>(s, nb, n, nsr, nl, box, gE, T, lam, gw, A, sep);
      case 6: return adj_g_nl<6, 1>(s, nb, n, nsr, nl, box, gE, T, lam, gw, A, sep);
      default: return -1;
    }
  }
  if (span == 3) {
    switch (p) {
      case 3: return adj_g_nl<3, 3>(s, nb, n, nsr, nl, box, gE, T, lam, gw, A, sep);
      case 4: return adj_g_nl<4, 3>(s, nb, n, nsr, nl, box, gE, T, lam, gw, A, sep);
      case 5: return adj_g_nl<5, 3>(s, nb, n, nsr, nl, box, gE, T, lam, gw, A, sep);
      case 6: return adj_g_nl<6, 3>(s, nb, n, nsr, nl, box, gE, T, lam, gw, A, sep);
      default: return -1;
    }
  }
  return -1;
}

#undef FEP3M_NL_SWITCH

}  // namespace fep3m
