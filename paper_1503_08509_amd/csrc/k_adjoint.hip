// Adjoint (reverse) pass of the discrete energy U = 1/2 sum Q_i Phi_i:
// forces F = -dU/dx and dU/dQ.  In element units (g = x / h, U_hat = h U):
//
//   g_E[m]   = sum_{i in E} Q_i u_m(u_i)                    (charge deposit)
//   G        = assembled g; lambda = gauge(K^+ compat(G))   (second mesh solve)
//   A[E][a]  = 4 pi <lambda_E, G_a> - sum_D <g_{E+D}, T_a[D]>
//   dU_hat/dg_i = Q_i sum_j Q_j (g_j - g_i)/r^3              (pair part)
//               + 1/2 Q_i [ sum_m W_E[m] grad u_m(u_i) + sum_a A[E][a] grad u^a ]
//   dU_hat/dQ_i = Phi_p + 1/2 Phi_m + 1/2 sum_a A[E][a] u_i^a
//
// with W_E = phi_E - Psi_E from the forward pass; F = -(1/h^2) dU_hat/dg.
// The operators are not symmetric (the paper notes the lack of exact
// momentum conservation), so dU/dQ differs from Phi.
#include "kernels.hpp"

namespace fep3m {

// Fixed-shape block sum for any block of whole waves (up to 8): shuffle tree
// inside each wave, then the wave sums in order; valid in thread 0.
__device__ __forceinline__ double block_sum_waves_a(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < int(blockDim.x >> 6); ++w) r += red[w];
  return r;
}

// g_E[m] = sum over the element's charges of Q l_mx(u_x) l_my(u_y) l_mz(u_z):
// one wave (block) per element.  Charges go in chunks of 64: lane j
// evaluates the 3 (p+1) one-dimensional basis values of charge j of the
// chunk once (Q folded into the x factor) into LDS (rows padded to 65: no
// bank conflicts when lanes read different rows of one charge); then lane l
// accumulates its nodes m = l + 64 k from three LDS values per charge.
template <int PO>
__global__ __launch_bounds__(64) void k_deposit(int n, int MT, int64_t N, GllBasis bas, const int *__restrict__ start,
                                                const double *__restrict__ sg, const double *__restrict__ sQ,
                                                double *__restrict__ gE) {
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1, NK = (NM + 63) / 64;
  __shared__ double Lb[3 * Q1][65];   // [axis * (p+1) + a][charge of the chunk]
  const int E = blockIdx.x;           // element of the whole batch
  const int lane = threadIdx.x;
  const int El = E % (n * n * n);
  const int ex = El % n, ey = (El / n) % n, ez = El / (n * n);
  int ix[NK], iy[NK], iz[NK];
  double acc[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int m = min(lane + 64 * k, NM - 1);
    ix[k] = m % Q1; iy[k] = Q1 + (m / Q1) % Q1; iz[k] = 2 * Q1 + m / (Q1 * Q1);
    acc[k] = 0.0;
  }
  const int s0 = start[E], s1 = start[E + 1];
  for (int c0 = s0; c0 < s1; c0 += 64) {
    const int cnt = min(64, s1 - c0);
    __syncthreads();   // the previous chunk's values are no longer read
    if (lane < cnt) {
      const int s = c0 + lane;
      const double u[3] = {sg[s] - ex - 0.5, sg[N + s] - ey - 0.5, sg[2 * N + s] - ez - 0.5};
      const double q = sQ[s];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
#pragma unroll
        for (int a = 0; a < Q1; ++a) {
          double v = bas.w[a];
#pragma unroll
          for (int j = 0; j < Q1; ++j)
            if (j != a) v *= u[ax] - bas.x[j];
          Lb[ax * Q1 + a][lane] = ax == 0 ? q * v : v;
        }
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j)
#pragma unroll
      for (int k = 0; k < NK; ++k) acc[k] += Lb[ix[k]][j] * Lb[iy[k]][j] * Lb[iz[k]][j];
  }
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int m = lane + 64 * k;
    if (m < NM) gE[size_t(E) * NM + m] = acc[k];
  }
}

// G at each global node: sum of the owning elements' g values (gather form),
// with per-configuration block partials (K blocks per configuration) of
// sum G for the compatibility projection.
template <int PO>
__global__ __launch_bounds__(512) void k_assemble(int n, int K, const double *__restrict__ gEall,
                                                  double *__restrict__ Gall, double *__restrict__ partial) {
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1;
  __shared__ double red[8];
  const int P = PO * n;
  const size_t total = size_t(P) * P * P;
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const double *gE = gEall + size_t(cfg) * n * n * n * NM;
  double *G = Gall + size_t(cfg) * total;
  double acc = 0.0;
  (void)total;
  auto owners = [n](int g, int (&e)[2], int (&k)[2]) {   // one owner, or two at a vertex (element below first)
    e[0] = g / PO;
    k[0] = g - e[0] * PO;
    if (k[0] != 0) return 1;
    e[1] = e[0] == 0 ? n - 1 : e[0] - 1;
    k[1] = PO;
    return 2;
  };
  for (int row = kb; row < P * P; row += K) {   // one (gz, gy) row per pass, x along the threads
    const int gz = row / P, gy = row - gz * P;
    int ey[2], ky[2], ez[2], kz[2];
    const int ny = owners(gy, ey, ky), nz = owners(gz, ez, kz);
    for (int gx = threadIdx.x; gx < P; gx += blockDim.x) {
    const size_t g = size_t(row) * P + gx;
    int ex[2], kx[2];
    const int nx = owners(gx, ex, kx);
    double s = 0.0;
    for (int iz = 0; iz < nz; ++iz)
      for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
          const size_t E = size_t(ex[ix]) + size_t(n) * (ey[iy] + size_t(n) * ez[iz]);
          s += gE[E * NM + (kz[iz] * Q1 + ky[iy]) * Q1 + kx[ix]];
        }
    G[g] = s;
    acc += s;
    }
  }
  double t = block_sum_waves_a(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// A[E][a] = 4 pi <lambda_E, G_a> - sum_D <g_{E+D}, T_a[D]>.
// The second term is the transpose of the near-screen field: per element a
// contraction over (D, m) with only 8 outputs, so the reduction over nodes m
// is split across lanes:
//   block  = an 8 x 4 x 4 brick of target elements, 256 threads,
//   thread = the 8 elements of one x-row of the brick x 4 of the 8 moments
//            (32 float64 accumulators) for one lane of an 8-node chunk,
//   phase  = one (D_z, node chunk): the deposits g of the source slab and the
//            tables of the 49 offsets of that D_z (transposed copy
//            Tt[D][m][a], the chunk's nodes) are staged in LDS, the next
//            phase's deposits already in flight into registers; per D_y a thread
//            loads the 2 NSR + 8 sources its row sees into registers once
//            and slides over D_x,
//   the 8 node lanes are reduced with shuffles at the end.
// v mod n for v in [-n, 3n), without an integer division (n is a run-time
// value, so v % n would cost a full division sequence per use).
__device__ __forceinline__ int wrap3(int v, int n) {
  v += v < 0 ? n : 0;
  v -= v >= n ? n : 0;
  v -= v >= n ? n : 0;
  return v;
}

template <int NSR, int PO>
__global__ __launch_bounds__(256, 2) void k_adj_moments(int n, int box, const double *__restrict__ gE,
                                                     const double *__restrict__ Tt, const double *__restrict__ lam,
                                                     const double *__restrict__ gw, double *__restrict__ Aout) {
  constexpr int BX = 8, BY = 4, BZ = 4;
  constexpr int HX = BX + 2 * NSR, HY = BY + 2 * NSR, S = 2 * NSR + 1;
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1;
  constexpr int MC = 8, MS = MC + 1;             // nodes per chunk, padded stride
  constexpr int NCH = (NM + MC - 1) / MC;
  constexpr int SLAB = BZ * HY * HX;             // source elements of one D_z
  constexpr int AH = 4;                          // moments per thread
  constexpr int TS = S * S * MC * 8;             // staged table values per phase
  static_assert(MC * BY * BZ * (8 / AH) == 256, "thread map");
  static_assert(BX * BY * BZ * 8 <= SLAB * MS, "reduction reuses the slab");
  __shared__ double Gs[SLAB * MS];               // [lz][hy][hx][m]
  __shared__ __align__(16) double Ts[TS];        // [D_y D_x][m][a]
  const int bx_n = (n + BX - 1) / BX, by_n = (n + BY - 1) / BY, bz_n = (n + BZ - 1) / BZ;
  {  // configuration of this brick
    const int cfg = blockIdx.x / (bx_n * by_n * bz_n);
    const size_t M = size_t(n) * n * n, P = size_t(PO) * n + (box ? 1 : 0);
    gE += size_t(cfg) * M * NM;
    lam += size_t(cfg) * P * P * P;
    Aout += size_t(cfg) * M * 8;
  }
  int b = blockIdx.x % (bx_n * by_n * bz_n);
  const int bx = b % bx_n;
  b /= bx_n;
  const int by = b % by_n;
  const int bz = b / by_n;
  const int x0 = bx * BX, y0 = by * BY, z0 = bz * BZ;
  const int tid = threadIdx.x;
  const int ml = tid % MC, ah = (tid / MC) & 1, row = tid / (2 * MC);
  const int ly = row % BY, lz = row / BY;
  double acc[BX][AH];
#pragma unroll
  for (int e = 0; e < BX; ++e)
#pragma unroll
    for (int a = 0; a < AH; ++a) acc[e][a] = 0.0;

  // Phases (D_z, node chunk) are software-pipelined: the next phase's
  // deposits and tables are fetched into registers while this one computes.
  constexpr int NPH = S * NCH;
  constexpr int GPF = (MC * SLAB + 255) / 256;
  double gpf[GPF];
  auto fetch = [&](int ph) {
    const int Dz = ph / NCH - NSR, ch = ph % NCH;
#pragma unroll
    for (int r = 0; r < GPF; ++r) {   // lanes walk nodes: contiguous loads
      const int i = tid + 256 * r;
      const int mm = i % MC, h = i / MC;
      const int m = ch * MC + mm;
      const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
      const int sx = x0 - NSR + hx, sy = y0 - NSR + hy, sz = z0 + hz + Dz;
      const bool in = sx >= 0 && sx < n && sy >= 0 && sy < n && sz >= 0 && sz < n;   // box: no source outside
      const int ex = wrap3(sx, n), ey = wrap3(sy, n), ez = wrap3(sz, n);
      gpf[r] = (i < MC * SLAB && m < NM && (in || !box)) ? gE[(size_t(ex) + size_t(n) * (ey + size_t(n) * ez)) * NM + m]
                                                        : 0.0;
    }
  };
  fetch(0);
  for (int ph = 0; ph < NPH; ++ph) {
    {
      __syncthreads();   // the previous phase is done with the LDS slabs
#pragma unroll
      for (int r = 0; r < GPF; ++r) {
        const int i = tid + 256 * r;
        if (i < MC * SLAB) Gs[(i / MC) * MS + i % MC] = gpf[r];
      }
      {   // tables of this phase (shared by every block: L2-resident)
        const int Dz = ph / NCH - NSR, ch = ph % NCH;
        for (int i = tid; i < TS; i += 256) {   // 64 contiguous values per offset
          const int a = i % 8, mm = (i / 8) % MC, dyx = i / (8 * MC);
          const int m = ch * MC + mm;
          Ts[i] = m < NM ? Tt[(size_t(dyx + S * S * (Dz + NSR)) * NM + m) * 8 + a] : 0.0;
        }
      }
      __syncthreads();
      if (ph + 1 < NPH) fetch(ph + 1);
#pragma unroll 1
      for (int Dy = -NSR; Dy <= NSR; ++Dy) {
        // the x-row of sources this thread's 8 targets see at every D_x:
        // target e, offset D_x reads window position e + D_x + NSR
        double win[HX];
        const double *gr = Gs + ((lz * HY + (ly + Dy + NSR)) * HX) * MS + ml;
#pragma unroll
        for (int hx = 0; hx < HX; ++hx) win[hx] = gr[hx * MS];
#pragma unroll
        for (int Dx = -NSR; Dx <= NSR; ++Dx) {
          const int dyx = (Dx + NSR) + S * (Dy + NSR);
          const double *tp = Ts + (dyx * MC + ml) * 8 + ah * AH;
          double tv[AH];
#pragma unroll
          for (int a = 0; a < AH; ++a) tv[a] = tp[a];
#pragma unroll
          for (int e = 0; e < BX; ++e) {
            const double gv = win[e + Dx + NSR];
#pragma unroll
            for (int a = 0; a < AH; ++a) acc[e][a] += tv[a] * gv;
          }
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < BX; ++e)
#pragma unroll
    for (int a = 0; a < AH; ++a) {
      double v = acc[e][a];
      for (int off = MC / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      acc[e][a] = v;
    }
  __syncthreads();
  double *red = Gs;  // [BX BY BZ elements][8 moments], element = lx + BX (ly + BY lz)
  if (ml == 0) {
#pragma unroll
    for (int e = 0; e < BX; ++e)
#pragma unroll
      for (int a = 0; a < AH; ++a) red[(e + BX * row) * 8 + ah * AH + a] = acc[e][a];
  }
  __syncthreads();
  if (tid >= BX * BY * BZ) return;
  const int ex = x0 + tid % BX, ey = y0 + (tid / BX) % BY, ez = z0 + tid / (BX * BY);
  if (ex >= n || ey >= n || ez >= n) return;
  if (!lam) {   // the near part alone (screens whose mesh part spans more elements add it after)
    const size_t E = size_t(ex) + size_t(n) * (ey + size_t(n) * ez);
#pragma unroll
    for (int a = 0; a < 8; ++a) Aout[E * 8 + a] = -red[tid * 8 + a];
    return;
  }
  const int P = PO * n + (box ? 1 : 0);   // box: (PO n + 1)^3 nodes, no index leaves it
  double a1[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int mm = 0; mm < NM; ++mm) {
    const int mx = mm % Q1, my = (mm / Q1) % Q1, mz = mm / (Q1 * Q1);
    const int gx = wrap3(PO * ex + mx, P), gy = wrap3(PO * ey + my, P), gz = wrap3(PO * ez + mz, P);
    const double lv = lam[(size_t(gz) * P + gy) * P + gx];
    const double gx0 = gw[mx], gx1 = gw[Q1 + mx], gy0 = gw[my], gy1 = gw[Q1 + my], gz0 = gw[mz], gz1 = gw[Q1 + mz];
    a1[0] += lv * gx0 * gy0 * gz0;
    a1[1] += lv * gx1 * gy0 * gz0;
    a1[2] += lv * gx0 * gy1 * gz0;
    a1[3] += lv * gx1 * gy1 * gz0;
    a1[4] += lv * gx0 * gy0 * gz1;
    a1[5] += lv * gx1 * gy0 * gz1;
    a1[6] += lv * gx0 * gy1 * gz1;
    a1[7] += lv * gx1 * gy1 * gz1;
  }
  const size_t E = size_t(ex) + size_t(n) * (ey + size_t(n) * ez);
#pragma unroll
  for (int a = 0; a < 8; ++a) Aout[E * 8 + a] = 4.0 * M_PI * a1[a] - red[tid * 8 + a];
}

// Forces and dU/dQ per sorted charge, scattered to caller order.
template <int PO, int NL, class WT>
__global__ __launch_bounds__(256) void k_forces(int n, int64_t N, int nb, const int *__restrict__ off, double inv_h,
                                                GllBasis bas,
                                                const double *__restrict__ sg, const double *__restrict__ sQ,
                                                const WT *__restrict__ Wel, const double *__restrict__ Aadj,
                                                const double *__restrict__ fpair, const double *__restrict__ phip,
                                                const double *__restrict__ phim_s, const int *__restrict__ perm,
                                                double *__restrict__ F, double *__restrict__ dUdQ) {
  constexpr int Q1 = PO + 1;
  for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < N; s += int64_t(gridDim.x) * blockDim.x) {
    double l[3][Q1], dl[3][Q1], u[3];
    int e[3];
    for (int k = 0; k < 3; ++k) {
      const double g = sg[k * N + s];
      double ef = floor(g);
      if (ef > double(n - 1)) ef = double(n - 1);
      e[k] = int(ef);
      u[k] = g - ef - 0.5;
#pragma unroll
      for (int a = 0; a < Q1; ++a) {
        double v = bas.w[a], dv = 0.0;
#pragma unroll
        for (int j = 0; j < Q1; ++j) {
          if (j == a) continue;
          dv = dv * (u[k] - bas.x[j]) + v;   // product rule, running
          v *= (u[k] - bas.x[j]);
        }
        l[k][a] = v;
        dl[k][a] = dv;
      }
    }
    const size_t E = size_t(cfg_of(off, nb, s)) * n * n * n + size_t(e[0]) + size_t(n) * (e[1] + size_t(n) * e[2]);
    const WT *w = Wel + E * (Q1 * Q1 * Q1);
    double gxs = 0.0, gys = 0.0, gzs = 0.0;
#pragma unroll
    for (int mz = 0; mz < Q1; ++mz) {
      double sy_ll = 0.0, sy_dl = 0.0, sy_ld = 0.0;
#pragma unroll
      for (int my = 0; my < Q1; ++my) {
        double rl = 0.0, rd = 0.0;
#pragma unroll
        for (int mx = 0; mx < Q1; ++mx) {
          const double wv = double(w[(mz * Q1 + my) * Q1 + mx]);
          rl += l[0][mx] * wv;
          rd += dl[0][mx] * wv;
        }
        sy_ll += l[1][my] * rl;   // x value, y value
        sy_dl += l[1][my] * rd;   // x deriv, y value
        sy_ld += dl[1][my] * rl;  // x value, y deriv
      }
      gxs += l[2][mz] * sy_dl;
      gys += l[2][mz] * sy_ld;
      gzs += dl[2][mz] * sy_ll;
    }
    constexpr int NA = NL * NL * NL;
    const double *A = Aadj + E * NA;
    const double ux = u[0], uy = u[1], uz = u[2];
    double ax, ay, az, au;
    if constexpr (NL == 2) {
      // grad of u^a, a = ax + 2 ay + 4 az, each exponent 0 or 1
      ax = A[1] + A[3] * uy + A[5] * uz + A[7] * uy * uz;
      ay = A[2] + A[3] * ux + A[6] * uz + A[7] * ux * uz;
      az = A[4] + A[5] * ux + A[6] * uy + A[7] * ux * uy;
      au = A[0] + A[1] * ux + A[2] * uy + A[3] * ux * uy + A[4] * uz + A[5] * ux * uz + A[6] * uy * uz +
           A[7] * ux * uy * uz;
    } else {
      // powers u^k and their derivatives k u^(k-1) per axis, a = ax + NL ay + NL^2 az
      double pw[3][NL], dp[3][NL];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        pw[k][0] = 1.0;
        dp[k][0] = 0.0;
#pragma unroll
        for (int j = 1; j < NL; ++j) {
          pw[k][j] = pw[k][j - 1] * u[k];
          dp[k][j] = double(j) * pw[k][j - 1];
        }
      }
      ax = ay = az = au = 0.0;
      for (int kz = 0; kz < NL; ++kz)
        for (int ky = 0; ky < NL; ++ky) {
          double rv = 0.0, rd = 0.0;
          for (int kx = 0; kx < NL; ++kx) {
            const double c = A[(kz * NL + ky) * NL + kx];
            rv += c * pw[0][kx];
            rd += c * dp[0][kx];
          }
          au += pw[2][kz] * pw[1][ky] * rv;
          ax += pw[2][kz] * pw[1][ky] * rd;
          ay += pw[2][kz] * dp[1][ky] * rv;
          az += dp[2][kz] * pw[1][ky] * rv;
        }
    }
    const double q = sQ[s];
    const double s2 = inv_h * inv_h;
    const int i = perm[s];
    if (F) {
      F[3 * size_t(i) + 0] = -s2 * (q * fpair[s] + 0.5 * q * (gxs + ax));
      F[3 * size_t(i) + 1] = -s2 * (q * fpair[N + s] + 0.5 * q * (gys + ay));
      F[3 * size_t(i) + 2] = -s2 * (q * fpair[2 * N + s] + 0.5 * q * (gzs + az));
    }
    if (dUdQ) dUdQ[i] = inv_h * phip[s] + 0.5 * phim_s[s] + 0.5 * inv_h * au;
  }
}

// ----------------------------------------------------------------- launchers

int launch_deposit(hipStream_t s, int nb, int p, int n, int64_t N, const GllBasis &bas, const int *start,
                   const double *sg, const double *sQ, double *gE) {
  const int MT = nb * n * n * n;
  switch (p) {
    case 3: hipLaunchKernelGGL(k_deposit<3>, dim3(MT), dim3(64), 0, s, n, MT, N, bas, start, sg, sQ, gE); return 0;
    case 4: hipLaunchKernelGGL(k_deposit<4>, dim3(MT), dim3(64), 0, s, n, MT, N, bas, start, sg, sQ, gE); return 0;
    case 5: hipLaunchKernelGGL(k_deposit<5>, dim3(MT), dim3(64), 0, s, n, MT, N, bas, start, sg, sQ, gE); return 0;
    case 6: hipLaunchKernelGGL(k_deposit<6>, dim3(MT), dim3(64), 0, s, n, MT, N, bas, start, sg, sQ, gE); return 0;
    default: return -1;
  }
}
int launch_assemble(hipStream_t s, int nb, int p, int n, const double *gE, double *G, double *partial) {
  const int K = row_blocks(nb, p * n);
  const dim3 g(nb * K), b(row_threads(p * n));
  switch (p) {
    case 3: hipLaunchKernelGGL(k_assemble<3>, g, b, 0, s, n, K, gE, G, partial); return K;
    case 4: hipLaunchKernelGGL(k_assemble<4>, g, b, 0, s, n, K, gE, G, partial); return K;
    case 5: hipLaunchKernelGGL(k_assemble<5>, g, b, 0, s, n, K, gE, G, partial); return K;
    case 6: hipLaunchKernelGGL(k_assemble<6>, g, b, 0, s, n, K, gE, G, partial); return K;
    default: return -1;
  }
}
int launch_adj_moments(hipStream_t s, int nb, int p, int n, int nsr, int box, const double *gE, const double *Tt,
                       const double *lam, const double *gw, double *A) {
  if (p == 3) {   // 27-element q = 1 (8 moments, order 3): the near part alone
    if (lam) return -1;
    const int bxn = (n + 7) / 8, byn = (n + 3) / 4, bzn = (n + 3) / 4;
    dim3 g(nb * bxn * byn * bzn);
    switch (nsr) {
      case 1: hipLaunchKernelGGL((k_adj_moments<1, 3>), g, dim3(256), 0, s, n, box, gE, Tt, lam, gw, A); return 0;
      case 2: hipLaunchKernelGGL((k_adj_moments<2, 3>), g, dim3(256), 0, s, n, box, gE, Tt, lam, gw, A); return 0;
      case 3: hipLaunchKernelGGL((k_adj_moments<3, 3>), g, dim3(256), 0, s, n, box, gE, Tt, lam, gw, A); return 0;
      default: return -1;
    }
  }
  if (p != 5) return -1;
  const int bxn = (n + 7) / 8, byn = (n + 3) / 4, bzn = (n + 3) / 4;
  dim3 g(nb * bxn * byn * bzn);
  switch (nsr) {
    case 1: hipLaunchKernelGGL((k_adj_moments<1, 5>), g, dim3(256), 0, s, n, box, gE, Tt, lam, gw, A); return 0;
    case 2: hipLaunchKernelGGL((k_adj_moments<2, 5>), g, dim3(256), 0, s, n, box, gE, Tt, lam, gw, A); return 0;
    case 3: hipLaunchKernelGGL((k_adj_moments<3, 5>), g, dim3(256), 0, s, n, box, gE, Tt, lam, gw, A); return 0;
    default: return -1;
  }
}
template <class WT>
int launch_forces(hipStream_t s, int nb, const int *off, int p, int n, int nl, int64_t N, double inv_h,
                  const GllBasis &bas, const double *sg, const double *sQ, const WT *Wel, const double *A,
                  const double *fpair, const double *phip, const double *phim_s, const int *perm, double *F,
                  double *dUdQ) {
  int64_t gb = (N + 255) / 256;
  if (gb > 4096) gb = 4096;
#define CALL(PO, NL)                                                                                                \
  hipLaunchKernelGGL((k_forces<PO, NL, WT>), dim3(int(gb)), dim3(256), 0, s, n, N, nb, off, inv_h, bas, sg, sQ, Wel, \
                     A, fpair, phip, phim_s, perm, F, dUdQ)
  const int key = 10 * p + nl;   // the screen families: (p, nl) = (5, 2) and q + 2 with q - 1 or q + 1
  switch (key) {
    case 52: CALL(5, 2); return 0;
    case 32: CALL(3, 2); return 0;
    case 43: CALL(4, 3); return 0;
    case 54: CALL(5, 4); return 0;
    case 65: CALL(6, 5); return 0;
    case 63: CALL(6, 3); return 0;
    case 41: CALL(4, 1); return 0;
    default: return -1;
  }
#undef CALL
}
template int launch_forces<double>(hipStream_t, int, const int *, int, int, int, int64_t, double, const GllBasis &,
                                   const double *, const double *, const double *, const double *, const double *,
                                   const double *, const double *, const int *, double *, double *);
template int launch_forces<float>(hipStream_t, int, const int *, int, int, int, int64_t, double, const GllBasis &,
                                  const double *, const double *, const float *, const double *, const double *,
                                  const double *, const double *, const int *, double *, double *);

}  // namespace fep3m
