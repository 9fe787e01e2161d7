// Near-screen field (element-to-point evaluation of Section 3, eq. sc with
// the Remark's order-p tables):
//
//   Psi_E[m] = sum_{D in [-NSR, NSR]^3} sum_a T[a][D][m] C[E - D][a]
//
// the potential, at the order-p nodes m of target element E, of the combined
// screens of every element in E's near block (D = 0 is the self term).  The
// kernel writes W_E = phi_E - Psi_E, the field the charges of E interpolate.
//
// Work decomposition (a dense contraction over (D, a) with an implicit,
// gathered left operand):
//   block  = a 4 x 4 x 4 brick of target elements,
//   thread = 8 target elements (a 2 x 2 x 2 sub-brick) x 8 nodes m, held as
//            64 float64 accumulators; 216 of 256 threads compute,
//   tables T[.][D][.] (8 x 216 values per offset) stream through a double
//            LDS buffer, prefetched one offset ahead into registers, one
//            barrier per offset; every table value fetched from L2 serves the
//            brick's 64 elements,
//   moments C of the source elements sit in LDS as one z-slab per D_z.
//
// The arithmetic type T is double, or float for the mixed-precision path:
// then the tables and moments are float32, each D_z slab (8 (2 NSR + 1)^2
// products per output) is summed into a float32 partial, and the seven slab
// partials are added with Kahan compensation; phi stays float64 and W is
// written as float32.
#include <type_traits>

#include "kernels.hpp"

namespace fep3m {

template <int NSR, int PO, class T>
__global__ __launch_bounds__(256, 2) void k_psi(int n, const double *__restrict__ C, const T *__restrict__ Tab,
                                             const double *__restrict__ phi, T *__restrict__ Wel) {
  constexpr bool kComp = std::is_same<T, float>::value;   // compensated slab sums
  constexpr int BS = 4;                       // brick edge (elements)
  constexpr int H = BS + 2 * NSR;             // halo edge in x and y
  constexpr int S = 2 * NSR + 1;
  constexpr int ND = S * S * S;
  constexpr int Q1 = PO + 1;
  constexpr int NM = Q1 * Q1 * Q1;            // nodes per element (216 for p = 5)
  constexpr int MT = 8;                       // nodes per thread
  constexpr int NGM = NM / MT;                // node groups
  constexpr int NTHR = 8 * NGM;               // computing threads
  constexpr int TV = 8 * NM;                  // table values per offset
  constexpr int TPF = (TV + 255) / 256;       // prefetch registers per thread
  constexpr int SLAB = BS * H * H;            // one z-slab of the halo
  static_assert(NM % MT == 0 && NTHR <= 256, "thread tile");
  __shared__ __align__(16) T Ts[2][TV];
  __shared__ __align__(16) T Cs[8 * SLAB];

  const int bricks = (n + BS - 1) / BS;
  const int lin = xcd_linear(blockIdx.x, gridDim.x);
  {  // configuration of this brick
    const int cfg = lin / (bricks * bricks * bricks);
    const size_t M = size_t(n) * n * n, P = size_t(PO) * n;
    C += size_t(cfg) * M * 8;
    phi += size_t(cfg) * P * P * P;
    Wel += size_t(cfg) * M * NM;
  }
  int b = lin % (bricks * bricks * bricks);
  const int bx = b % bricks;
  b /= bricks;
  const int by = b % bricks;
  const int bz = b / bricks;
  const int x0 = bx * BS, y0 = by * BS, z0 = bz * BS;
  const int tid = threadIdx.x;
  const bool comp = tid < NTHR;
  const int ge = tid % 8, gm = tid / 8;
  const int ex0 = 2 * (ge & 1), ey0 = 2 * ((ge >> 1) & 1), ez0 = 2 * (ge >> 2);
  const int m0 = gm * MT;

  T acc[8][MT];                       // slab partial (float) or the whole sum (double)
  T tot[kComp ? 8 : 1][MT], cmp[kComp ? 8 : 1][MT];   // Kahan total and compensation (float)
#pragma unroll
  for (int e = 0; e < 8; ++e)
#pragma unroll
    for (int j = 0; j < MT; ++j) {
      acc[e][j] = T(0);
      if (kComp) { tot[e][j] = T(0); cmp[e][j] = T(0); }
    }

  // table values of offset 0 into buffer 0
  for (int i = tid; i < TV; i += 256) {
    const int a = i / NM, m = i % NM;
    Ts[0][i] = Tab[(size_t(a) * ND + 0) * NM + m];
  }
  int iD = 0;
  for (int Dz = -NSR; Dz <= NSR; ++Dz) {
    // stage the moments of the source slab for this D_z: target layer lz
    // reads halo layer lz - Dz + NSR
    __syncthreads();
    for (int h = tid; h < SLAB; h += 256) {
      const int hx = h % H, hy = (h / H) % H, lz = h / (H * H);
      const int ex = (x0 - NSR + hx + 2 * n) % n, ey = (y0 - NSR + hy + 2 * n) % n;
      const int ez = (z0 + lz - Dz + 2 * n) % n;
      const double *c = C + (size_t(ex) + size_t(n) * (ey + size_t(n) * ez)) * 8;
#pragma unroll
      for (int a = 0; a < 8; ++a) Cs[a * SLAB + h] = T(c[a]);
    }
    __syncthreads();
    for (int Dyx = 0; Dyx < S * S; ++Dyx, ++iD) {
      const int Dx = Dyx % S - NSR, Dy = Dyx / S - NSR;
      const int cur = iD & 1;
      // prefetch the next offset's tables into registers
      T tp[TPF];
      const bool more = iD + 1 < ND;
      if (more) {
#pragma unroll
        for (int r = 0; r < TPF; ++r) {
          const int i = tid + 256 * r;
          if (i < TV) {
            const int a = i / NM, m = i % NM;
            tp[r] = Tab[(size_t(a) * ND + iD + 1) * NM + m];
          }
        }
      }
      if (comp) {
        const T *tb = Ts[cur];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          T tv[MT];
#pragma unroll
          for (int j = 0; j < MT; ++j) tv[j] = tb[a * NM + m0 + j];
          T cv[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int lx = ex0 + (e & 1), ly = ey0 + ((e >> 1) & 1), lz = ez0 + (e >> 2);
            cv[e] = Cs[a * SLAB + (lz * H + (ly - Dy + NSR)) * H + (lx - Dx + NSR)];
          }
#pragma unroll
          for (int e = 0; e < 8; ++e)
#pragma unroll
            for (int j = 0; j < MT; ++j) acc[e][j] += tv[j] * cv[e];
        }
      }
      if (more) {
#pragma unroll
        for (int r = 0; r < TPF; ++r) {
          const int i = tid + 256 * r;
          if (i < TV) Ts[cur ^ 1][i] = tp[r];
        }
      }
      __syncthreads();
    }
    if (kComp) {   // fold this slab's partial into the compensated total
#pragma unroll
      for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int j = 0; j < MT; ++j) {
          const T y = acc[e][j] - cmp[e][j];
          const T t = tot[e][j] + y;
          cmp[e][j] = (t - tot[e][j]) - y;
          tot[e][j] = t;
          acc[e][j] = T(0);
        }
    }
  }
  if (!comp) return;
  const int P = PO * n;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int ex = x0 + ex0 + (e & 1), ey = y0 + ey0 + ((e >> 1) & 1), ez = z0 + ez0 + (e >> 2);
    if (ex >= n || ey >= n || ez >= n) continue;
    const size_t E = size_t(ex) + size_t(n) * (ey + size_t(n) * ez);
#pragma unroll
    for (int j = 0; j < MT; ++j) {
      const int m = m0 + j;
      const int mx = m % Q1, my = (m / Q1) % Q1, mz = m / (Q1 * Q1);
      const int gx = (PO * ex + mx) % P, gy = (PO * ey + my) % P, gz = (PO * ez + mz) % P;
      const double psi = kComp ? double(tot[e][j]) - double(cmp[e][j]) : double(acc[e][j]);
      Wel[E * NM + m] = T(phi[(size_t(gz) * P + gy) * P + gx] - psi);
    }
  }
}

template <class T>
int launch_psi(hipStream_t s, int nb, int n, int nsr, int p, const double *C, const T *Tab, const double *phi, T *Wel) {
  if (p != 5) return -1;
  const int bricks = (n + 3) / 4;
  dim3 g(nb * bricks * bricks * bricks);
  switch (nsr) {
    case 1: hipLaunchKernelGGL((k_psi<1, 5, T>), g, dim3(256), 0, s, n, C, Tab, phi, Wel); return 0;
    case 2: hipLaunchKernelGGL((k_psi<2, 5, T>), g, dim3(256), 0, s, n, C, Tab, phi, Wel); return 0;
    case 3: hipLaunchKernelGGL((k_psi<3, 5, T>), g, dim3(256), 0, s, n, C, Tab, phi, Wel); return 0;
    default: return -1;
  }
}
template int launch_psi<double>(hipStream_t, int, int, int, int, const double *, const double *, const double *,
                                double *);
template int launch_psi<float>(hipStream_t, int, int, int, int, const double *, const float *, const double *,
                               float *);

}  // namespace fep3m
