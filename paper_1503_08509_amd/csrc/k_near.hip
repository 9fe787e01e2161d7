// Near-screen field (element-to-point evaluation of Section 3, eq. sc with
// the Remark's order-p tables):
//
//   Psi_E[m] = sum_{D in [-NSR, NSR]^3} sum_a T[a][D][m] C[E - D][a]
//
// the potential, at the order-p nodes m of target element E, of the combined
// screens of every element in E's near block (D = 0 is the self term).  The
// kernel writes W_E = phi_E - Psi_E, the field the charges of E interpolate.
//
// This is a dense contraction over k = (D, a) (343 x 8 terms) with a
// gathered left operand, run on the matrix cores:
//   block  = a 4 x 4 x 8 brick of target elements, 8 waves,
//   wave   = two 4 x 4 element layers (two 16-row tiles) x 7 of the 14
//            16-node tiles, 14 accumulator tiles of 16 x 16,
//   k-step = one offset D and four moments: one 16 x 16 x 4 MFMA per tile
//            (float64, or float32 on the mixed-precision path),
//   tables T[.][D][.] (8 x 216 values per offset, rows padded to 224 with
//            zeros) stream through a double LDS buffer, prefetched one
//            offset ahead into registers, one barrier per offset,
//   moments C of the source elements sit in LDS as one z-slab per D_z.
// On gfx950 these MFMAs round like four fused multiply-adds in k order: the
// results equal those of a sequential loop over (D, a) bit for bit (checked
// against such a loop on random operands, float64 and float32).
//
// On the mixed-precision path the tables and moments are float32, each D_z
// slab (8 (2 NSR + 1)^2 products per output) is summed into a float32
// partial, and the seven slab partials are added with Kahan compensation;
// phi stays float64 and W is written as float32.
#include <type_traits>

#include "kernels.hpp"

namespace fep3m {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 matrix-core step acc += A B: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator value v of lane l is row row(l, v),
// column l % 16.
template <class T> struct Mfma16;
template <> struct Mfma16<double> {
  using V = f64x4;
  static __device__ __forceinline__ V step(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Mfma16<float> {
  using V = f32x4;
  static __device__ __forceinline__ V step(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int kPsiBS = 4;    // brick edge in x and y (elements)
constexpr int kPsiBZ = 8;    // brick depth in z
constexpr int kPsiThreads = 64 * kPsiBZ;

// NA moments per element (8 for the default screen; the other screen
// families: 1, 8, 27 or 64), taken 8 at a time: for each chunk of 8 the
// offsets are walked again (the missing moments of the last chunk read as
// zero), with the chunk's moments of each source slab and its tables of
// each offset staged as for 8.
template <int NSR, int PO, class T, int NA = 8>
__global__ __launch_bounds__(kPsiThreads, 1) void k_psi(int n, int box, const double *__restrict__ C,
                                                        const T *__restrict__ Tab, const double *__restrict__ phi,
                                                        T *__restrict__ Wel) {
  using M = Mfma16<T>;
  using V = typename M::V;
  constexpr bool kComp = std::is_same<T, float>::value;   // compensated slab sums
  constexpr int BS = kPsiBS, BZ = kPsiBZ, NTH = kPsiThreads;
  constexpr int H = BS + 2 * NSR;             // halo edge in x and y
  constexpr int S = 2 * NSR + 1;
  constexpr int ND = S * S * S;
  constexpr int Q1 = PO + 1;
  constexpr int NM = Q1 * Q1 * Q1;            // nodes per element (216 for p = 5)
  constexpr int NT = (NM + 15) / 16;          // 16-node tiles
  constexpr int NTW = NT / 2;                 // node tiles per wave
  constexpr int NMP = NT * 16;                // padded table row
  constexpr int TV = 8 * NM;                  // table values per offset and chunk of 8 moments
  constexpr int NCH = (NA + 7) / 8;           // moment chunks
  constexpr int NST = NCH * ND;               // table stages: (chunk, offset)
  constexpr int TPF = (TV + NTH - 1) / NTH;   // prefetch registers per thread
  constexpr int SLAB = BZ * H * H;            // one z-slab of the halo
  static_assert(NT % 2 == 0 && BZ % 2 == 0, "wave tiling");
  __shared__ __align__(16) T Ts[2][8 * NMP];
  __shared__ __align__(16) T Cs[8 * SLAB];

  const int bricks = (n + BS - 1) / BS, bricksz = (n + BZ - 1) / BZ;
  const int per = bricks * bricks * bricksz;
  const int lin = xcd_linear(blockIdx.x, gridDim.x);
  {  // configuration of this brick
    const int cfg = lin / per;
    const size_t Mn = size_t(n) * n * n, P = size_t(PO) * n + (box ? 1 : 0);
    C += size_t(cfg) * Mn * NA;
    if (phi) phi += size_t(cfg) * P * P * P;
    Wel += size_t(cfg) * Mn * NM;
  }
  int b = lin % per;
  const int bx = b % bricks;
  b /= bricks;
  const int by = b % bricks;
  const int bz = b / bricks;
  const int x0 = bx * BS, y0 = by * BS, z0 = bz * BZ;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int mh = w % (BZ / 2), nh = w / (BZ / 2);   // element layers 2 mh, 2 mh + 1; node tiles nh NTW + [0, NTW)
  const int r = lane & 15, kq = lane >> 4;           // A row (element of the layer) and k (moment) of this lane
  const int alx = r & 3, aly = r >> 2;

  V acc[2 * NTW];                                    // slab partial (float) or the whole sum (double)
  V tot[kComp ? 2 * NTW : 1], cmp[kComp ? 2 * NTW : 1];   // Kahan total and compensation (float)
#pragma unroll
  for (int t = 0; t < 2 * NTW; ++t) {
    acc[t] = V{0, 0, 0, 0};
    if (kComp) { tot[t] = V{0, 0, 0, 0}; cmp[t] = V{0, 0, 0, 0}; }
  }
  for (int i = tid; i < 2 * 8 * NMP; i += NTH) (&Ts[0][0])[i] = T(0);   // padding stays zero
  __syncthreads();
  // table value i of stage st (chunk st / ND, offset st % ND); zero past the last moment
  auto table = [&](int st, int i) -> T {
    const int ch = NCH == 1 ? 0 : st / ND, iD = NCH == 1 ? st : st - ch * ND;
    const int a = ch * 8 + i / NM, m = i % NM;
    return (NA % 8 == 0 || a < NA) ? Tab[(size_t(a) * ND + iD) * NM + m] : T(0);
  };
  for (int i = tid; i < TV; i += NTH) Ts[0][(i / NM) * NMP + i % NM] = table(0, i);   // stage 0 into buffer 0
  int st = 0;
  for (int a0 = 0; a0 < NA; a0 += 8)
  for (int Dz = -NSR; Dz <= NSR; ++Dz) {
    // stage moments a0 .. a0 + 7 of the source slab for this D_z: target
    // layer lz reads halo layer lz - Dz + NSR
    __syncthreads();
    for (int h = tid; h < SLAB; h += NTH) {
      const int hx = h % H, hy = (h / H) % H, lz = h / (H * H);
      const int sx = x0 - NSR + hx, sy = y0 - NSR + hy, sz = z0 + lz - Dz;
      if (box && (sx < 0 || sx >= n || sy < 0 || sy >= n || sz < 0 || sz >= n)) {   // no source outside the box
#pragma unroll
        for (int a = 0; a < 8; ++a) Cs[a * SLAB + h] = T(0);
        continue;
      }
      const int ex = (sx + 2 * n) % n, ey = (sy + 2 * n) % n, ez = (sz + 2 * n) % n;
      const double *c = C + (size_t(ex) + size_t(n) * (ey + size_t(n) * ez)) * NA + a0;
#pragma unroll
      for (int a = 0; a < 8; ++a) Cs[a * SLAB + h] = (NA % 8 == 0 || a0 + a < NA) ? T(c[a]) : T(0);
    }
    __syncthreads();
    for (int Dyx = 0; Dyx < S * S; ++Dyx, ++st) {
      const int Dx = Dyx % S - NSR, Dy = Dyx / S - NSR;
      const int cur = st & 1;
      // prefetch the next stage's tables into registers
      T tp[TPF];
      const bool more = st + 1 < NST;
      if (more) {
#pragma unroll
        for (int q = 0; q < TPF; ++q) {
          const int i = tid + NTH * q;
          if (i < TV) tp[q] = table(st + 1, i);
        }
      }
      const T *tb = Ts[cur];
      const int cb = ((2 * mh) * H + (aly - Dy + NSR)) * H + (alx - Dx + NSR);
#pragma unroll
      for (int k0 = 0; k0 < 8; k0 += 4) {
        if (NA < 8 && k0 >= NA) break;                     // fewer than 8 moments: the zero half is skipped
        const T av0 = Cs[(k0 + kq) * SLAB + cb];           // layer 2 mh
        const T av1 = Cs[(k0 + kq) * SLAB + cb + H * H];   // layer 2 mh + 1
        const T *brow = tb + (k0 + kq) * NMP + 16 * NTW * nh + r;
        T bv[NTW];
#pragma unroll
        for (int t = 0; t < NTW; ++t) bv[t] = brow[16 * t];
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
          acc[t] = M::step(av0, bv[t], acc[t]);
          acc[NTW + t] = M::step(av1, bv[t], acc[NTW + t]);
        }
      }
      if (more) {
#pragma unroll
        for (int q = 0; q < TPF; ++q) {
          const int i = tid + NTH * q;
          if (i < TV) {
            const int a = i / NM, m = i % NM;
            Ts[cur ^ 1][a * NMP + m] = tp[q];
          }
        }
      }
      __syncthreads();
    }
    if (kComp) {   // fold this slab's partial into the compensated total
#pragma unroll
      for (int t = 0; t < 2 * NTW; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T y = acc[t][v] - cmp[t][v];
          const T s = tot[t][v] + y;
          cmp[t][v] = (s - tot[t][v]) - y;
          tot[t][v] = s;
          acc[t][v] = T(0);
        }
    }
  }
  const int P = PO * n + (box ? 1 : 0);
#pragma unroll
  for (int hh = 0; hh < 2; ++hh)
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      const int ti = hh * NTW + t;
      const int m = 16 * (NTW * nh + t) + r;
      if (m >= NM) continue;
      const int mx = m % Q1, my = (m / Q1) % Q1, mz = m / (Q1 * Q1);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int e = M::row(lane, v);
        const int ex = x0 + (e & 3), ey = y0 + (e >> 2), ez = z0 + 2 * mh + hh;
        if (ex >= n || ey >= n || ez >= n) continue;
        const size_t E = size_t(ex) + size_t(n) * (ey + size_t(n) * ez);
        const int gx = (PO * ex + mx) % P, gy = (PO * ey + my) % P, gz = (PO * ez + mz) % P;
        const double psi = kComp ? double(tot[ti][v]) - double(cmp[ti][v]) : double(acc[ti][v]);
        Wel[E * NM + m] = T((phi ? phi[(size_t(gz) * P + gy) * P + gx] : 0.0) - psi);
      }
    }
}

// Near part of the moment adjoint on the matrix cores, for the screen
// families with many moments (NA = 27, 64, 125):
//
//   A[E][a] = - sum_D sum_m g_{E+D}[m] T[a][D][m]
//
// a contraction over k = (D, m) with a gathered left operand (the deposits
// of the sources E + D) and the tables, transposed to Tt[D][m][a], on the
// right:
//   block  = a 4 x 4 x 8 brick of target elements, 4 waves,
//   wave   = two 4 x 4 element layers (two 16-row tiles) x every 16-moment
//            column tile of a (NAT = ceil(NA / 16) of them),
//   k-step = one offset D and four nodes m: one 16 x 16 x 4 float64 MFMA
//            per tile,
//   stages = (node chunk of 8, offset D): the chunk's deposits of one z-slab
//            of sources per D_z in LDS, the chunk's tables of one offset
//            (8 x NA values, contiguous in Tt) in a double LDS buffer
//            prefetched one stage ahead into registers.
// Missing nodes of the last chunk and moments past NA read as zero.
constexpr int kAdjThreads = 256;

template <int NSR, int PO, int NA>
__global__ __launch_bounds__(kAdjThreads, 2) void k_adj_mfma(int n, int box, const double *__restrict__ gE,
                                                        const double *__restrict__ Tt, double *__restrict__ Aout) {
  using M = Mfma16<double>;
  using V = typename M::V;
  constexpr int BS = kPsiBS, BZ = kPsiBZ, NTH = kAdjThreads;
  constexpr int H = BS + 2 * NSR;             // halo edge in x and y
  constexpr int S = 2 * NSR + 1, ND = S * S * S;
  constexpr int Q1 = PO + 1, NM = Q1 * Q1 * Q1;
  constexpr int NCH = (NM + 7) / 8;           // node chunks
  constexpr int NAT = (NA + 15) / 16;         // 16-moment column tiles
  constexpr int NAP = NAT * 16;               // padded table row
  constexpr int TV = 8 * NA;                  // table values per stage
  constexpr int TPF = (TV + NTH - 1) / NTH;   // prefetch registers per thread
  constexpr int SLAB = BZ * H * H;            // one z-slab of the halo
  constexpr int NST = NCH * ND;               // stages
  static_assert(BZ == 2 * (NTH / 64), "two element layers per wave");
  __shared__ __align__(16) double Ts[2][8 * NAP];
  __shared__ __align__(16) double Gs[8 * SLAB];

  const int bricks = (n + BS - 1) / BS, bricksz = (n + BZ - 1) / BZ;
  const int per = bricks * bricks * bricksz;
  const int lin = xcd_linear(blockIdx.x, gridDim.x);
  {  // configuration of this brick
    const int cfg = lin / per;
    const size_t Mn = size_t(n) * n * n;
    gE += size_t(cfg) * Mn * NM;
    Aout += size_t(cfg) * Mn * NA;
  }
  int b = lin % per;
  const int bx = b % bricks;
  b /= bricks;
  const int by = b % bricks;
  const int bz = b / bricks;
  const int x0 = bx * BS, y0 = by * BS, z0 = bz * BZ;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;   // layers 2 w, 2 w + 1
  const int r = lane & 15, kq = lane >> 4;                       // A row (element of the layer) and k (node)
  const int alx = r & 3, aly = r >> 2;

  V acc[2][NAT];
#pragma unroll
  for (int hh = 0; hh < 2; ++hh)
#pragma unroll
    for (int t = 0; t < NAT; ++t) acc[hh][t] = V{0, 0, 0, 0};
  for (int i = tid; i < 2 * 8 * NAP; i += NTH) (&Ts[0][0])[i] = 0.0;   // padding stays zero
  __syncthreads();
  // table value i of stage st (chunk st / ND, offset st % ND): Tt[D][m][a] with m = 8 chunk + i / NA
  auto table = [&](int st, int i) -> double {
    const int ch = st / ND, iD = st - ch * ND;
    const int m = ch * 8 + i / NA;
    return m < NM ? Tt[(size_t(iD) * NM + m) * NA + i % NA] : 0.0;
  };
  for (int i = tid; i < TV; i += NTH) Ts[0][(i / NA) * NAP + i % NA] = table(0, i);
  int st = 0;
  for (int m0 = 0; m0 < NM; m0 += 8)
  for (int Dz = -NSR; Dz <= NSR; ++Dz) {
    // deposits of nodes m0 .. m0 + 7 of the source slab for this D_z: target
    // layer lz reads halo layer lz (sources at z + D_z)
    __syncthreads();
    for (int h = tid; h < SLAB; h += NTH) {
      const int hx = h % H, hy = (h / H) % H, lz = h / (H * H);
      const int sx = x0 - NSR + hx, sy = y0 - NSR + hy, sz = z0 + lz + Dz;
      if (box && (sx < 0 || sx >= n || sy < 0 || sy >= n || sz < 0 || sz >= n)) {   // no source outside the box
#pragma unroll
        for (int mm = 0; mm < 8; ++mm) Gs[mm * SLAB + h] = 0.0;
        continue;
      }
      const int ex = (sx + 2 * n) % n, ey = (sy + 2 * n) % n, ez = (sz + 2 * n) % n;
      const double *g = gE + (size_t(ex) + size_t(n) * (ey + size_t(n) * ez)) * NM + m0;
#pragma unroll
      for (int mm = 0; mm < 8; ++mm) Gs[mm * SLAB + h] = (NM % 8 == 0 || m0 + mm < NM) ? g[mm] : 0.0;
    }
    __syncthreads();
    for (int Dyx = 0; Dyx < S * S; ++Dyx, ++st) {
      const int Dx = Dyx % S - NSR, Dy = Dyx / S - NSR;
      const int cur = st & 1;
      double tp[TPF];
      const bool more = st + 1 < NST;
      if (more) {
#pragma unroll
        for (int q = 0; q < TPF; ++q) {
          const int i = tid + NTH * q;
          if (i < TV) tp[q] = table(st + 1, i);
        }
      }
      const double *tb = Ts[cur];
      const int cb = ((2 * w) * H + (aly + Dy + NSR)) * H + (alx + Dx + NSR);
#pragma unroll
      for (int k0 = 0; k0 < 8; k0 += 4) {
        const double av0 = Gs[(k0 + kq) * SLAB + cb];           // layer 2 w
        const double av1 = Gs[(k0 + kq) * SLAB + cb + H * H];   // layer 2 w + 1
        const double *brow = tb + (k0 + kq) * NAP + r;
#pragma unroll
        for (int t = 0; t < NAT; ++t) {
          const double bv = brow[16 * t];
          acc[0][t] = M::step(av0, bv, acc[0][t]);
          acc[1][t] = M::step(av1, bv, acc[1][t]);
        }
      }
      if (more) {
#pragma unroll
        for (int q = 0; q < TPF; ++q) {
          const int i = tid + NTH * q;
          if (i < TV) Ts[cur ^ 1][(i / NA) * NAP + i % NA] = tp[q];
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int hh = 0; hh < 2; ++hh)
#pragma unroll
    for (int t = 0; t < NAT; ++t) {
      const int a = 16 * t + r;
      if (a >= NA) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int e = M::row(lane, v);
        const int ex = x0 + (e & 3), ey = y0 + (e >> 2), ez = z0 + 2 * w + hh;
        if (ex >= n || ey >= n || ez >= n) continue;
        Aout[(size_t(ex) + size_t(n) * (ey + size_t(n) * ez)) * NA + a] = -acc[hh][t][v];
      }
    }
}

template <int PO, int NA>
static int adj_mfma_nsr(hipStream_t s, dim3 g, int n, int nsr, int box, const double *gE, const double *Tt, double *A) {
  switch (nsr) {
    case 1: hipLaunchKernelGGL((k_adj_mfma<1, PO, NA>), g, dim3(kAdjThreads), 0, s, n, box, gE, Tt, A); return 0;
    case 2: hipLaunchKernelGGL((k_adj_mfma<2, PO, NA>), g, dim3(kAdjThreads), 0, s, n, box, gE, Tt, A); return 0;
    case 3: hipLaunchKernelGGL((k_adj_mfma<3, PO, NA>), g, dim3(kAdjThreads), 0, s, n, box, gE, Tt, A); return 0;
    default: return -1;
  }
}

int launch_adj_near_mfma(hipStream_t s, int nb, int n, int nsr, int p, int nl, int box, const double *gE,
                         const double *Tt, double *A) {
  const int bricks = (n + kPsiBS - 1) / kPsiBS, bricksz = (n + kPsiBZ - 1) / kPsiBZ;
  dim3 g(nb * bricks * bricks * bricksz);
  switch (10 * p + nl) {   // the families with 27 or more moments
    case 43: return adj_mfma_nsr<4, 27>(s, g, n, nsr, box, gE, Tt, A);
    case 54: return adj_mfma_nsr<5, 64>(s, g, n, nsr, box, gE, Tt, A);
    case 63: return adj_mfma_nsr<6, 27>(s, g, n, nsr, box, gE, Tt, A);
    case 65: return adj_mfma_nsr<6, 125>(s, g, n, nsr, box, gE, Tt, A);
    default: return -1;
  }
}

template <class T>
int launch_psi(hipStream_t s, int nb, int n, int nsr, int p, int box, const double *C, const T *Tab, const double *phi,
               T *Wel) {
  if (p != 5) return -1;
  const int bricks = (n + kPsiBS - 1) / kPsiBS, bricksz = (n + kPsiBZ - 1) / kPsiBZ;
  dim3 g(nb * bricks * bricks * bricksz);
  switch (nsr) {
    case 1: hipLaunchKernelGGL((k_psi<1, 5, T>), g, dim3(kPsiThreads), 0, s, n, box, C, Tab, phi, Wel); return 0;
    case 2: hipLaunchKernelGGL((k_psi<2, 5, T>), g, dim3(kPsiThreads), 0, s, n, box, C, Tab, phi, Wel); return 0;
    case 3: hipLaunchKernelGGL((k_psi<3, 5, T>), g, dim3(kPsiThreads), 0, s, n, box, C, Tab, phi, Wel); return 0;
    default: return -1;
  }
}
template int launch_psi<double>(hipStream_t, int, int, int, int, int, const double *, const double *, const double *,
                                double *);

template <int PO, int NA>
static int psi_mfma_nsr(hipStream_t s, dim3 g, int n, int nsr, int box, const double *C, const double *Tab,
                        const double *phi, double *Wel) {
  switch (nsr) {
    case 1: hipLaunchKernelGGL((k_psi<1, PO, double, NA>), g, dim3(kPsiThreads), 0, s, n, box, C, Tab, phi, Wel); return 0;
    case 2: hipLaunchKernelGGL((k_psi<2, PO, double, NA>), g, dim3(kPsiThreads), 0, s, n, box, C, Tab, phi, Wel); return 0;
    case 3: hipLaunchKernelGGL((k_psi<3, PO, double, NA>), g, dim3(kPsiThreads), 0, s, n, box, C, Tab, phi, Wel); return 0;
    default: return -1;
  }
}

int launch_psi_mfma_g(hipStream_t s, int nb, int n, int nsr, int p, int nl, int box, const double *C, const double *Tab,
                      const double *phi, double *Wel) {
  const int bricks = (n + kPsiBS - 1) / kPsiBS, bricksz = (n + kPsiBZ - 1) / kPsiBZ;
  dim3 g(nb * bricks * bricks * bricksz);
  switch (10 * p + nl) {   // (order, moments per axis) of the screen families up to order 5
    case 52: return psi_mfma_nsr<5, 8>(s, g, n, nsr, box, C, Tab, phi, Wel);
    case 32: return psi_mfma_nsr<3, 8>(s, g, n, nsr, box, C, Tab, phi, Wel);
    case 43: return psi_mfma_nsr<4, 27>(s, g, n, nsr, box, C, Tab, phi, Wel);
    case 54: return psi_mfma_nsr<5, 64>(s, g, n, nsr, box, C, Tab, phi, Wel);
    case 63: return psi_mfma_nsr<6, 27>(s, g, n, nsr, box, C, Tab, phi, Wel);
    case 65: return psi_mfma_nsr<6, 125>(s, g, n, nsr, box, C, Tab, phi, Wel);
    default: return -1;   // one moment (one-element q = 2): the table sums are faster
  }
}
template int launch_psi<float>(hipStream_t, int, int, int, int, int, const double *, const float *, const double *,
                               float *);

}  // namespace fep3m
