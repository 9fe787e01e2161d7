// Near-screen field (element-to-point evaluation of Section 3, eq. sc with
// the Remark's order-p tables):
//
//   Psi_E[m] = sum_{D in [-NSR, NSR]^3} sum_a T[a][D][m] C[E - D][a]
//
// the potential, at the order-p nodes m of target element E, of the combined
// screens of every element in E's near block (D = 0 is the self term).  The
// kernel writes W_E = phi_E - Psi_E, the field the charges of E interpolate.
//
// Block = a 4 x 4 x 4 brick of target elements and 8 wavefronts: lane l of
// every wave owns target element l of the brick, wave w owns the 27 nodes
// m = 27 w .. 27 w + 26.  The moments C of the brick's halo
// ((4 + 2 NSR)^3 elements) sit in LDS; the tables are streamed through LDS
// one offset D at a time and read as wave-uniform broadcasts, so every table
// value fetched from L2 feeds 64 target elements.
#include "kernels.hpp"

namespace fep3m {

template <int NSR, int PO>
__global__ __launch_bounds__(512) void k_psi(int n, const double *__restrict__ C, const double *__restrict__ T,
                                             const double *__restrict__ phi, double *__restrict__ Wel) {
  constexpr int BS = 4;                       // brick edge (elements)
  constexpr int H = BS + 2 * NSR;             // halo edge
  constexpr int H3 = H * H * H;
  constexpr int S = 2 * NSR + 1;
  constexpr int ND = S * S * S;
  constexpr int Q1 = PO + 1;
  constexpr int NM = Q1 * Q1 * Q1;            // 216 for p = 5
  constexpr int MW = (NM + 7) / 8;            // nodes per wave
  __shared__ double Cs[8 * H3];
  __shared__ double Ts[8 * NM];
  const int bricks = (n + BS - 1) / BS;
  int b = blockIdx.x;
  const int bx = b % bricks;
  b /= bricks;
  const int by = b % bricks;
  const int bz = b / bricks;
  const int x0 = bx * BS, y0 = by * BS, z0 = bz * BS;
  for (int h = threadIdx.x; h < H3; h += blockDim.x) {
    const int hx = h % H, hy = (h / H) % H, hz = h / (H * H);
    const int ex = (x0 - NSR + hx + 2 * n) % n, ey = (y0 - NSR + hy + 2 * n) % n, ez = (z0 - NSR + hz + 2 * n) % n;
    const double *c = C + (size_t(ex) + size_t(n) * (ey + size_t(n) * ez)) * 8;
#pragma unroll
    for (int a = 0; a < 8; ++a) Cs[a * H3 + h] = c[a];
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lx = lane % BS, ly = (lane / BS) % BS, lz = lane / (BS * BS);
  const int m0 = wave * MW;
  double acc[MW];
#pragma unroll
  for (int j = 0; j < MW; ++j) acc[j] = 0.0;
  for (int iD = 0; iD < ND; ++iD) {
    __syncthreads();
    for (int i = threadIdx.x; i < 8 * NM; i += blockDim.x) {
      const int a = i / NM, m = i % NM;
      Ts[i] = T[(size_t(a) * ND + iD) * NM + m];
    }
    __syncthreads();
    const int Dx = iD % S - NSR, Dy = (iD / S) % S - NSR, Dz = iD / (S * S) - NSR;
    const int h = (lx - Dx + NSR) + H * ((ly - Dy + NSR) + H * (lz - Dz + NSR));
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const double c = Cs[a * H3 + h];
      const double *t = Ts + a * NM + m0;
#pragma unroll
      for (int j = 0; j < MW; ++j)
        if (m0 + j < NM) acc[j] += t[j] * c;
    }
  }
  const int ex = x0 + lx, ey = y0 + ly, ez = z0 + lz;
  if (ex >= n || ey >= n || ez >= n) return;
  const int P = PO * n;
  const size_t E = size_t(ex) + size_t(n) * (ey + size_t(n) * ez);
#pragma unroll
  for (int j = 0; j < MW; ++j) {
    const int m = m0 + j;
    if (m >= NM) break;
    const int mx = m % Q1, my = (m / Q1) % Q1, mz = m / (Q1 * Q1);
    const int gx = (PO * ex + mx) % P, gy = (PO * ey + my) % P, gz = (PO * ez + mz) % P;
    Wel[E * NM + m] = phi[(size_t(gz) * P + gy) * P + gx] - acc[j];
  }
}

int launch_psi(hipStream_t s, int n, int nsr, int p, const double *C, const double *T, const double *phi, double *Wel) {
  if (p != 5) return -1;
  const int bricks = (n + 3) / 4;
  dim3 g(bricks * bricks * bricks);
  switch (nsr) {
    case 1: hipLaunchKernelGGL((k_psi<1, 5>), g, dim3(512), 0, s, n, C, T, phi, Wel); return 0;
    case 2: hipLaunchKernelGGL((k_psi<2, 5>), g, dim3(512), 0, s, n, C, T, phi, Wel); return 0;
    case 3: hipLaunchKernelGGL((k_psi<3, 5>), g, dim3(512), 0, s, n, C, T, phi, Wel); return 0;
    default: return -1;
  }
}

}  // namespace fep3m
