// The grounded box (Section 2.6, eq. bcadjust with g = 0): the mesh
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
// partial[nb K + cfg K + kb] = sum b^2 over this block's interior nodes.
__global__ __launch_bounds__(256) void k_box_resid(int P, int K, int nb, const double *__restrict__ ball,
                                                   const double *__restrict__ yall, double *__restrict__ partial) {
  __shared__ double red[2][4];
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const int Pi = P - 2;
  const size_t per = size_t(P) * P * P, peri = size_t(Pi) * Pi * Pi;
  double sr = 0.0, sb = 0.0;
  for (size_t l = size_t(kb) * blockDim.x + threadIdx.x; l < peri; l += size_t(K) * blockDim.x) {
    const int i = int(l % Pi), j = int((l / Pi) % Pi), k = int(l / (size_t(Pi) * Pi));
    const size_t g = size_t(cfg) * per + (size_t(k + 1) * P + (j + 1)) * P + (i + 1);
    const double bv = ball[g], rv = bv - yall[g];
    sr += rv * rv;
    sb += bv * bv;
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

inline int grid_of(size_t count) {
  size_t g = (count + 255) / 256;
  if (g < 1) g = 1;
  return int(g > 65536 ? 65536 : g);
}

}  // namespace

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

int launch_box_resid(hipStream_t s, int P, int nb, const double *b, const double *y, double *partial) {
  const size_t Pi = size_t(P) - 2;
  const size_t peri = Pi * Pi * Pi;
  int K = int(std::min<size_t>((peri + 255) / 256, size_t(1024) / size_t(nb > 0 ? nb : 1)));
  if (K < 1) K = 1;
  hipLaunchKernelGGL(k_box_resid, dim3(nb * K), dim3(256), 0, s, P, K, nb, b, y, partial);
  return K;
}

}  // namespace fep3m
