// Exact periodic mesh solve by Fourier analysis over the element lattice
// (the solver option of fep3m.h for meshes whose edge is a power of two).
//
// On the uniform periodic mesh the 1-D operators K1, M1 are block circulant:
// node p e + k (owned local index k < p of element e) couples only to the
// nodes of elements e - 1, e, e + 1.  A DFT over the element index turns them
// into p x p Hermitian blocks per frequency f,
//   K^(f) = B0 + B+ w^f + B- w^-f,   w = exp(2 pi i / n),
// and the 3-D operator K = K1 (x) M1 (x) M1 + ... into independent p^3 x p^3
// blocks per frequency triple.  With the generalized eigenvectors of each
// 1-D block, K^(f) W_f = M^(f) W_f diag(lam_f), W_f^H M^(f) W_f = I, the block
// solve is  x^ = (W (x) W (x) W) diag(1 / (lam_x + lam_y + lam_z)) (W (x) W (x) W)^H b^
// (the constant mode, all three null modes at f = 0, dropped: int phi = 0).
//
// Data path per solve: gather the mesh vector into element-major complex
// channels [E][kz][ky][kx] (two real systems as the real and imaginary
// parts of one complex system: the operator is real), three FFT passes over
// the element lattice, the per-frequency block solve, three inverse passes,
// scatter back (real part: first system, imaginary part: second).
#include "kernels.hpp"

namespace fep3m {
namespace {

// Mesh vectors of systems 2c and 2c + 1 -> complex system c, element-major.
template <int PO>
__global__ __launch_bounds__(256) void k_fs_gather(int n, int nsys, const double *__restrict__ v,
                                                   double2 *__restrict__ Z) {
  constexpr int NCH = PO * PO * PO;
  const int P = PO * n;
  const size_t per = size_t(P) * P * P;
  const int ncs = (nsys + 1) / 2;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < per * ncs; t += size_t(gridDim.x) * blockDim.x) {
    const int cs = int(t / per);
    const size_t g = t % per;
    const int gx = int(g % P), gy = int((g / P) % P), gz = int(g / (size_t(P) * P));
    const int ex = gx / PO, ey = gy / PO, ez = gz / PO;
    const int k = ((gz - PO * ez) * PO + (gy - PO * ey)) * PO + (gx - PO * ex);
    const double re = v[size_t(2 * cs) * per + g];
    const double im = (2 * cs + 1 < nsys) ? v[size_t(2 * cs + 1) * per + g] : 0.0;
    Z[(size_t(cs) * n * n * n + (size_t(ez) * n + ey) * n + ex) * NCH + k] = make_double2(re, im);
  }
}

template <int PO>
__global__ __launch_bounds__(256) void k_fs_scatter(int n, int nsys, const double2 *__restrict__ Z,
                                                    double *__restrict__ v) {
  constexpr int NCH = PO * PO * PO;
  const int P = PO * n;
  const size_t per = size_t(P) * P * P;
  const int ncs = (nsys + 1) / 2;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < per * ncs; t += size_t(gridDim.x) * blockDim.x) {
    const int cs = int(t / per);
    const size_t g = t % per;
    const int gx = int(g % P), gy = int((g / P) % P), gz = int(g / (size_t(P) * P));
    const int ex = gx / PO, ey = gy / PO, ez = gz / PO;
    const int k = ((gz - PO * ez) * PO + (gy - PO * ey)) * PO + (gx - PO * ex);
    const double2 z = Z[(size_t(cs) * n * n * n + (size_t(ez) * n + ey) * n + ex) * NCH + k];
    v[size_t(2 * cs) * per + g] = z.x;
    if (2 * cs + 1 < nsys) v[size_t(2 * cs + 1) * per + g] = z.y;
  }
}

// One frequency triple per block: the p^3 values of complex system cs at
// (fx, fy, fz), transformed by W^H along x, y, z, divided by the eigenvalue
// sums (times `scale`, the inverse transform's 1 / n^3), transformed back.
// W[f][k][i]: component k of mode i of frequency f; lam[f][i].
template <int PO>
__global__ __launch_bounds__(256) void k_fs_solve(int n, const double2 *__restrict__ W, const double *__restrict__ lam,
                                                  double2 *__restrict__ Z, double scale) {
  constexpr int NCH = PO * PO * PO, P2 = PO * PO;
  __shared__ double2 buf[2][NCH];
  __shared__ double2 w[3][P2];
  __shared__ double l[3][PO];
  const size_t M = size_t(n) * n * n;
  const size_t f = blockIdx.x % M, cs = blockIdx.x / M;
  const int fx = int(f % n), fy = int((f / n) % n), fz = int(f / (size_t(n) * n));
  const int tid = threadIdx.x;
  const int fa[3] = {fx, fy, fz};
  for (int i = tid; i < 3 * P2; i += blockDim.x) w[i / P2][i % P2] = W[size_t(fa[i / P2]) * P2 + i % P2];
  for (int i = tid; i < 3 * PO; i += blockDim.x) l[i / PO][i % PO] = lam[size_t(fa[i / PO]) * PO + i % PO];
  double2 *zf = Z + (cs * M + f) * NCH;
  const bool act = tid < NCH;
  const int kx = tid % PO, ky = (tid / PO) % PO, kz = tid / P2;
  if (act) buf[0][tid] = zf[tid];
  __syncthreads();
  // y = (W^H)_z (W^H)_y (W^H)_x b: out index i along the axis takes
  // sum_k conj(W[k][i]) in[k]
  int cur = 0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (act) {
      const int i = ax == 0 ? kx : (ax == 1 ? ky : kz);
      const int stride = ax == 0 ? 1 : (ax == 1 ? PO : P2);
      const int base = tid - i * stride;
      double2 s = make_double2(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < PO; ++k) {
        const double2 a = w[ax][k * PO + i], b = buf[cur][base + k * stride];
        s.x += a.x * b.x + a.y * b.y;
        s.y += a.x * b.y - a.y * b.x;
      }
      buf[cur ^ 1][tid] = s;
    }
    cur ^= 1;
    __syncthreads();
  }
  if (act) {
    const double den = l[0][kx] + l[1][ky] + l[2][kz];
    const double r = den == 0.0 ? 0.0 : scale / den;
    buf[cur][tid].x *= r;
    buf[cur][tid].y *= r;
  }
  __syncthreads();
  // x = W_x W_y W_z y: out index k along the axis takes sum_i W[k][i] in[i]
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (act) {
      const int k = ax == 0 ? kx : (ax == 1 ? ky : kz);
      const int stride = ax == 0 ? 1 : (ax == 1 ? PO : P2);
      const int base = tid - k * stride;
      double2 s = make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < PO; ++i) {
        const double2 a = w[ax][k * PO + i], b = buf[cur][base + i * stride];
        s.x += a.x * b.x - a.y * b.y;
        s.y += a.x * b.y + a.y * b.x;
      }
      buf[cur ^ 1][tid] = s;
    }
    cur ^= 1;
    __syncthreads();
  }
  if (act) zf[tid] = buf[cur][tid];
}

// Dense transform along one axis of nsys P^3 arrays [z][y][x]:
// out[line][o] = sum_k A(o, k) in[line][k], A(o, k) = V[k + o P] (TRANS:
// V^T, the forward transform into modes) or V[o + k P] (back), V the
// column-major eigenvector matrix.  A block covers 64 outputs x 64 lines,
// k in chunks of KC staged in LDS, the next chunk's operands fetched into
// registers while the current one is multiplied; each of the four waves
// owns 32 x 32 of the block as 2 x 2 float64 matrix-core tiles (16 x 16 x 4
// steps: lane l supplies row l % 16, k l / 16 of the left operand and
// k l / 16, column l % 16 of the right one; accumulator value v of lane l is
// row l / 16 + 4 v, column l % 16).  LR: the tile rows are lines and the
// columns outputs (along x, where outputs are contiguous, so a store covers
// 16 consecutive outputs); otherwise rows are outputs and columns lines
// (along y and z, where consecutive lines are consecutive x).  Line
// addresses are formed once per block (no division in the k loop).  The
// steps accumulate in k order like fused multiply-adds, so every output
// equals a sequential loop over k.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <bool TRANS, bool LR>
__global__ __launch_bounds__(256) void k_axis_transform(int P, int axis, int nsys, const double *__restrict__ V,
                                                        const double *__restrict__ in, double *__restrict__ out) {
  constexpr int KC = 16, NR = KC * 64 / 256;   // operands per thread and chunk, for each matrix
  __shared__ double As[KC][65];   // [k][o]
  __shared__ double Xs[KC][65];   // [k][line]
  const size_t P2 = size_t(P) * P, per = P2 * P;
  const int otiles = (P + 63) / 64;
  const size_t lines = P2 * nsys;
  const size_t ltile = blockIdx.x / otiles;
  const int o0 = (blockIdx.x % otiles) * 64;
  const size_t l0 = ltile * 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int wo = (w & 1) * 32, wl = (w >> 1) * 32;
  const size_t kstride = axis == 0 ? 1 : (axis == 1 ? size_t(P) : P2);
  // address of element 0 of line l = (system, a, b), a, b the other two axes
  auto line_base = [&](size_t l) -> size_t {
    const size_t sys = l / P2, r = l % P2;
    if (axis == 0) return sys * per + r * P;
    if (axis == 1) return sys * per + (r / P) * P2 + (r % P);
    return sys * per + r;
  };
  // this thread's staging slots: (k in chunk, line or output) and the line
  // or matrix addresses at k = 0
  int xk[NR], ak[NR], ao[NR];
  size_t xb[NR];
  bool xok[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = tid + 256 * r;
    int kk, ll;
    if (axis == 0) { kk = i % KC; ll = i / KC; } else { ll = i % 64; kk = i / 64; }
    xk[r] = kk;
    xok[r] = l0 + ll < lines;
    xb[r] = xok[r] ? line_base(l0 + ll) : 0;
    int k2, oo;
    if (TRANS) { k2 = i % KC; oo = i / KC; } else { oo = i % 64; k2 = i / 64; }
    ak[r] = k2;
    ao[r] = o0 + oo;
  }
  double xv[NR], av[NR];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int k = k0 + xk[r];
      xv[r] = (k < P && xok[r]) ? in[xb[r] + size_t(k) * kstride] : 0.0;
      const int ka = k0 + ak[r], o = ao[r];
      av[r] = (ka < P && o < P) ? (TRANS ? V[ka + size_t(o) * P] : V[o + size_t(ka) * P]) : 0.0;
    }
  };
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  fetch(0);
  for (int k0 = 0; k0 < P; k0 += KC) {
    __syncthreads();   // the previous chunk is consumed
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = tid + 256 * r;
      if (axis == 0) Xs[i % KC][i / KC] = xv[r]; else Xs[i / 64][i % 64] = xv[r];
      if (TRANS) As[i % KC][i / KC] = av[r]; else As[i / 64][i % 64] = av[r];
    }
    __syncthreads();
    if (k0 + KC < P) fetch(k0 + KC);
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      double xa[2], ob[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) xa[i] = Xs[ks + kq][wl + 16 * i + r16];
#pragma unroll
      for (int j = 0; j < 2; ++j) ob[j] = As[ks + kq][wo + 16 * j + r16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = LR ? __builtin_amdgcn_mfma_f64_16x16x4f64(xa[i], ob[j], acc[i][j], 0, 0, 0)
                         : __builtin_amdgcn_mfma_f64_16x16x4f64(ob[j], xa[i], acc[i][j], 0, 0, 0);
    }
  }
  if (LR) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const size_t l = l0 + wl + 16 * i + kq + 4 * v;
        if (l >= lines) continue;
        const size_t b = line_base(l);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int o = o0 + wo + 16 * j + r16;
          if (o < P) out[b + size_t(o) * kstride] = acc[i][j][v];
        }
      }
  } else {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const size_t l = l0 + wl + 16 * i + r16;
      if (l >= lines) continue;
      const size_t b = line_base(l);
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int o = o0 + wo + 16 * j + kq + 4 * v;
          if (o < P) out[b + size_t(o) * kstride] = acc[i][j][v];
        }
    }
  }
}

inline int grid_of(size_t count) {
  size_t g = (count + 255) / 256;
  if (g < 1) g = 1;
  return int(g > 65536 ? 65536 : g);
}

template <int PO>
int fs_solve_impl(hipStream_t s, int nsys, int n, const double *rhs, double *out, double2 *Z, const double2 *tw,
                  const double2 *W, const double *lam) {
  const size_t P = size_t(PO) * n, per = P * P * P;
  const int ncs = (nsys + 1) / 2;
  const size_t M = size_t(n) * n * n;
  hipLaunchKernelGGL(k_fs_gather<PO>, dim3(grid_of(per * ncs)), dim3(256), 0, s, n, nsys, rhs, Z);
  if (launch_fft3_nodes(s, ncs, n, PO * PO * PO, Z, tw, false) != 0) return -1;
  hipLaunchKernelGGL(k_fs_solve<PO>, dim3(unsigned(M * ncs)), dim3(256), 0, s, n, W, lam, Z, 1.0 / double(M));
  if (launch_fft3_nodes(s, ncs, n, PO * PO * PO, Z, tw, true) != 0) return -1;
  hipLaunchKernelGGL(k_fs_scatter<PO>, dim3(grid_of(per * ncs)), dim3(256), 0, s, n, nsys, Z, out);
  return 0;
}

}  // namespace

void launch_axis_transform(hipStream_t s, int P, int axis, int nsys, const double *V, bool to_modes, const double *in,
                           double *out) {
  const size_t lines = size_t(P) * P * nsys;
  const unsigned grid = unsigned(((lines + 63) / 64) * ((P + 63) / 64));
  if (to_modes && axis == 0)
    hipLaunchKernelGGL((k_axis_transform<true, true>), dim3(grid), dim3(256), 0, s, P, axis, nsys, V, in, out);
  else if (to_modes)
    hipLaunchKernelGGL((k_axis_transform<true, false>), dim3(grid), dim3(256), 0, s, P, axis, nsys, V, in, out);
  else if (axis == 0)
    hipLaunchKernelGGL((k_axis_transform<false, true>), dim3(grid), dim3(256), 0, s, P, axis, nsys, V, in, out);
  else
    hipLaunchKernelGGL((k_axis_transform<false, false>), dim3(grid), dim3(256), 0, s, P, axis, nsys, V, in, out);
}

int launch_fs_solve(hipStream_t s, int nsys, int n, int p, const double *rhs, double *out, double2 *Z,
                    const double2 *tw, const double2 *W, const double *lam) {
  switch (p) {
    case 3: return fs_solve_impl<3>(s, nsys, n, rhs, out, Z, tw, W, lam);
    case 4: return fs_solve_impl<4>(s, nsys, n, rhs, out, Z, tw, W, lam);
    case 5: return fs_solve_impl<5>(s, nsys, n, rhs, out, Z, tw, W, lam);
    case 6: return fs_solve_impl<6>(s, nsys, n, rhs, out, Z, tw, W, lam);
    default: return -1;
  }
}

}  // namespace fep3m
