// Mesh-side kernels: load assembly, projections, the matrix-free periodic
// order-p stiffness operator (and the Chebyshev-Jacobi smoother fused into
// it), multigrid transfers, the coarse-grid solve and float64 reductions.
//
// Mesh vectors are [z][y][x] arrays of P^3 doubles, P = p n, global node
// index p e + k (mod P) along each axis.  The operator is the Kronecker sum
//   K = K1 (x) M1 (x) M1 + M1 (x) K1 (x) M1 + M1 (x) M1 (x) K1
// (the Galerkin stiffness of the tensor Q_p space on a uniform periodic
// mesh, Section 2.2), applied as y = Kx (My Mz x) + Mx (Ky Mz x + My Kz x)
// with banded 1-D passes on an LDS tile.
#include "kernels.hpp"

namespace fep3m {

__device__ __forceinline__ int wrapi(int i, int P) {
  int r = i % P;
  return r < 0 ? r + P : r;
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  // Fixed-shape tree over the block (deterministic).
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// ----------------------------------------------------------------- load

// b at node (gz, gy, gx): 4 pi sum over the 1..8 elements owning the node of
// sum_a C[E][a] g[ax][kx] g[ay][ky] g[az][kz] (gather form, no atomics),
// with block partial sums of b for the compatibility projection.
__global__ __launch_bounds__(256) void k_load(int n, int p, const double *__restrict__ C,
                                              const double *__restrict__ gw, double *__restrict__ b,
                                              double *__restrict__ partial) {
  __shared__ double red[256];
  const int P = p * n;
  const size_t total = size_t(P) * P * P;
  double acc = 0.0;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    const int gx = int(g % P), gy = int((g / P) % P), gz = int(g / (size_t(P) * P));
    int ex[2], kx[2], ey[2], ky[2], ez[2], kz[2];
    int nx = 1, ny = 1, nz = 1;
    ex[0] = gx / p; kx[0] = gx % p;
    ey[0] = gy / p; ky[0] = gy % p;
    ez[0] = gz / p; kz[0] = gz % p;
    if (kx[0] == 0) { ex[1] = (ex[0] + n - 1) % n; kx[1] = p; nx = 2; }
    if (ky[0] == 0) { ey[1] = (ey[0] + n - 1) % n; ky[1] = p; ny = 2; }
    if (kz[0] == 0) { ez[1] = (ez[0] + n - 1) % n; kz[1] = p; nz = 2; }
    double s = 0.0;
    for (int iz = 0; iz < nz; ++iz)
      for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
          const size_t E = size_t(ex[ix]) + size_t(n) * (ey[iy] + size_t(n) * ez[iz]);
          const double *c = C + E * 8;
          const double gx0 = gw[kx[ix]], gx1 = gw[(p + 1) + kx[ix]];
          const double gy0 = gw[ky[iy]], gy1 = gw[(p + 1) + ky[iy]];
          const double gz0 = gw[kz[iz]], gz1 = gw[(p + 1) + kz[iz]];
          s += gz0 * (gy0 * (gx0 * c[0] + gx1 * c[1]) + gy1 * (gx0 * c[2] + gx1 * c[3]))
             + gz1 * (gy0 * (gx0 * c[4] + gx1 * c[5]) + gy1 * (gx0 * c[6] + gx1 * c[7]));
        }
    s *= 4.0 * M_PI;
    b[g] = s;
    acc += s;
  }
  double t = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// v -= s * w1[kx] w1[ky] w1[kz] with s = scal[0] / V  (V = n^3 in element
// units): subtracts the uniform-background multiple of M 1.  Used on the
// load (compatibility) with scal = sum b.
__global__ __launch_bounds__(256) void k_sub_mass_ones(int n, int p, const double *__restrict__ w1,
                                                       const double *__restrict__ scal, double *__restrict__ v) {
  const int P = p * n;
  const size_t total = size_t(P) * P * P;
  const double s = scal[0] / (double(n) * n * n);
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    const int gx = int(g % P), gy = int((g / P) % P), gz = int(g / (size_t(P) * P));
    v[g] -= s * w1[gx % p] * w1[gy % p] * w1[gz % p];
  }
}

// Block partials of (M 1)^T v = sum w1 w1 w1 v (the integral of the FE field).
__global__ __launch_bounds__(256) void k_mass_dot(int n, int p, const double *__restrict__ w1,
                                                  const double *__restrict__ v, double *__restrict__ partial) {
  __shared__ double red[256];
  const int P = p * n;
  const size_t total = size_t(P) * P * P;
  double acc = 0.0;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    const int gx = int(g % P), gy = int((g / P) % P), gz = int(g / (size_t(P) * P));
    acc += w1[gx % p] * w1[gy % p] * w1[gz % p] * v[g];
  }
  double t = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// v -= scal[0] / V (constant shift; fixes int phi = 0).
__global__ __launch_bounds__(256) void k_sub_const(size_t total, double invV, const double *__restrict__ scal,
                                                   double *__restrict__ v) {
  const double s = scal[0] * invV;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x)
    v[g] -= s;
}

// ----------------------------------------------------------------- operator

template <int PO>
__device__ __forceinline__ double diag_at(const LevelOp &op, int kx, int ky, int kz) {
  return op.dk[kx] * op.dm[ky] * op.dm[kz] + op.dm[kx] * op.dk[ky] * op.dm[kz] + op.dm[kx] * op.dm[ky] * op.dk[kz];
}

template <int PO, int TE>
struct ApplyShape {
  static constexpr int O = TE * PO;          // owned nodes per axis
  static constexpr int I = O + PO + 1;       // input nodes per axis (with halo)
  static constexpr int NX = I * I * I;
  static constexpr int NA = O * I * I;
  static constexpr int NC = O * O * I;
  static constexpr bool kReuse = 2 * NC <= NX;
  static constexpr int LDS = NX + 2 * NA + (kReuse ? 0 : 2 * NC);
};

// One tile of TE^3 elements per block: y = K x on the owned nodes, then the
// mode's epilogue.  The owned nodes of a tile are p*e + k, k < p, for its
// elements; the inputs reach one element below and one node above.
template <int PO, int TE>
__global__ __launch_bounds__(256) void k_apply(LevelOp op, const double *__restrict__ x,
                                               const double *__restrict__ f, double *__restrict__ out,
                                               double *__restrict__ dvec, double *__restrict__ xo, double c1,
                                               double c2, int mode, double *__restrict__ partial) {
  using S = ApplyShape<PO, TE>;
  constexpr int O = S::O, I = S::I, Q1 = PO + 1;
  __shared__ double lds[S::LDS];
  __shared__ double red[256];
  double *xs = lds;
  double *A = lds + S::NX;
  double *B = A + S::NA;
  double *C1 = S::kReuse ? lds : B + S::NA;
  double *C2 = C1 + S::NC;
  const int P = op.P;
  const int tiles = (op.n + TE - 1) / TE;
  int t = blockIdx.x;
  const int tx = t % tiles;
  t /= tiles;
  const int ty = t % tiles;
  const int tz = t / tiles;
  const int ox0 = tx * O, oy0 = ty * O, oz0 = tz * O;

  for (int li = threadIdx.x; li < S::NX; li += blockDim.x) {
    const int lx = li % I, ly = (li / I) % I, lz = li / (I * I);
    const int gx = wrapi(ox0 - PO + lx, P), gy = wrapi(oy0 - PO + ly, P), gz = wrapi(oz0 - PO + lz, P);
    xs[li] = x[(size_t(gz) * P + gy) * P + gx];
  }
  __syncthreads();
  // z pass: A = Mz x, B = Kz x on owned z, all y, x
  for (int li = threadIdx.x; li < S::NA; li += blockDim.x) {
    const int lxy = li % (I * I), oz = li / (I * I);
    const int k = oz % PO, lz = oz + PO;
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int j = 0; j < Q1; ++j) {
      const double v = xs[(lz - k + j) * I * I + lxy];
      a += op.me[k * Q1 + j] * v;
      b += op.ke[k * Q1 + j] * v;
    }
    if (k == 0) {
#pragma unroll
      for (int j = 0; j < Q1; ++j) {
        const double v = xs[(lz - PO + j) * I * I + lxy];
        a += op.me[PO * Q1 + j] * v;
        b += op.ke[PO * Q1 + j] * v;
      }
    }
    A[li] = a;
    B[li] = b;
  }
  __syncthreads();
  // y pass: C1 = My A, C2 = Ky A + My B on owned z, y; all x
  for (int li = threadIdx.x; li < S::NC; li += blockDim.x) {
    const int lx = li % I, oy = (li / I) % O, oz = li / (I * O);
    const int k = oy % PO, ly = oy + PO;
    double c1v = 0.0, c2v = 0.0;
#pragma unroll
    for (int j = 0; j < Q1; ++j) {
      const int src = (oz * I + (ly - k + j)) * I + lx;
      const double av = A[src], bv = B[src];
      c1v += op.me[k * Q1 + j] * av;
      c2v += op.ke[k * Q1 + j] * av + op.me[k * Q1 + j] * bv;
    }
    if (k == 0) {
#pragma unroll
      for (int j = 0; j < Q1; ++j) {
        const int src = (oz * I + (ly - PO + j)) * I + lx;
        const double av = A[src], bv = B[src];
        c1v += op.me[PO * Q1 + j] * av;
        c2v += op.ke[PO * Q1 + j] * av + op.me[PO * Q1 + j] * bv;
      }
    }
    C1[li] = c1v;
    C2[li] = c2v;
  }
  __syncthreads();
  // x pass and epilogue on the owned nodes
  double acc = 0.0;
  for (int li = threadIdx.x; li < O * O * O; li += blockDim.x) {
    const int ox = li % O, oy = (li / O) % O, oz = li / (O * O);
    const int gx = ox0 + ox, gy = oy0 + oy, gz = oz0 + oz;
    const int k = ox % PO, lx = ox + PO;
    double y = 0.0;
    const int base = (oz * O + oy) * I;
#pragma unroll
    for (int j = 0; j < Q1; ++j) y += op.ke[k * Q1 + j] * C1[base + lx - k + j] + op.me[k * Q1 + j] * C2[base + lx - k + j];
    if (k == 0) {
#pragma unroll
      for (int j = 0; j < Q1; ++j)
        y += op.ke[PO * Q1 + j] * C1[base + lx - PO + j] + op.me[PO * Q1 + j] * C2[base + lx - PO + j];
    }
    if (gx >= P || gy >= P || gz >= P) continue;
    const size_t g = (size_t(gz) * P + gy) * P + gx;
    if (mode == kApply) {
      out[g] = y;
    } else if (mode == kResidual) {
      out[g] = f[g] - y;
    } else if (mode == kCheb) {
      const double D = diag_at<PO>(op, k, oy % PO, oz % PO);
      const double fv = f ? f[g] : 0.0;
      const double r = (fv - y) / D;
      const double dn = (c1 != 0.0 ? c1 * dvec[g] : 0.0) + c2 * r;
      dvec[g] = dn;
      if (xo) xo[g] = x[g] + dn;
    } else {  // kApplyDot
      out[g] = y;
      acc += x[g] * y;
    }
  }
  if (mode == kApplyDot) {
    double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// First Chebyshev step from a zero iterate: x = d = c2 D^-1 f.
__global__ __launch_bounds__(256) void k_cheb_first(LevelOp op, const double *__restrict__ f,
                                                    double *__restrict__ d, double *__restrict__ x, double c2) {
  const int P = op.P, p = op.p;
  const size_t total = size_t(P) * P * P;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    const int kx = int(g % P) % p, ky = int((g / P) % P) % p, kz = int(g / (size_t(P) * P)) % p;
    const double D = op.dk[kx] * op.dm[ky] * op.dm[kz] + op.dm[kx] * op.dk[ky] * op.dm[kz] + op.dm[kx] * op.dm[ky] * op.dk[kz];
    const double v = c2 * f[g] / D;
    d[g] = v;
    x[g] = v;
  }
}

// ----------------------------------------------------------------- transfers

// Coarse value = sum over the fine nodes that reference the coarse node of
// weight * fine value (restriction R = P^T, gather form).
__global__ __launch_bounds__(256) void k_restrict(Transfer tr, const double *__restrict__ rf, double *__restrict__ fc) {
  const int Pc = tr.Pc, Pf = tr.Pf, pc = tr.pc, nc = tr.nc, ns = tr.ns, pf = tr.pf, r = tr.r;
  const size_t total = size_t(Pc) * Pc * Pc;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    const int gc[3] = {int(g % Pc), int((g / Pc) % Pc), int(g / (size_t(Pc) * Pc))};
    int fidx[3][6 * kMaxP];
    double fw[3][6 * kMaxP];
    int cnt[3];
    for (int a = 0; a < 3; ++a) {
      const int e = gc[a] / pc, j = gc[a] % pc;
      int c = 0;
      for (int s = 0; s < ns; ++s) {
        const double w = tr.w[s * (pc + 1) + j];
        if (w != 0.0) { fidx[a][c] = (pf * r * e + s) % Pf; fw[a][c] = w; ++c; }
      }
      if (j == 0) {
        const int em = (e + nc - 1) % nc;
        for (int s = 0; s < ns; ++s) {
          const double w = tr.w[s * (pc + 1) + pc];
          if (w != 0.0) { fidx[a][c] = (pf * r * em + s) % Pf; fw[a][c] = w; ++c; }
        }
      }
      cnt[a] = c;
    }
    double acc = 0.0;
    for (int iz = 0; iz < cnt[2]; ++iz) {
      double sy = 0.0;
      for (int iy = 0; iy < cnt[1]; ++iy) {
        const double *row = rf + (size_t(fidx[2][iz]) * Pf + fidx[1][iy]) * Pf;
        double sx = 0.0;
        for (int ix = 0; ix < cnt[0]; ++ix) sx += fw[0][ix] * row[fidx[0][ix]];
        sy += fw[1][iy] * sx;
      }
      acc += fw[2][iz] * sy;
    }
    fc[g] = acc;
  }
}

// xf += P ec: fine node value of the coarse FE function.
__global__ __launch_bounds__(256) void k_prolong_add(Transfer tr, const double *__restrict__ ec, double *__restrict__ xf) {
  const int Pc = tr.Pc, Pf = tr.Pf, pc = tr.pc, ns = tr.ns;
  const size_t total = size_t(Pf) * Pf * Pf;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    const int gf[3] = {int(g % Pf), int((g / Pf) % Pf), int(g / (size_t(Pf) * Pf))};
    int ci[3][kMaxP + 1];
    const double *wv[3];
    for (int a = 0; a < 3; ++a) {
      const int e = gf[a] / ns, s = gf[a] % ns;
      wv[a] = tr.w + s * (pc + 1);
      for (int j = 0; j <= pc; ++j) ci[a][j] = (pc * e + j) % Pc;
    }
    double acc = 0.0;
    for (int jz = 0; jz <= pc; ++jz) {
      if (wv[2][jz] == 0.0) continue;
      double sy = 0.0;
      for (int jy = 0; jy <= pc; ++jy) {
        if (wv[1][jy] == 0.0) continue;
        const double *row = ec + (size_t(ci[2][jz]) * Pc + ci[1][jy]) * Pc;
        double sx = 0.0;
        for (int jx = 0; jx <= pc; ++jx) sx += wv[0][jx] * row[ci[0][jx]];
        sy += wv[1][jy] * sx;
      }
      acc += wv[2][jz] * sy;
    }
    xf[g] += acc;
  }
}

// ----------------------------------------------------------------- coarse solve

// Exact periodic solve on the coarsest Q_pc level by fast diagonalisation:
// x = (V (x) V (x) V) diag(1 / (l_i + l_j + l_k)) (V (x) V (x) V)^T f with the
// constant mode (l = 0) dropped.  One block; nc^3 <= kCoarseMax.
constexpr int kCoarseMax = 4096;
__global__ __launch_bounds__(256) void k_coarse_solve(int Pn, const double *__restrict__ V, const double *__restrict__ lam,
                                                      const double *__restrict__ f, double *__restrict__ x) {
  __shared__ double a[kCoarseMax];
  __shared__ double b[kCoarseMax];
  const int N3 = Pn * Pn * Pn;
  for (int i = threadIdx.x; i < N3; i += blockDim.x) a[i] = f[i];
  __syncthreads();
  // b = V^T along x
  for (int i = threadIdx.x; i < N3; i += blockDim.x) {
    const int ix = i % Pn, rest = i - ix;
    double s = 0.0;
    for (int c = 0; c < Pn; ++c) s += V[c * Pn + ix] * a[rest + c];
    b[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N3; i += blockDim.x) {
    const int ix = i % Pn, iy = (i / Pn) % Pn, iz = i / (Pn * Pn);
    double s = 0.0;
    for (int c = 0; c < Pn; ++c) s += V[c * Pn + iy] * b[(iz * Pn + c) * Pn + ix];
    a[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N3; i += blockDim.x) {
    const int ix = i % Pn, iy = (i / Pn) % Pn, iz = i / (Pn * Pn);
    double s = 0.0;
    for (int c = 0; c < Pn; ++c) s += V[c * Pn + iz] * a[(c * Pn + iy) * Pn + ix];
    const double L = lam[ix] + lam[iy] + lam[iz];
    b[i] = (ix == 0 && iy == 0 && iz == 0) ? 0.0 : s / L;
  }
  __syncthreads();
  // back: V along z, y, x
  for (int i = threadIdx.x; i < N3; i += blockDim.x) {
    const int ix = i % Pn, iy = (i / Pn) % Pn, iz = i / (Pn * Pn);
    double s = 0.0;
    for (int c = 0; c < Pn; ++c) s += V[iz * Pn + c] * b[(c * Pn + iy) * Pn + ix];
    a[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N3; i += blockDim.x) {
    const int ix = i % Pn, iy = (i / Pn) % Pn, iz = i / (Pn * Pn);
    double s = 0.0;
    for (int c = 0; c < Pn; ++c) s += V[iy * Pn + c] * a[(iz * Pn + c) * Pn + ix];
    b[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N3; i += blockDim.x) {
    const int ix = i % Pn, rest = i - ix;
    double s = 0.0;
    for (int c = 0; c < Pn; ++c) s += V[ix * Pn + c] * b[rest + c];
    x[i] = s;
  }
}

// ----------------------------------------------------------------- vectors

__global__ __launch_bounds__(256) void k_dot(size_t n, const double *__restrict__ a, const double *__restrict__ b,
                                             double *__restrict__ partial) {
  __shared__ double red[256];
  double acc = 0.0;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    acc += a[i] * b[i];
  double t = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// x += alpha p; r -= alpha q; partial of r.r
__global__ __launch_bounds__(256) void k_cg_update(size_t n, double alpha, const double *__restrict__ p,
                                                   const double *__restrict__ q, double *__restrict__ x,
                                                   double *__restrict__ r, double *__restrict__ partial) {
  __shared__ double red[256];
  double acc = 0.0;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    x[i] += alpha * p[i];
    const double rv = r[i] - alpha * q[i];
    r[i] = rv;
    acc += rv * rv;
  }
  double t = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// p = z + beta p
__global__ __launch_bounds__(256) void k_xpay(size_t n, double beta, const double *__restrict__ z, double *__restrict__ p) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

__global__ __launch_bounds__(256) void k_scale(size_t n, double s, const double *__restrict__ a, double *__restrict__ b) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    b[i] = s * a[i];
}

// Deterministic pseudo-random fill (power iteration start vector).
__global__ __launch_bounds__(256) void k_hash_fill(size_t n, uint32_t seed, double *__restrict__ v) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    uint32_t h = uint32_t(i) * 2654435761u ^ seed;
    h ^= h >> 16; h *= 0x7feb352du; h ^= h >> 15; h *= 0x846ca68bu; h ^= h >> 16;
    v[i] = double(h) / 4294967296.0 - 0.5;
  }
}

// Second stage of every reduction: one block sums `count` partials in a
// fixed order into out[0].
__global__ __launch_bounds__(256) void k_sum_partials(int count, const double *__restrict__ partial, double *__restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partial[i];
  double t = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = t;
}

// ----------------------------------------------------------------- launchers

namespace {
inline int grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  return int(g < kRedBlocks ? (g == 0 ? 1 : g) : kRedBlocks);
}
}  // namespace

void launch_load(hipStream_t s, int n, int p, const double *C, const double *gw, double *b, double *partial) {
  const size_t tot = size_t(p * n) * (p * n) * (p * n);
  hipLaunchKernelGGL(k_load, dim3(grid_for(tot)), dim3(256), 0, s, n, p, C, gw, b, partial);
}
int red_grid(size_t n) { return grid_for(n); }
void launch_sum_partials(hipStream_t s, int count, const double *partial, double *out) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, count, partial, out);
}
void launch_sub_mass_ones(hipStream_t s, int n, int p, const double *w1, const double *scal, double *v) {
  const size_t tot = size_t(p * n) * (p * n) * (p * n);
  hipLaunchKernelGGL(k_sub_mass_ones, dim3(grid_for(tot)), dim3(256), 0, s, n, p, w1, scal, v);
}
void launch_mass_dot(hipStream_t s, int n, int p, const double *w1, const double *v, double *partial) {
  const size_t tot = size_t(p * n) * (p * n) * (p * n);
  hipLaunchKernelGGL(k_mass_dot, dim3(grid_for(tot)), dim3(256), 0, s, n, p, w1, v, partial);
}
void launch_sub_const(hipStream_t s, size_t total, double invV, const double *scal, double *v) {
  hipLaunchKernelGGL(k_sub_const, dim3(grid_for(total)), dim3(256), 0, s, total, invV, scal, v);
}

template <int PO, int TE>
static int apply_impl(hipStream_t s, const LevelOp &op, const double *x, const double *f, double *out, double *d,
                      double *xo, double c1, double c2, int mode, double *partial) {
  const int tiles = (op.n + TE - 1) / TE;
  const int nb = tiles * tiles * tiles;
  hipLaunchKernelGGL((k_apply<PO, TE>), dim3(nb), dim3(256), 0, s, op, x, f, out, d, xo, c1, c2, mode, partial);
  return nb;
}

int launch_apply(hipStream_t s, const LevelOp &op, const double *x, const double *f, double *out, double *d,
                 double *xo, double c1, double c2, int mode, double *partial) {
  switch (op.p) {
    case 1: return apply_impl<1, 8>(s, op, x, f, out, d, xo, c1, c2, mode, partial);
    case 2: return apply_impl<2, 4>(s, op, x, f, out, d, xo, c1, c2, mode, partial);
    case 3: return apply_impl<3, 3>(s, op, x, f, out, d, xo, c1, c2, mode, partial);
    case 5: return apply_impl<5, 2>(s, op, x, f, out, d, xo, c1, c2, mode, partial);
    default: return -1;
  }
}

int apply_blocks(const LevelOp &op) {
  int TE = op.p == 1 ? 8 : op.p == 2 ? 4 : op.p == 3 ? 3 : 2;
  int tiles = (op.n + TE - 1) / TE;
  return tiles * tiles * tiles;
}

void launch_cheb_first(hipStream_t s, const LevelOp &op, const double *f, double *d, double *x, double c2) {
  const size_t tot = size_t(op.P) * op.P * op.P;
  hipLaunchKernelGGL(k_cheb_first, dim3(grid_for(tot)), dim3(256), 0, s, op, f, d, x, c2);
}
void launch_restrict(hipStream_t s, const Transfer &tr, const double *rf, double *fc) {
  const size_t tot = size_t(tr.Pc) * tr.Pc * tr.Pc;
  hipLaunchKernelGGL(k_restrict, dim3(grid_for(tot)), dim3(256), 0, s, tr, rf, fc);
}
void launch_prolong_add(hipStream_t s, const Transfer &tr, const double *ec, double *xf) {
  const size_t tot = size_t(tr.Pf) * tr.Pf * tr.Pf;
  hipLaunchKernelGGL(k_prolong_add, dim3(grid_for(tot)), dim3(256), 0, s, tr, ec, xf);
}
void launch_coarse_solve(hipStream_t s, int Pn, const double *V, const double *lam, const double *f, double *x) {
  hipLaunchKernelGGL(k_coarse_solve, dim3(1), dim3(256), 0, s, Pn, V, lam, f, x);
}
void launch_dot(hipStream_t s, size_t n, const double *a, const double *b, double *partial) {
  hipLaunchKernelGGL(k_dot, dim3(grid_for(n)), dim3(256), 0, s, n, a, b, partial);
}
void launch_cg_update(hipStream_t s, size_t n, double alpha, const double *p, const double *q, double *x, double *r,
                      double *partial) {
  hipLaunchKernelGGL(k_cg_update, dim3(grid_for(n)), dim3(256), 0, s, n, alpha, p, q, x, r, partial);
}
void launch_xpay(hipStream_t s, size_t n, double beta, const double *z, double *p) {
  hipLaunchKernelGGL(k_xpay, dim3(grid_for(n)), dim3(256), 0, s, n, beta, z, p);
}
void launch_scale(hipStream_t s, size_t n, double sc, const double *a, double *b) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(256), 0, s, n, sc, a, b);
}
void launch_hash_fill(hipStream_t s, size_t n, uint32_t seed, double *v) {
  hipLaunchKernelGGL(k_hash_fill, dim3(grid_for(n)), dim3(256), 0, s, n, seed, v);
}

}  // namespace fep3m
