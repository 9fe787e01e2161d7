// Mesh-side kernels: load assembly, projections, the matrix-free periodic
// order-p stiffness operator (and the Chebyshev-Jacobi smoother fused into
// it), multigrid transfers, the coarse-grid solve and float64 reductions.
//
// Mesh vectors are [z][y][x] arrays of P^3 doubles, P = p n, global node
// index p e + k (mod P) along each axis.  The operator is the Kronecker sum
//   K = K1 (x) M1 (x) M1 + M1 (x) K1 (x) M1 + M1 (x) M1 (x) K1
// (the Galerkin stiffness of the tensor Q_p space on a uniform periodic
// mesh, Section 2.2), applied as y = Kx (My Mz x) + Mx (Ky Mz x + My Kz x)
// with banded 1-D passes over register columns of an LDS-staged tile.
#include "kernels.hpp"

namespace fep3m {

// Periodic wrap of an index known to lie in [-P, 2P).
__device__ __forceinline__ int wrapi(int i, int P) { return i < 0 ? i + P : (i >= P ? i - P : i); }

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


// Tile order.  Workgroups are dispatched round-robin over the 8 XCDs, each
// with its own L2.  When the tile grid splits into octants of power-of-two
// edge, XCD x takes octant x and walks it in Morton order, so the tiles that
// re-read each other's halos run close together in time on one L2;
// otherwise the order is linear (x fastest).
__device__ __forceinline__ int compact_bits(int v) {  // every third bit
  v &= 0x09249249;
  v = (v ^ (v >> 2)) & 0x030c30c3;
  v = (v ^ (v >> 4)) & 0x0300f00f;
  v = (v ^ (v >> 8)) & 0xff0000ff;
  v = (v ^ (v >> 16)) & 0x000003ff;
  return v;
}
__device__ __forceinline__ void tile_coords(int b, int tiles, int &tx, int &ty, int &tz) {
  const int half = tiles >> 1;
  if ((tiles & 1) == 0 && half > 0 && (half & (half - 1)) == 0) {
    const int xcd = b & 7, idx = b >> 3;
    tx = compact_bits(idx) + half * (xcd & 1);
    ty = compact_bits(idx >> 1) + half * ((xcd >> 1) & 1);
    tz = compact_bits(idx >> 2) + half * (xcd >> 2);
  } else {
    tx = b % tiles;
    ty = (b / tiles) % tiles;
    tz = b / (tiles * tiles);
  }
}

template <int PO, int TE>
struct ApplyShape {
  static constexpr int O = TE * PO;          // owned nodes per axis
  static constexpr int I = O + PO + 1;       // input nodes per axis (with halo)
  static constexpr int SA = I * I + 16;      // stride of one z-plane of A, B (bank padding)
  static constexpr int RS = I + 1;           // row stride of C1, C2
  static constexpr int SC = O * RS;          // plane stride of C1, C2
  static constexpr int YS = O + 1;           // row stride of the output tile
  static constexpr int LDS_AB = 2 * O * SA;
  static constexpr int LDS_C = 2 * O * SC;
  static constexpr int LDS_Y = O * O * YS;
  static constexpr int LDS = LDS_AB > LDS_C + LDS_Y ? LDS_AB : LDS_C + LDS_Y;
  static_assert(I * I <= 256 && O * I <= 256 && O * O <= 256, "tile columns must fit one pass of 256 threads");
};

// Banded 1-D element-assembled operator on a column held in registers:
// out[o] = sum_j a[k][j] v[o + PO - k + j] (+ a[PO][j] v[o + j] for k = 0),
// k = o mod PO, with v indexed from one element below the first output.
// Every coefficient index is a compile-time constant, so the (wave-uniform)
// coefficients come from scalar registers.
template <int PO, int NOUT>
__device__ __forceinline__ void band_apply(const double *__restrict__ a, const double (&v)[NOUT + PO + 1],
                                           double (&out)[NOUT]) {
  constexpr int Q1 = PO + 1;
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    const int k = o % PO;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < Q1; ++j) s += a[k * Q1 + j] * v[o + PO - k + j];
    if (k == 0) {
#pragma unroll
      for (int j = 0; j < Q1; ++j) s += a[PO * Q1 + j] * v[o + j];
    }
    out[o] = s;
  }
}

template <int PO, int NOUT>
__device__ __forceinline__ void band_apply_acc(const double *__restrict__ a, const double (&v)[NOUT + PO + 1],
                                               double (&out)[NOUT]) {
  double t[NOUT];
  band_apply<PO, NOUT>(a, v, t);
#pragma unroll
  for (int o = 0; o < NOUT; ++o) out[o] += t[o];
}

// Barrier for LDS hand-offs only: waits for LDS traffic, leaves global
// loads in flight (the next tile's prefetch crosses it).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The it-th of the TPB tiles handled by block b (Morton order inside each
// XCD's octant when the grid allows it, else linear).  False past the end.
__device__ __forceinline__ bool block_tile(int b, int it, int tpb, int tiles, int &tx, int &ty, int &tz) {
  const int half = tiles >> 1;
  if ((tiles & 1) == 0 && half > 0 && (half & (half - 1)) == 0 && (half * half * half) % tpb == 0) {
    const int xcd = b & 7, idx = (b >> 3) * tpb + it;
    tx = compact_bits(idx) + half * (xcd & 1);
    ty = compact_bits(idx >> 1) + half * ((xcd >> 1) & 1);
    tz = compact_bits(idx >> 2) + half * (xcd >> 2);
    return true;
  }
  const int t = b * tpb + it;
  if (t >= tiles * tiles * tiles) return false;
  tx = t % tiles;
  ty = (t / tiles) % tiles;
  tz = t / (tiles * tiles);
  return true;
}

// TPB tiles of TE^3 elements per block: y = K x on the owned nodes of each
// tile, then the mode's epilogue.  The owned nodes of a tile are p*e + k,
// k < p, for its elements; the inputs reach one element below and one node
// above.  Pass z: each thread streams one (x, y) column of the input from
// global memory and writes A = Mz x, B = Kz x; pass y: one (z, x) column of A
// and B gives C1 = My A and C2 = Ky A + My B; pass x: one (z, y) row of C1,
// C2 gives y = Kx C1 + Mx C2; the epilogue walks the owned nodes x-fastest.
// The next tile's column and epilogue operands are fetched while the
// current tile runs its LDS passes.
template <int PO, int TE, int TPB>
__global__ __launch_bounds__(256) void k_apply(LevelOp op, const double *__restrict__ x,
                                               const double *__restrict__ f, double *__restrict__ out,
                                               const double *xprev, double *xo, double c1, double c2, int mode,
                                               double *__restrict__ partial) {
  using S = ApplyShape<PO, TE>;
  constexpr int O = S::O, I = S::I;
  constexpr int NIT = (O * O * O + 255) / 256;
  __shared__ double lds[S::LDS];         // A, B; then C1, C2, Y; last the dot-product tree
  __shared__ double invd[PO * PO * PO];  // 1 / diag(K) by local node index
  __shared__ double Xo[O * O * O];       // x on the owned nodes (from the z-pass columns)
  double *A = lds;
  double *B = lds + O * S::SA;
  double *C1 = lds;
  double *C2 = lds + O * S::SC;
  double *Y = lds + 2 * O * S::SC;
  const int P = op.P;
  const int tiles = (op.n + TE - 1) / TE;
  const int tid = threadIdx.x;
  const bool need_f = (mode == kResidual) || (mode == kCheb);
  const bool need_d = (mode == kCheb) && (c1 != 0.0);
  for (int i = tid; i < PO * PO * PO; i += 256) {
    const int kx = i % PO, ky = (i / PO) % PO, kz = i / (PO * PO);
    invd[i] = 1.0 / (op.dk[kx] * op.dm[ky] * op.dm[kz] + op.dm[kx] * op.dk[ky] * op.dm[kz] +
                     op.dm[kx] * op.dm[ky] * op.dk[kz]);
  }
  // global inputs of one tile: this thread's z-column and epilogue operands
  auto fetch = [&](int tx, int ty, int tz, double (&v)[I], double (&ff)[NIT], double (&fd)[NIT]) {
    const int ox0 = tx * O, oy0 = ty * O, oz0 = tz * O;
    if (tid < I * I) {
      const int lx = tid % I, ly = tid / I;
      const int gx = wrapi(ox0 - PO + lx, P), gy = wrapi(oy0 - PO + ly, P);
#pragma unroll
      for (int z = 0; z < I; ++z) v[z] = x[(size_t(wrapi(oz0 - PO + z, P)) * P + gy) * P + gx];
    }
#pragma unroll
    for (int r = 0; r < NIT; ++r) {
      const int li = tid + 256 * r;
      const int ox = li % O, oy = (li / O) % O, oz = li / (O * O);
      const int gx = ox0 + ox, gy = oy0 + oy, gz = oz0 + oz;
      const bool ok = li < O * O * O && gx < P && gy < P && gz < P;
      const size_t g = ok ? (size_t(gz) * P + gy) * P + gx : 0;
      ff[r] = (ok && need_f) ? f[g] : 0.0;
      fd[r] = (ok && need_d) ? xprev[g] : 0.0;
    }
  };
  int tx = 0, ty = 0, tz = 0;
  bool valid = block_tile(blockIdx.x, 0, TPB, tiles, tx, ty, tz);
  double v[I], pf_f[NIT], pf_d[NIT];
  if (valid) fetch(tx, ty, tz, v, pf_f, pf_d);
  double acc = 0.0;
  for (int it = 0; it < TPB && valid; ++it) {
    const int ox0 = tx * O, oy0 = ty * O, oz0 = tz * O;
    int ntx = 0, nty = 0, ntz = 0;
    const bool nvalid = (it + 1 < TPB) && block_tile(blockIdx.x, it + 1, TPB, tiles, ntx, nty, ntz);
    double vn[I], nf[NIT], nd[NIT];
    if (nvalid) fetch(ntx, nty, ntz, vn, nf, nd);
    // pass z
    if (tid < I * I) {
      const int lx = tid % I, ly = tid / I;
      if (lx >= PO && lx < PO + O && ly >= PO && ly < PO + O) {
#pragma unroll
        for (int oz = 0; oz < O; ++oz) Xo[(oz * O + (ly - PO)) * O + (lx - PO)] = v[oz + PO];
      }
      double a[O];
      band_apply<PO, O>(op.me, v, a);
#pragma unroll
      for (int oz = 0; oz < O; ++oz) A[oz * S::SA + tid] = a[oz];
      band_apply<PO, O>(op.ke, v, a);
#pragma unroll
      for (int oz = 0; oz < O; ++oz) B[oz * S::SA + tid] = a[oz];
    }
    lds_barrier();
    // pass y
    double c1v[O], c2v[O];
    const bool act2 = tid < O * I;
    const int oz2 = tid / I, lx2 = tid % I;
    if (act2) {
      double w[I];
#pragma unroll
      for (int y = 0; y < I; ++y) w[y] = A[oz2 * S::SA + y * I + lx2];
      band_apply<PO, O>(op.me, w, c1v);
      band_apply<PO, O>(op.ke, w, c2v);
#pragma unroll
      for (int y = 0; y < I; ++y) w[y] = B[oz2 * S::SA + y * I + lx2];
      band_apply_acc<PO, O>(op.me, w, c2v);
    }
    lds_barrier();
    if (act2) {
#pragma unroll
      for (int oy = 0; oy < O; ++oy) {
        C1[oz2 * S::SC + oy * S::RS + lx2] = c1v[oy];
        C2[oz2 * S::SC + oy * S::RS + lx2] = c2v[oy];
      }
    }
    lds_barrier();
    // pass x
    if (tid < O * O) {
      const int oz = tid / O, oy = tid % O;
      double w[I], yv[O];
#pragma unroll
      for (int xx = 0; xx < I; ++xx) w[xx] = C1[oz * S::SC + oy * S::RS + xx];
      band_apply<PO, O>(op.ke, w, yv);
#pragma unroll
      for (int xx = 0; xx < I; ++xx) w[xx] = C2[oz * S::SC + oy * S::RS + xx];
      band_apply_acc<PO, O>(op.me, w, yv);
#pragma unroll
      for (int ox = 0; ox < O; ++ox) Y[(oz * O + oy) * S::YS + ox] = yv[ox];
    }
    lds_barrier();
    // epilogue on the owned nodes, x fastest
#pragma unroll
    for (int r = 0; r < NIT; ++r) {
      const int li = tid + 256 * r;
      const int ox = li % O, oy = (li / O) % O, oz = li / (O * O);
      const int gx = ox0 + ox, gy = oy0 + oy, gz = oz0 + oz;
      const bool ok = li < O * O * O && gx < P && gy < P && gz < P;
      const int lc = ok ? li : 0;
      const int cx = lc % O, cy = (lc / O) % O, cz = lc / (O * O);
      const double y = Y[(cz * O + cy) * S::YS + cx];
      const double xv = Xo[lc];
      const double rr = (pf_f[r] - y) * invd[(ox % PO) + PO * ((oy % PO) + PO * (oz % PO))];
      const size_t g = (size_t(gz) * P + gy) * P + gx;
      if (ok) {
        if (mode == kApply) out[g] = y;
        else if (mode == kResidual) out[g] = pf_f[r] - y;
        else if (mode == kCheb) xo[g] = xv + c1 * (xv - pf_d[r]) + c2 * rr;  // may overwrite x_prev
        else if (mode == kDinvApply) out[g] = -rr;                            // f = 0: -rr = D^-1 K x
        else { out[g] = y; acc += xv * y; }
      }
    }
    lds_barrier();  // LDS free for the next tile
#pragma unroll
    for (int z = 0; z < I; ++z) v[z] = vn[z];
#pragma unroll
    for (int r = 0; r < NIT; ++r) { pf_f[r] = nf[r]; pf_d[r] = nd[r]; }
    tx = ntx; ty = nty; tz = ntz;
    valid = nvalid;
  }
  if (mode == kApplyDot) {
    __syncthreads();
    double s = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// First Chebyshev step from a zero iterate: x = c2 D^-1 f, and x_prev = 0.
__global__ __launch_bounds__(256) void k_cheb_first(LevelOp op, const double *__restrict__ f,
                                                    double *__restrict__ xprev, double *__restrict__ x, double c2) {
  const int P = op.P, p = op.p;
  const size_t total = size_t(P) * P * P;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    const int kx = int(g % P) % p, ky = int((g / P) % P) % p, kz = int(g / (size_t(P) * P)) % p;
    const double D = op.dk[kx] * op.dm[ky] * op.dm[kz] + op.dm[kx] * op.dk[ky] * op.dm[kz] + op.dm[kx] * op.dm[ky] * op.dk[kz];
    x[g] = c2 * f[g] / D;
    xprev[g] = 0.0;
  }
}

// ----------------------------------------------------------------- transfers

// Restriction R = P^T as three separable passes on a tile of TE^3 coarse
// elements.  Along one axis, coarse node (e, j) collects the fine nodes s of
// coarse element e with weight w[s][j] and, for the vertex j = 0, those of
// element e - 1 with weight w[s][PC].  The tile reads the fine nodes of its
// elements plus one coarse element below.
template <int PF, int PC, int R, int TE>
struct XferShape {
  static constexpr int NS = R * PF;            // fine nodes per coarse element and axis
  static constexpr int CO = PC * TE;           // owned coarse nodes per axis
  static constexpr int NF = NS * (TE + 1);     // fine nodes read per axis (restriction)
  static constexpr int CI = PC * TE + 1;       // coarse nodes read per axis (prolongation)
  static constexpr int FO = NS * TE;           // owned fine nodes per axis (prolongation)
};

// 1-D restriction of a register column v (fine nodes of the tile, from one
// coarse element below) to the CO owned coarse nodes.
template <int PC, int NS, int CO, int NF>
__device__ __forceinline__ void restrict_col(const double *__restrict__ w, const double (&v)[NF], double (&o)[CO]) {
  constexpr int Q = PC + 1;
#pragma unroll
  for (int c = 0; c < CO; ++c) {
    const int ec = c / PC, j = c % PC;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NS; ++q) s += w[q * Q + j] * v[NS * (ec + 1) + q];
    if (j == 0) {
#pragma unroll
      for (int q = 0; q < NS; ++q) s += w[q * Q + PC] * v[NS * ec + q];
    }
    o[c] = s;
  }
}

template <int PF, int PC, int R, int TE>
__global__ __launch_bounds__(256) void k_restrict(Transfer tr, const double *__restrict__ rf, double *__restrict__ fc) {
  using S = XferShape<PF, PC, R, TE>;
  constexpr int NS = S::NS, CO = S::CO, NF = S::NF;
  static_assert(NF * NF <= 256 && NF * CO <= 256 && CO * CO <= 256, "restriction tile too large");
  __shared__ double G1[CO * NF * (NF + 1)];   // [cz][fy][fx]
  __shared__ double G2[CO * CO * (NF + 1)];   // [cz][cy][fx]
  __shared__ double Out[CO * CO * CO];        // [cz][cy][cx]
  const int Pf = tr.Pf, Pc = tr.Pc;
  const int tiles = (tr.nc + TE - 1) / TE;
  int t = blockIdx.x;
  const int tx = t % tiles;
  t /= tiles;
  const int ty = t % tiles;
  const int tz = t / tiles;
  const int tid = threadIdx.x;
  const int fx0 = NS * (tx * TE - 1), fy0 = NS * (ty * TE - 1), fz0 = NS * (tz * TE - 1);
  if (tid < NF * NF) {  // pass z: one fine (x, y) column per thread, lanes along x
    const int fx = tid % NF, fy = tid / NF;
    const int gx = wrapi(fx0 + fx, Pf), gy = wrapi(fy0 + fy, Pf);
    double v[NF], o[CO];
#pragma unroll
    for (int i = 0; i < NF; ++i) v[i] = rf[(size_t(wrapi(fz0 + i, Pf)) * Pf + gy) * Pf + gx];
    restrict_col<PC, NS, CO, NF>(tr.w, v, o);
#pragma unroll
    for (int c = 0; c < CO; ++c) G1[(c * NF + fy) * (NF + 1) + fx] = o[c];
  }
  __syncthreads();
  if (tid < CO * NF) {  // pass y
    const int fx = tid % NF, cz = tid / NF;
    double v[NF], o[CO];
#pragma unroll
    for (int i = 0; i < NF; ++i) v[i] = G1[(cz * NF + i) * (NF + 1) + fx];
    restrict_col<PC, NS, CO, NF>(tr.w, v, o);
#pragma unroll
    for (int c = 0; c < CO; ++c) G2[(cz * CO + c) * (NF + 1) + fx] = o[c];
  }
  __syncthreads();
  if (tid < CO * CO) {  // pass x
    const int cy = tid % CO, cz = tid / CO;
    double v[NF], o[CO];
#pragma unroll
    for (int i = 0; i < NF; ++i) v[i] = G2[(cz * CO + cy) * (NF + 1) + i];
    restrict_col<PC, NS, CO, NF>(tr.w, v, o);
#pragma unroll
    for (int c = 0; c < CO; ++c) Out[(cz * CO + cy) * CO + c] = o[c];
  }
  __syncthreads();
  for (int li = tid; li < CO * CO * CO; li += 256) {
    const int cx = li % CO, cy = (li / CO) % CO, cz = li / (CO * CO);
    const int gx = tx * CO + cx, gy = ty * CO + cy, gz = tz * CO + cz;
    if (gx < Pc && gy < Pc && gz < Pc) fc[(size_t(gz) * Pc + gy) * Pc + gx] = Out[li];
  }
}

// 1-D prolongation of a coarse register column (CI nodes from the tile's
// first coarse node) to the FO owned fine nodes.
template <int PC, int NS, int CI, int FO>
__device__ __forceinline__ void prolong_col(const double *__restrict__ w, const double (&v)[CI], double (&o)[FO]) {
  constexpr int Q = PC + 1;
#pragma unroll
  for (int f = 0; f < FO; ++f) {
    const int e = f / NS, s = f % NS;
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < Q; ++j) a += w[s * Q + j] * v[PC * e + j];
    o[f] = a;
  }
}

// xf += P ec on a tile of TE^3 coarse elements (three separable passes).
template <int PF, int PC, int R, int TE>
__global__ __launch_bounds__(256) void k_prolong_add(Transfer tr, const double *__restrict__ ec,
                                                     double *__restrict__ xf) {
  using S = XferShape<PF, PC, R, TE>;
  constexpr int NS = S::NS, CI = S::CI, FO = S::FO;
  static_assert(CI * CI <= 256 && CI * FO <= 256 && FO * FO <= 256, "prolongation tile too large");
  __shared__ double H1[FO * CI * (CI + 1)];   // [fz][cy][cx]
  __shared__ double H2[FO * FO * (CI + 1)];   // [fz][fy][cx]
  __shared__ double Out[FO * FO * FO];        // [fz][fy][fx]
  const int Pf = tr.Pf, Pc = tr.Pc;
  const int tiles = (tr.nc + TE - 1) / TE;
  int t = blockIdx.x;
  const int tx = t % tiles;
  t /= tiles;
  const int ty = t % tiles;
  const int tz = t / tiles;
  const int tid = threadIdx.x;
  const int cx0 = PC * TE * tx, cy0 = PC * TE * ty, cz0 = PC * TE * tz;
  constexpr int NIT = (FO * FO * FO + 255) / 256;
  double pf[NIT];  // fine values to update, fetched before the passes
#pragma unroll
  for (int r = 0; r < NIT; ++r) {
    const int li = tid + 256 * r;
    const int fx = li % FO, fy = (li / FO) % FO, fz = li / (FO * FO);
    const int gx = NS * TE * tx + fx, gy = NS * TE * ty + fy, gz = NS * TE * tz + fz;
    const bool ok = li < FO * FO * FO && gx < Pf && gy < Pf && gz < Pf;
    pf[r] = ok ? xf[(size_t(gz) * Pf + gy) * Pf + gx] : 0.0;
  }
  if (tid < CI * CI) {  // pass z
    const int cx = tid % CI, cy = tid / CI;
    const int gx = wrapi(cx0 + cx, Pc), gy = wrapi(cy0 + cy, Pc);
    double v[CI], o[FO];
#pragma unroll
    for (int i = 0; i < CI; ++i) v[i] = ec[(size_t(wrapi(cz0 + i, Pc)) * Pc + gy) * Pc + gx];
    prolong_col<PC, NS, CI, FO>(tr.w, v, o);
#pragma unroll
    for (int f = 0; f < FO; ++f) H1[(f * CI + cy) * (CI + 1) + cx] = o[f];
  }
  __syncthreads();
  if (tid < FO * CI) {  // pass y
    const int cx = tid % CI, fz = tid / CI;
    double v[CI], o[FO];
#pragma unroll
    for (int i = 0; i < CI; ++i) v[i] = H1[(fz * CI + i) * (CI + 1) + cx];
    prolong_col<PC, NS, CI, FO>(tr.w, v, o);
#pragma unroll
    for (int f = 0; f < FO; ++f) H2[(fz * FO + f) * (CI + 1) + cx] = o[f];
  }
  __syncthreads();
  if (tid < FO * FO) {  // pass x
    const int fy = tid % FO, fz = tid / FO;
    double v[CI], o[FO];
#pragma unroll
    for (int i = 0; i < CI; ++i) v[i] = H2[(fz * FO + fy) * (CI + 1) + i];
    prolong_col<PC, NS, CI, FO>(tr.w, v, o);
#pragma unroll
    for (int f = 0; f < FO; ++f) Out[(fz * FO + fy) * FO + f] = o[f];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NIT; ++r) {
    const int li = tid + 256 * r;
    const int fx = li % FO, fy = (li / FO) % FO, fz = li / (FO * FO);
    const int gx = NS * TE * tx + fx, gy = NS * TE * ty + fy, gz = NS * TE * tz + fz;
    if (li < FO * FO * FO && gx < Pf && gy < Pf && gz < Pf) xf[(size_t(gz) * Pf + gy) * Pf + gx] = pf[r] + Out[li];
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

// Tiles per block.  One: with several tiles per block the prefetch registers
// lower occupancy more than the overlap gains (measured).
static inline int apply_tpb(int) { return 1; }

template <int PO, int TE>
static int apply_impl(hipStream_t s, const LevelOp &op, const double *x, const double *f, double *out,
                      const double *d, double *xo, double c1, double c2, int mode, double *partial) {
  const int tiles = (op.n + TE - 1) / TE;
  const int nt = tiles * tiles * tiles;
  const int tpb = apply_tpb(tiles);
  const int nb = (nt + tpb - 1) / tpb;
  hipLaunchKernelGGL((k_apply<PO, TE, 1>), dim3(nb), dim3(256), 0, s, op, x, f, out, d, xo, c1, c2, mode, partial);
  return nb;
}

int launch_apply(hipStream_t s, const LevelOp &op, const double *x, const double *f, double *out,
                 const double *d, double *xo, double c1, double c2, int mode, double *partial) {
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
  const int tpb = apply_tpb(tiles);
  return (tiles * tiles * tiles + tpb - 1) / tpb;
}

void launch_cheb_first(hipStream_t s, const LevelOp &op, const double *f, double *d, double *x, double c2) {
  // d receives x_prev = 0
  const size_t tot = size_t(op.P) * op.P * op.P;
  hipLaunchKernelGGL(k_cheb_first, dim3(grid_for(tot)), dim3(256), 0, s, op, f, d, x, c2);
}
template <int PF, int PC, int R, int TE>
static void restrict_impl(hipStream_t s, const Transfer &tr, const double *in, double *out) {
  const int tiles = (tr.nc + TE - 1) / TE;
  hipLaunchKernelGGL((k_restrict<PF, PC, R, TE>), dim3(tiles * tiles * tiles), dim3(256), 0, s, tr, in, out);
}
template <int PF, int PC, int R, int TE>
static void prolong_impl(hipStream_t s, const Transfer &tr, const double *in, double *out) {
  const int tiles = (tr.nc + TE - 1) / TE;
  hipLaunchKernelGGL((k_prolong_add<PF, PC, R, TE>), dim3(tiles * tiles * tiles), dim3(256), 0, s, tr, in, out);
}

// Supported transfers: p 5 -> 3 and 3 -> 1 on one mesh, Q1 coarsening by 2 or 3.
int launch_transfer(hipStream_t s, const Transfer &tr, const double *in, double *out, bool restrict_) {
  if (tr.pf == 5 && tr.pc == 3 && tr.r == 1) {
    if (restrict_) restrict_impl<5, 3, 1, 2>(s, tr, in, out); else prolong_impl<5, 3, 1, 2>(s, tr, in, out);
  } else if (tr.pf == 3 && tr.pc == 1 && tr.r == 1) {
    if (restrict_) restrict_impl<3, 1, 1, 4>(s, tr, in, out); else prolong_impl<3, 1, 1, 5>(s, tr, in, out);
  } else if (tr.pf == 1 && tr.pc == 1 && tr.r == 2) {
    if (restrict_) restrict_impl<1, 1, 2, 7>(s, tr, in, out); else prolong_impl<1, 1, 2, 8>(s, tr, in, out);
  } else if (tr.pf == 1 && tr.pc == 1 && tr.r == 3) {
    if (restrict_) restrict_impl<1, 1, 3, 4>(s, tr, in, out); else prolong_impl<1, 1, 3, 5>(s, tr, in, out);
  } else {
    return -1;
  }
  return 0;
}
void launch_restrict(hipStream_t s, const Transfer &tr, const double *rf, double *fc) {
  launch_transfer(s, tr, rf, fc, true);
}
void launch_prolong_add(hipStream_t s, const Transfer &tr, const double *ec, double *xf) {
  launch_transfer(s, tr, ec, xf, false);
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
