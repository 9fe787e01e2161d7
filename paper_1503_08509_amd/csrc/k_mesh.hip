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

// Fixed-shape block sum for any block of whole waves (up to 8): shuffle
// tree inside each wave, then the wave sums in order.  The result is valid
// in thread 0.
__device__ __forceinline__ double block_sum_waves(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < int(blockDim.x >> 6); ++w) r += red[w];
  return r;
}

// ----------------------------------------------------------------- load

// Elements owning global node g along one axis (order p, n elements,
// periodic) and the node's local index in each: one, or two at a vertex
// (the element below first with local index p).
__device__ __forceinline__ int node_owners(int g, int p, int n, int (&e)[2], int (&k)[2]) {
  e[0] = g / p;
  k[0] = g - e[0] * p;
  if (k[0] != 0) return 1;
  e[1] = e[0] == 0 ? n - 1 : e[0] - 1;
  k[1] = p;
  return 2;
}

// b at node (gz, gy, gx): 4 pi sum over the 1..8 elements owning the node of
// sum_a C[E][a] g[ax][kx] g[ay][ky] g[az][kz] (gather form, no atomics),
// with per-configuration block partial sums of b (K blocks per
// configuration) for the compatibility projection.
template <int PO>
__global__ __launch_bounds__(512) void k_load(int n, int K, const double *__restrict__ Call,
                                              const double *__restrict__ gw, double *__restrict__ ball,
                                              double *__restrict__ partial) {
  constexpr int p = PO;
  __shared__ double red[8];
  const int P = p * n;
  const size_t total = size_t(P) * P * P;
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const double *C = Call + size_t(cfg) * n * n * n * 8;
  double *b = ball + size_t(cfg) * total;
  double acc = 0.0;
  (void)total;
  for (int row = kb; row < P * P; row += K) {   // one (gz, gy) row per pass, x along the threads
    const int gz = row / P, gy = row - gz * P;
    int ey[2], ky[2], ez[2], kz[2];
    const int ny = node_owners(gy, p, n, ey, ky), nz = node_owners(gz, p, n, ez, kz);
    for (int gx = threadIdx.x; gx < P; gx += blockDim.x) {
    const size_t g = size_t(row) * P + gx;
    int ex[2], kx[2];
    const int nx = node_owners(gx, p, n, ex, kx);
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
  }
  double t = block_sum_waves(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// v -= s * w1[kx] w1[ky] w1[kz] with s = scal[b] / V  (V = n^3 in element
// units) on configuration b: subtracts the uniform-background multiple of
// M 1.  Used on the load (compatibility) with scal = sum b.
template <int PO>
__global__ __launch_bounds__(512) void k_sub_mass_ones(int n, int K, const double *__restrict__ w1,
                                                       const double *__restrict__ scal, double *__restrict__ vall) {
  constexpr int p = PO;
  const int P = p * n;
  const size_t total = size_t(P) * P * P;
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  double *v = vall + size_t(cfg) * total;
  const double s = scal[cfg] / (double(n) * n * n);
  (void)total;
  for (int row = kb; row < P * P; row += K) {
    const int gz = row / P, gy = row - gz * P;
    const double wy = w1[gy % p], wz = w1[gz % p];
    for (int gx = threadIdx.x; gx < P; gx += blockDim.x) {
      const size_t g = size_t(row) * P + gx;
      v[g] -= s * w1[gx % p] * wy * wz;
    }
  }
}

// Per-configuration block partials of (M 1)^T v = sum w1 w1 w1 v (the
// integral of the FE field).
template <int PO>
__global__ __launch_bounds__(512) void k_mass_dot(int n, int K, const double *__restrict__ w1,
                                                  const double *__restrict__ vall, double *__restrict__ partial) {
  constexpr int p = PO;
  __shared__ double red[8];
  const int P = p * n;
  const size_t total = size_t(P) * P * P;
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const double *v = vall + size_t(cfg) * total;
  double acc = 0.0;
  (void)total;
  for (int row = kb; row < P * P; row += K) {
    const int gz = row / P, gy = row - gz * P;
    const double wy = w1[gy % p], wz = w1[gz % p];
    for (int gx = threadIdx.x; gx < P; gx += blockDim.x) acc += w1[gx % p] * wy * wz * v[size_t(row) * P + gx];
  }
  double t = block_sum_waves(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// v -= scal[b] / V on configuration b (constant shift; fixes int phi = 0).
__global__ __launch_bounds__(256) void k_sub_const(size_t per, int K, double invV, const double *__restrict__ scal,
                                                   double *__restrict__ vall) {
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  double *v = vall + size_t(cfg) * per;
  const double s = scal[cfg] * invV;
  for (size_t g = size_t(kb) * blockDim.x + threadIdx.x; g < per; g += size_t(K) * blockDim.x) v[g] -= s;
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

// An entry of op.dk / op.dm at a run-time local index, as a select over the
// compile-time indices: an indexed read of the by-value operator argument
// would copy the whole operator to scratch memory.
template <int PO, class T>
__device__ __forceinline__ T pick(const T (&v)[kMaxP], int k) {
  T r = v[0];
#pragma unroll
  for (int j = 1; j < PO; ++j) r = (k == j) ? v[j] : r;
  return r;
}

template <int PO, int TE, int NT = 256>
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
  static_assert(I * I <= NT && O * I <= NT && O * O <= NT, "tile columns must fit one pass of the block");
};

// Banded 1-D element-assembled operator on a column held in registers:
// out[o] = sum_j a[k][j] v[o + PO - k + j] (+ a[PO][j] v[o + j] for k = 0),
// k = o mod PO, with v indexed from one element below the first output.
// Every coefficient index is a compile-time constant, so the (wave-uniform)
// coefficients come from scalar registers.
template <int PO, int NOUT, class T>
__device__ __forceinline__ void band_apply(const T *__restrict__ a, const T (&v)[NOUT + PO + 1], T (&out)[NOUT]) {
  constexpr int Q1 = PO + 1;
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    const int k = o % PO;
    T s = T(0);
#pragma unroll
    for (int j = 0; j < Q1; ++j) s += a[k * Q1 + j] * v[o + PO - k + j];
    if (k == 0) {
#pragma unroll
      for (int j = 0; j < Q1; ++j) s += a[PO * Q1 + j] * v[o + j];
    }
    out[o] = s;
  }
}

template <int PO, int NOUT, class T>
__device__ __forceinline__ void band_apply_acc(const T *__restrict__ a, const T (&v)[NOUT + PO + 1], T (&out)[NOUT]) {
  T t[NOUT];
  band_apply<PO, NOUT>(a, v, t);
#pragma unroll
  for (int o = 0; o < NOUT; ++o) out[o] += t[o];
}

// Residual restricted in the operator's epilogue (p = 5 to p = 3 on the same
// elements, whole 2^3-element tiles): 1-D weights w[s][j] (fine node s of an
// element, coarse basis j, j = 3 the element's upper vertex) and the output
// of 7^3 partial coarse values per tile.
template <class T>
struct RestrictArgs {
  T w[5 * 4];
  T *part;
};

// 1-D partial restriction of the 10 fine nodes of a 2-element row to the 7
// coarse nodes they touch: (element ec, basis j < 3) for ec = 0, 1 and the
// upper vertex of element 1.  The lower vertex of element 0 still lacks the
// contribution of the element below, which the tile below supplies as its
// seventh value.
template <class T>
__device__ __forceinline__ void restrict_partial(const T *__restrict__ w, const T (&v)[10], T (&o)[7]) {
#pragma unroll
  for (int ec = 0; ec < 2; ++ec)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T s = T(0);
#pragma unroll
      for (int q = 0; q < 5; ++q) s += w[q * 4 + j] * v[5 * ec + q];
      if (j == 0 && ec == 1) {
#pragma unroll
        for (int q = 0; q < 5; ++q) s += w[q * 4 + 3] * v[q];
      }
      o[3 * ec + j] = s;
    }
  T s = T(0);
#pragma unroll
  for (int q = 0; q < 5; ++q) s += w[q * 4 + 3] * v[5 + q];
  o[6] = s;
}

// One tile of TE^3 elements per block: y = K x on the owned nodes, then the
// mode's epilogue.  The owned nodes of a tile are p*e + k, k < p, for its
// elements; the inputs reach one element below and one node above.
// Pass z: each thread streams one (x, y) column of the input from global
// memory and writes A = Mz x, B = Kz x; pass y: one (z, x) column of A and B
// gives C1 = My A and C2 = Ky A + My B; pass x: one (z, y) row of C1, C2
// gives y = Kx C1 + Mx C2; the epilogue then walks the owned nodes x-fastest.
// With RR (kResidual, PO = 5, TE = 2, whole tiles) the residual is not
// stored: the tile restricts it to 7^3 partial coarse values (RestrictArgs).
// NT threads per block (one per input column of the z pass: 384 for the
// 19^2 columns of a p = 6 tile of 2^3 elements).
template <class T, int PO, int TE, bool RR, int NT = 256>
__global__ __launch_bounds__(NT) void k_apply(LevelOpT<T> op, const T *__restrict__ x, const T *__restrict__ f,
                                               T *__restrict__ out, const T *xprev, T *xo, T c1, T c2, int mode,
                                               double *__restrict__ partial, T s0, RestrictArgs<T> ra,
                                               const T *__restrict__ cg) {
  static_assert(!RR || (PO == 5 && TE == 2), "the fused restriction covers p = 5 tiles of 2^3 elements");
  using S = ApplyShape<PO, TE, NT>;
  constexpr int O = S::O, I = S::I;
  static_assert(S::LDS * sizeof(T) >= 256 * sizeof(double), "the dot-product tree reuses the tile");
  __shared__ __align__(16) T lds[S::LDS];  // A, B; then C1, C2, Y; last the dot-product tree
  __shared__ T invd[PO * PO * PO];         // 1 / diag(K) by local node index
  // x on the owned nodes, from the z-pass columns; p = 6 reads it from global
  // memory in the epilogue instead (a tile then needs little enough LDS for
  // two blocks per compute unit)
  constexpr bool kXoLds = PO != 6;
  __shared__ T Xo[kXoLds ? O * O * O : 1];
  // p = 6: the band coefficients (2 x 49 values) come from the device copy
  // op.cg at wave-uniform addresses (scalar loads); read through the by-value
  // argument they make the compiler copy the whole operator to scratch
  // memory, and held in vector registers they spill
  constexpr bool kGlobalCoef = PO == 6;
  T *A = lds;
  T *B = lds + O * S::SA;
  T *C1 = lds;
  T *C2 = lds + O * S::SC;
  T *Y = lds + 2 * O * S::SC;
  const int P = op.P;
  const int tiles = (op.n + TE - 1) / TE;
  {  // configuration of this tile: every vector moves to its block
    const int tiles3 = tiles * tiles * tiles;
    const size_t off = size_t(blockIdx.x / tiles3) * P * P * P;
    if (RR) ra.part += size_t(blockIdx.x / tiles3) * tiles3 * 343;
    if (x) x += off;   // null in kChebZ2 mode
    if (f) f += off;
    if (out) out += off;
    if (xprev) xprev += off;
    if (xo) xo += off;
  }
  int tx, ty, tz;
  tile_coords(blockIdx.x % (tiles * tiles * tiles), tiles, tx, ty, tz);
  const int ox0 = tx * O, oy0 = ty * O, oz0 = tz * O;
  const int tid = threadIdx.x;

  // Epilogue operands of this thread's owned nodes, fetched now so their
  // latency hides behind the three passes.
  constexpr int NIT = (O * O * O + NT - 1) / NT;
  const bool zstart = (mode == kChebZ2);   // input columns are s0 D^-1 f
  const bool cheb = (mode == kCheb) || (mode == kChebDot);
  const bool need_f = (mode == kResidual) || cheb || zstart || (mode == kChebZ3);
  const bool need_d = cheb && (c1 != T(0)) && (xprev != nullptr);   // null x_prev reads as zero
  const bool need_x = !kXoLds && !zstart && (cheb || mode == kChebZ3 || mode == kApplyDot);
  for (int i = tid; i < PO * PO * PO; i += NT) {
    const int kx = i % PO, ky = (i / PO) % PO, kz = i / (PO * PO);
    const T dkx = pick<PO>(op.dk, kx), dky = pick<PO>(op.dk, ky), dkz = pick<PO>(op.dk, kz);
    const T dmx = pick<PO>(op.dm, kx), dmy = pick<PO>(op.dm, ky), dmz = pick<PO>(op.dm, kz);
    invd[i] = T(1) / (dkx * dmy * dmz + dmx * dky * dmz + dmx * dmy * dkz);
  }
  const T *cme = op.me, *cke = op.ke;
  if constexpr (kGlobalCoef) {
    cme = cg;
    cke = cg + (PO + 1) * (PO + 1);
  }
  // Addresses: a block-uniform 64-bit tile base plus 32-bit offsets inside
  // the tile (at most O P^2 + O P + O < 2^31 for every supported n).
  const size_t tbase = (size_t(oz0) * P + oy0) * P + ox0;
  T pf_f[NIT], pf_d[NIT], pf_x[kXoLds ? 1 : NIT];
#pragma unroll
  for (int r = 0; r < NIT; ++r) {
    const int li = tid + NT * r;
    const int ox = li % O, oy = (li / O) % O, oz = li / (O * O);
    const bool ok = li < O * O * O && ox0 + ox < P && oy0 + oy < P && oz0 + oz < P;
    const size_t g = tbase + unsigned(ok ? (oz * P + oy) * P + ox : 0);
    pf_f[r] = (ok && need_f) ? f[g] : T(0);
    pf_d[r] = (ok && need_d) ? xprev[g] : T(0);
    if constexpr (!kXoLds) pf_x[r] = (ok && need_x) ? x[g] : T(0);
  }

  // pass z
  if (zstart) __syncthreads();   // the z pass scales by the inverse diagonal
  if (tid < I * I) {
    const int lx = tid % I, ly = tid / I;
    const int gx = wrapi(ox0 - PO + lx, P), gy = wrapi(oy0 - PO + ly, P);
    const T *col = (zstart ? f : x) + (size_t(gy) * P + gx);   // this thread's (x, y) column
    const size_t P2 = size_t(P) * P;
    T v[I];
#pragma unroll
    for (int z = 0; z < I; ++z) v[z] = col[size_t(wrapi(oz0 - PO + z, P)) * P2];   // plane offset is block-uniform
    if (zstart) {
      // tile origins are multiples of PO, so the local node index of input
      // (lx, ly, z) along each axis is its tile offset mod PO
      const T *id = invd + (lx % PO) + PO * (ly % PO);
#pragma unroll
      for (int z = 0; z < I; ++z) v[z] *= s0 * id[PO * PO * (z % PO)];
    }
    if (kXoLds && lx >= PO && lx < PO + O && ly >= PO && ly < PO + O) {
#pragma unroll
      for (int oz = 0; oz < O; ++oz) Xo[(oz * O + (ly - PO)) * O + (lx - PO)] = v[oz + PO];
    }
    T a[O];
    band_apply<PO, O>(cme, v, a);
#pragma unroll
    for (int oz = 0; oz < O; ++oz) A[oz * S::SA + tid] = a[oz];
    band_apply<PO, O>(cke, v, a);
#pragma unroll
    for (int oz = 0; oz < O; ++oz) B[oz * S::SA + tid] = a[oz];
  }
  __syncthreads();
  // pass y
  T c1v[O], c2v[O];
  const bool act2 = tid < O * I;
  const int oz2 = tid / I, lx2 = tid % I;
  if (act2) {
    T v[I];
#pragma unroll
    for (int y = 0; y < I; ++y) v[y] = A[oz2 * S::SA + y * I + lx2];
    band_apply<PO, O>(cme, v, c1v);
    band_apply<PO, O>(cke, v, c2v);
#pragma unroll
    for (int y = 0; y < I; ++y) v[y] = B[oz2 * S::SA + y * I + lx2];
    band_apply_acc<PO, O>(cme, v, c2v);
  }
  __syncthreads();
  if (act2) {
#pragma unroll
    for (int oy = 0; oy < O; ++oy) {
      C1[oz2 * S::SC + oy * S::RS + lx2] = c1v[oy];
      C2[oz2 * S::SC + oy * S::RS + lx2] = c2v[oy];
    }
  }
  __syncthreads();
  // pass x
  if (tid < O * O) {
    const int oz = tid / O, oy = tid % O;
    T v[I], yv[O];
#pragma unroll
    for (int xx = 0; xx < I; ++xx) v[xx] = C1[oz * S::SC + oy * S::RS + xx];
    band_apply<PO, O>(cke, v, yv);
#pragma unroll
    for (int xx = 0; xx < I; ++xx) v[xx] = C2[oz * S::SC + oy * S::RS + xx];
    band_apply_acc<PO, O>(cme, v, yv);
#pragma unroll
    for (int ox = 0; ox < O; ++ox) Y[(oz * O + oy) * S::YS + ox] = yv[ox];
  }
  __syncthreads();
  if (RR) {
    // r on the owned nodes into Xo (x itself is not needed here), then three
    // separable partial restrictions: x rows, y columns, z columns.
#pragma unroll
    for (int r = 0; r < NIT; ++r) {
      const int li = tid + NT * r;
      if (li < O * O * O) {
        const int cx = li % O, cy = (li / O) % O, cz = li / (O * O);
        Xo[li] = pf_f[r] - Y[(cz * O + cy) * S::YS + cx];
      }
    }
    __syncthreads();
    T *R1 = lds;              // [oz][oy][7]
    T *R2 = lds + O * O * 7;  // [oz][cy][cx]
    T v[10], o[7];
    if (tid < O * O) {
      const int oz = tid / O, oy = tid % O;
#pragma unroll
      for (int i = 0; i < 10; ++i) v[i] = Xo[(oz * O + oy) * O + i];
      restrict_partial<T>(ra.w, v, o);
#pragma unroll
      for (int k = 0; k < 7; ++k) R1[(oz * O + oy) * 7 + k] = o[k];
    }
    __syncthreads();
    if (tid < O * 7) {
      const int oz = tid / 7, cx = tid % 7;
#pragma unroll
      for (int i = 0; i < 10; ++i) v[i] = R1[(oz * O + i) * 7 + cx];
      restrict_partial<T>(ra.w, v, o);
#pragma unroll
      for (int k = 0; k < 7; ++k) R2[(oz * 7 + k) * 7 + cx] = o[k];
    }
    __syncthreads();
    if (tid < 49) {
      const int cy = tid / 7, cx = tid % 7;
#pragma unroll
      for (int i = 0; i < 10; ++i) v[i] = R2[(i * 7 + cy) * 7 + cx];
      restrict_partial<T>(ra.w, v, o);
      T *dst = ra.part + size_t((tz * tiles + ty) * tiles + tx) * 343 + cy * 7 + cx;
#pragma unroll
      for (int k = 0; k < 7; ++k) dst[k * 49] = o[k];
    }
    return;
  }
  // epilogue on the owned nodes, x fastest: every result and address first,
  // then the stores back to back (a store whose registers the next one
  // reused would make it wait for the earlier store)
  double acc = 0.0;
  T res[NIT];
  T *dst[NIT];
  T *const base = (cheb || zstart || mode == kChebZ3) ? xo : out;   // xo may overwrite x_prev
#pragma unroll
  for (int r = 0; r < NIT; ++r) {
    const int li = tid + NT * r;
    const int ox = li % O, oy = (li / O) % O, oz = li / (O * O);
    const bool ok = li < O * O * O && ox0 + ox < P && oy0 + oy < P && oz0 + oz < P;
    const int lc = ok ? li : 0;
    const int cx = lc % O, cy = (lc / O) % O, cz = lc / (O * O);
    const T y = Y[(cz * O + cy) * S::YS + cx];
    const T id = invd[(ox % PO) + PO * ((oy % PO) + PO * (oz % PO))];
    T xv;
    if constexpr (kXoLds) xv = Xo[lc];
    else xv = zstart ? pf_f[r] * (s0 * id) : pf_x[r];   // the z pass's input: s0 D^-1 f, else x
    const T rr = (pf_f[r] - y) * id;
    T v;
    if (mode == kApply || mode == kApplyDot) v = y;
    else if (mode == kResidual) v = pf_f[r] - y;
    else if (cheb || zstart) v = xv + c1 * (xv - pf_d[r]) + c2 * rr;
    else if (mode == kChebZ3) v = xv + c1 * (xv - s0 * id * pf_f[r]) + c2 * rr;
    else v = -rr;                                                          // kDinvApply (f = 0): D^-1 K x
    if (ok && mode == kApplyDot) acc += double(xv) * double(y);
    if (ok && mode == kChebDot) acc += double(v) * double(pf_f[r]);
    res[r] = v;
    asm volatile("" : "+v"(res[r]));   // computed here, in registers of its own
    dst[r] = ok ? base + (tbase + unsigned((oz * P + oy) * P + ox)) : nullptr;
  }
#pragma unroll
  for (int r = 0; r < NIT; ++r)
    if (dst[r]) *dst[r] = res[r];
  if (mode == kApplyDot || mode == kChebDot) {
    __syncthreads();  // every thread is done with Y before the tree reuses it
    double s;
    if constexpr (NT == 256) s = block_sum(acc, reinterpret_cast<double *>(lds));
    else s = block_sum_waves(acc, reinterpret_cast<double *>(lds));   // whole waves, not a power of two
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// First Chebyshev step from a zero iterate: x = c2 D^-1 f (the next step
// reads its zero x_prev as a null pointer).
template <class T>
__global__ __launch_bounds__(256) void k_cheb_first(LevelOpT<T> op, int K, const T *__restrict__ fall,
                                                    T *__restrict__ xall, T c2) {
  const int P = op.P, p = op.p;
  const size_t total = size_t(P) * P * P;
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const T *f = fall + size_t(cfg) * total;
  T *x = xall + size_t(cfg) * total;
  for (size_t g = size_t(kb) * blockDim.x + threadIdx.x; g < total; g += size_t(K) * blockDim.x) {
    const int kx = int(g % P) % p, ky = int((g / P) % P) % p, kz = int(g / (size_t(P) * P)) % p;
    const T D = op.dk[kx] * op.dm[ky] * op.dm[kz] + op.dm[kx] * op.dk[ky] * op.dm[kz] + op.dm[kx] * op.dm[ky] * op.dk[kz];
    x[g] = c2 * f[g] / D;
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
template <int PC, int NS, int CO, int NF, class T>
__device__ __forceinline__ void restrict_col(const T *__restrict__ w, const T (&v)[NF], T (&o)[CO]) {
  constexpr int Q = PC + 1;
#pragma unroll
  for (int c = 0; c < CO; ++c) {
    const int ec = c / PC, j = c % PC;
    T s = T(0);
#pragma unroll
    for (int q = 0; q < NS; ++q) s += w[q * Q + j] * v[NS * (ec + 1) + q];
    if (j == 0) {
#pragma unroll
      for (int q = 0; q < NS; ++q) s += w[q * Q + PC] * v[NS * ec + q];
    }
    o[c] = s;
  }
}

// NT threads per block, one per fine input column of the z pass (384 for the
// 18^2 columns of a p = 6 tile of 2^3 coarse elements).
template <class T, int PF, int PC, int R, int TE, int NT = 256>
__global__ __launch_bounds__(NT) void k_restrict(TransferT<T> tr, const T *__restrict__ rf, T *__restrict__ fc) {
  using S = XferShape<PF, PC, R, TE>;
  constexpr int NS = S::NS, CO = S::CO, NF = S::NF;
  static_assert(NF * NF <= NT && NF * CO <= NT && CO * CO <= NT, "restriction tile too large");
  __shared__ T G1[CO * NF * (NF + 1)];   // [cz][fy][fx]
  __shared__ T G2[CO * CO * (NF + 1)];   // [cz][cy][fx]
  __shared__ T Out[CO * CO * CO];        // [cz][cy][cx]
  const int Pf = tr.Pf, Pc = tr.Pc;
  const int tiles = (tr.nc + TE - 1) / TE;
  const int cfg = blockIdx.x / (tiles * tiles * tiles);
  rf += size_t(cfg) * Pf * Pf * Pf;
  fc += size_t(cfg) * Pc * Pc * Pc;
  int t = blockIdx.x % (tiles * tiles * tiles);
  const int tx = t % tiles;
  t /= tiles;
  const int ty = t % tiles;
  const int tz = t / tiles;
  const int tid = threadIdx.x;
  const int fx0 = NS * (tx * TE - 1), fy0 = NS * (ty * TE - 1), fz0 = NS * (tz * TE - 1);
  if (tid < NF * NF) {  // pass z: one fine (x, y) column per thread, lanes along x
    const int fx = tid % NF, fy = tid / NF;
    const int gx = wrapi(fx0 + fx, Pf), gy = wrapi(fy0 + fy, Pf);
    T v[NF], o[CO];
#pragma unroll
    for (int i = 0; i < NF; ++i) v[i] = rf[(size_t(wrapi(fz0 + i, Pf)) * Pf + gy) * Pf + gx];
    restrict_col<PC, NS, CO, NF>(tr.w, v, o);
#pragma unroll
    for (int c = 0; c < CO; ++c) G1[(c * NF + fy) * (NF + 1) + fx] = o[c];
  }
  __syncthreads();
  if (tid < CO * NF) {  // pass y
    const int fx = tid % NF, cz = tid / NF;
    T v[NF], o[CO];
#pragma unroll
    for (int i = 0; i < NF; ++i) v[i] = G1[(cz * NF + i) * (NF + 1) + fx];
    restrict_col<PC, NS, CO, NF>(tr.w, v, o);
#pragma unroll
    for (int c = 0; c < CO; ++c) G2[(cz * CO + c) * (NF + 1) + fx] = o[c];
  }
  __syncthreads();
  if (tid < CO * CO) {  // pass x
    const int cy = tid % CO, cz = tid / CO;
    T v[NF], o[CO];
#pragma unroll
    for (int i = 0; i < NF; ++i) v[i] = G2[(cz * CO + cy) * (NF + 1) + i];
    restrict_col<PC, NS, CO, NF>(tr.w, v, o);
#pragma unroll
    for (int c = 0; c < CO; ++c) Out[(cz * CO + cy) * CO + c] = o[c];
  }
  __syncthreads();
  for (int li = tid; li < CO * CO * CO; li += NT) {
    const int cx = li % CO, cy = (li / CO) % CO, cz = li / (CO * CO);
    const int gx = tx * CO + cx, gy = ty * CO + cy, gz = tz * CO + cz;
    if (gx < Pc && gy < Pc && gz < Pc) fc[(size_t(gz) * Pc + gy) * Pc + gx] = Out[li];
  }
}

// 1-D prolongation of a coarse register column (CI nodes from the tile's
// first coarse node) to the FO owned fine nodes.
template <int PC, int NS, int CI, int FO, class T>
__device__ __forceinline__ void prolong_col(const T *__restrict__ w, const T (&v)[CI], T (&o)[FO]) {
  constexpr int Q = PC + 1;
#pragma unroll
  for (int f = 0; f < FO; ++f) {
    const int e = f / NS, s = f % NS;
    T a = T(0);
#pragma unroll
    for (int j = 0; j < Q; ++j) a += w[s * Q + j] * v[PC * e + j];
    o[f] = a;
  }
}

// xf += P ec on a tile of TE^3 coarse elements (three separable passes).
template <class T, int PF, int PC, int R, int TE>
__global__ __launch_bounds__(256) void k_prolong_add(TransferT<T> tr, const T *__restrict__ ec, T *__restrict__ xf) {
  using S = XferShape<PF, PC, R, TE>;
  constexpr int NS = S::NS, CI = S::CI, FO = S::FO;
  static_assert(CI * CI <= 256 && CI * FO <= 256 && FO * FO <= 256, "prolongation tile too large");
  __shared__ T H1[FO * CI * (CI + 1)];   // [fz][cy][cx]
  __shared__ T H2[FO * FO * (CI + 1)];   // [fz][fy][cx]
  __shared__ T Out[FO * FO * FO];        // [fz][fy][fx]
  const int Pf = tr.Pf, Pc = tr.Pc;
  const int tiles = (tr.nc + TE - 1) / TE;
  const int cfg = blockIdx.x / (tiles * tiles * tiles);
  ec += size_t(cfg) * Pc * Pc * Pc;
  xf += size_t(cfg) * Pf * Pf * Pf;
  int t = blockIdx.x % (tiles * tiles * tiles);
  const int tx = t % tiles;
  t /= tiles;
  const int ty = t % tiles;
  const int tz = t / tiles;
  const int tid = threadIdx.x;
  const int cx0 = PC * TE * tx, cy0 = PC * TE * ty, cz0 = PC * TE * tz;
  constexpr int NIT = (FO * FO * FO + 255) / 256;
  T pf[NIT];  // fine values to update, fetched before the passes
#pragma unroll
  for (int r = 0; r < NIT; ++r) {
    const int li = tid + 256 * r;
    const int fx = li % FO, fy = (li / FO) % FO, fz = li / (FO * FO);
    const int gx = NS * TE * tx + fx, gy = NS * TE * ty + fy, gz = NS * TE * tz + fz;
    const bool ok = li < FO * FO * FO && gx < Pf && gy < Pf && gz < Pf;
    pf[r] = ok ? xf[(size_t(gz) * Pf + gy) * Pf + gx] : T(0);
  }
  if (tid < CI * CI) {  // pass z
    const int cx = tid % CI, cy = tid / CI;
    const int gx = wrapi(cx0 + cx, Pc), gy = wrapi(cy0 + cy, Pc);
    T v[CI], o[FO];
#pragma unroll
    for (int i = 0; i < CI; ++i) v[i] = ec[(size_t(wrapi(cz0 + i, Pc)) * Pc + gy) * Pc + gx];
    prolong_col<PC, NS, CI, FO>(tr.w, v, o);
#pragma unroll
    for (int f = 0; f < FO; ++f) H1[(f * CI + cy) * (CI + 1) + cx] = o[f];
  }
  __syncthreads();
  if (tid < FO * CI) {  // pass y
    const int cx = tid % CI, fz = tid / CI;
    T v[CI], o[FO];
#pragma unroll
    for (int i = 0; i < CI; ++i) v[i] = H1[(fz * CI + i) * (CI + 1) + cx];
    prolong_col<PC, NS, CI, FO>(tr.w, v, o);
#pragma unroll
    for (int f = 0; f < FO; ++f) H2[(fz * FO + f) * (CI + 1) + cx] = o[f];
  }
  __syncthreads();
  if (tid < FO * FO) {  // pass x
    const int fy = tid % FO, fz = tid / FO;
    T v[CI], o[FO];
#pragma unroll
    for (int i = 0; i < CI; ++i) v[i] = H2[(fz * FO + fy) * (CI + 1) + i];
    prolong_col<PC, NS, CI, FO>(tr.w, v, o);
#pragma unroll
    for (int f = 0; f < FO; ++f) Out[(fz * FO + fy) * FO + f] = o[f];
  }
  __syncthreads();
  // every address and sum first, then the stores back to back: a store
  // whose registers are reused by the next one would make it wait
  T *dst[NIT];
#pragma unroll
  for (int r = 0; r < NIT; ++r) {
    const int li = tid + 256 * r;
    const int fx = li % FO, fy = (li / FO) % FO, fz = li / (FO * FO);
    const int gx = NS * TE * tx + fx, gy = NS * TE * ty + fy, gz = NS * TE * tz + fz;
    const bool ok = li < FO * FO * FO && gx < Pf && gy < Pf && gz < Pf;
    dst[r] = ok ? xf + ((size_t(gz) * Pf + gy) * Pf + gx) : nullptr;
    pf[r] += Out[ok ? li : 0];
    asm volatile("" : "+v"(pf[r]));   // keep each sum in its own registers, computed here
  }
#pragma unroll
  for (int r = 0; r < NIT; ++r)
    if (dst[r]) *dst[r] = pf[r];
}

// ----------------------------------------------------------------- coarse solve

// Exact periodic solve on the coarsest Q_pc level by fast diagonalisation:
// x = (V (x) V (x) V) diag(1 / (l_i + l_j + l_k)) (V (x) V (x) V)^T f with the
// constant mode (l = 0) dropped.  One block; nc^3 <= kCoarseMax.
constexpr int kCoarseMax = 4096;
template <class T>
__global__ __launch_bounds__(256) void k_coarse_solve(int Pn, const double *__restrict__ V, const double *__restrict__ lam,
                                                      const T *__restrict__ f, T *__restrict__ x) {
  __shared__ double a[kCoarseMax];
  __shared__ double b[kCoarseMax];
  const int N3 = Pn * Pn * Pn;
  f += size_t(blockIdx.x) * N3;   // one block per configuration
  x += size_t(blockIdx.x) * N3;
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
    x[i] = T(s);
  }
}

// ----------------------------------------------------------------- vectors

// Per-configuration vector kernels: configuration b = blockIdx / K owns
// entries [b per, (b + 1) per); block partials land at partial[blockIdx].
__global__ __launch_bounds__(256) void k_dot(size_t per, int K, const double *__restrict__ a,
                                             const double *__restrict__ b, double *__restrict__ partial) {
  __shared__ double red[256];
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  a += size_t(cfg) * per;
  b += size_t(cfg) * per;
  double acc = 0.0;
  for (size_t i = size_t(kb) * blockDim.x + threadIdx.x; i < per; i += size_t(K) * blockDim.x)
    acc += a[i] * b[i];
  double t = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// x += alpha_b p; r -= alpha_b q; partial of r.r
// r_out = r_in - alpha_b q and block partials of r_out . r_out (r_in may be
// r_out, or the right side in the first iteration).
// r_out = r_in - alpha q, block partials of |r_out|^2; with rf, also a
// float32 copy of r_out (the mixed-precision V-cycle's right side)
__global__ __launch_bounds__(256) void k_r_update(size_t per, int K, const double *__restrict__ alphas,
                                                  const double *__restrict__ q, const double *r_in,
                                                  double *r_out, float *__restrict__ rf,
                                                  double *__restrict__ partial) {
  __shared__ double red[256];
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const size_t o = size_t(cfg) * per;
  q += o; r_in += o; r_out += o;
  if (rf) rf += o;
  const double alpha = alphas[cfg];
  double acc = 0.0;
  // four elements per thread and pass: every load first, then the stores
  constexpr int U = 4;
  const size_t stride = size_t(K) * blockDim.x;
  for (size_t i0 = size_t(kb) * blockDim.x + threadIdx.x; i0 < per; i0 += U * stride) {
    double qv[U], rv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = i0 + u * stride;
      const bool ok = i < per;
      qv[u] = ok ? q[i] : 0.0;
      rv[u] = ok ? r_in[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      rv[u] -= alpha * qv[u];
      acc += rv[u] * rv[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = i0 + u * stride;
      if (i < per) {
        r_out[i] = rv[u];
        if (rf) rf[i] = float(rv[u]);
      }
    }
  }
  double t = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// The iterate's update of the previous iteration, deferred to the pass that
// forms the next direction: x = x + alpha_b p (x = alpha_b p when xinit is
// 0: x is not read), then p = z + beta_b p.  z float64 or float32.
template <class ZT>
__global__ __launch_bounds__(256) void k_xp_update(size_t per, int K, const double *__restrict__ alphas,
                                                   const double *__restrict__ betas, const ZT *__restrict__ z,
                                                   double *__restrict__ p, double *__restrict__ x, int xinit) {
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const size_t o = size_t(cfg) * per;
  z += o; p += o; x += o;
  const double alpha = alphas[cfg], beta = betas[cfg];
  const size_t i = size_t(kb) * blockDim.x + threadIdx.x;   // one element per thread
  if (i < per) {
    const double pv = p[i], zv = double(z[i]);
    const double xv = xinit ? x[i] : 0.0;
    x[i] = xv + alpha * pv;
    p[i] = zv + beta * pv;
  }
}

// p = z (first direction; p is not read).  z float64 or float32.
template <class ZT>
__global__ __launch_bounds__(256) void k_p_init(size_t per, int K, const ZT *__restrict__ z, double *__restrict__ p) {
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const size_t i = size_t(kb) * blockDim.x + threadIdx.x;
  if (i < per) p[size_t(cfg) * per + i] = double(z[size_t(cfg) * per + i]);
}

// x = x + alpha_b p (x = alpha_b p when xinit is 0): the last iteration's
// update after the loop has stopped.
__global__ __launch_bounds__(256) void k_x_final(size_t per, int K, const double *__restrict__ alphas,
                                                 const double *__restrict__ p, double *__restrict__ x, int xinit) {
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const size_t o = size_t(cfg) * per;
  const double alpha = alphas[cfg];
  const size_t i = size_t(kb) * blockDim.x + threadIdx.x;
  if (i < per) x[o + i] = (xinit ? x[o + i] : 0.0) + alpha * p[o + i];
}

__global__ __launch_bounds__(256) void k_scale(size_t n, double s, const double *__restrict__ a, double *__restrict__ b) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    b[i] = s * a[i];
}

// Copy as a kernel (usable inside a captured graph, unlike a memcpy node).
__global__ __launch_bounds__(256) void k_copy_f64(size_t n, const double *__restrict__ a, double *__restrict__ b) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) b[i] = a[i];
}

// Fast-diagonalisation solve, middle step: coefficient (i, j, k) of each
// configuration (x index i fastest) divided by lam_i + lam_j + lam_k; the
// constant mode (i = j = k = i0) is set to zero.
__global__ __launch_bounds__(256) void k_fdm_scale(size_t total, int P, int i0, const double *__restrict__ lam,
                                                   double *__restrict__ X) {
  const size_t P3 = size_t(P) * P * P;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    const size_t l = g % P3;
    const int i = int(l % P), j = int((l / P) % P), k = int(l / (size_t(P) * P));
    X[g] = (i == i0 && j == i0 && k == i0) ? 0.0 : X[g] / (lam[i] + lam[j] + lam[k]);
  }
}

// Deterministic pseudo-random fill (power iteration start vector).
__global__ __launch_bounds__(256) void k_hash_fill(size_t n, uint32_t seed, double *__restrict__ v) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    uint32_t h = uint32_t(i) * 2654435761u ^ seed;
    h ^= h >> 16; h *= 0x7feb352du; h ^= h >> 15; h *= 0x846ca68bu; h ^= h >> 16;
    v[i] = double(h) / 4294967296.0 - 0.5;
  }
}

// Mixed precision: the float64 PCG hands its residual to a float32 V-cycle
// and takes the preconditioned residual back.
__global__ __launch_bounds__(256) void k_to_f32(size_t n, const double *__restrict__ a, float *__restrict__ b) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    b[i] = float(a[i]);
}

// Block partials of z.r (first gridDim slots) and z.q (next gridDim),
// float64 sums of a float32 z, per configuration.
__global__ __launch_bounds__(256) void k_dot2_f32(size_t per, int K, const float *__restrict__ z,
                                                  const double *__restrict__ r, const double *__restrict__ q,
                                                  double *__restrict__ partial) {
  __shared__ double red[256];
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const size_t o = size_t(cfg) * per;
  z += o;
  r += o;
  if (q) q += o;
  double a = 0.0, b = 0.0;
  for (size_t i = size_t(kb) * blockDim.x + threadIdx.x; i < per; i += size_t(K) * blockDim.x) {
    const double zi = double(z[i]);
    a += zi * r[i];
    if (q) b += zi * q[i];
  }
  const double ta = block_sum(a, red);
  const double tb = block_sum(b, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = ta;
    partial[gridDim.x + blockIdx.x] = tb;
  }
}

// PCG scalars, one thread per configuration, on arrays of nb values:
//   kPcgStart  act = (bn2 > 0); beta = 0; rz = rzn
//   kPcgAlpha  alpha = act ? rz / pq : 0
//   kPcgResid  rel = sqrt(rr) / sqrt(bn2) (0 if bn2 = 0); act &= rel > rtol
//   kPcgBeta   beta = act ? rzn / rz : 0; rz = rzn
//   kPcgBetaPR beta = act ? -alpha zq / rz : 0; rz = rzn (flexible form)
__global__ __launch_bounds__(64) void k_pcg_scalars(int nb, int step, double rtol, PcgScalars s) {
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    switch (step) {
      case kPcgStart:
        s.act[b] = s.bn2[b] > 0.0 ? 1.0 : 0.0;
        s.beta[b] = 0.0;
        s.rz[b] = s.rzn[b];
        break;
      case kPcgAlpha: s.alpha[b] = s.act[b] != 0.0 ? s.rz[b] / s.pq[b] : 0.0; break;
      case kPcgResid: {
        const double rel = s.bn2[b] > 0.0 ? sqrt(s.rr[b]) / sqrt(s.bn2[b]) : 0.0;
        s.rel[b] = rel;
        if (!(rel > rtol)) s.act[b] = 0.0;
        break;
      }
      case kPcgBeta:
        s.beta[b] = s.act[b] != 0.0 ? s.rzn[b] / s.rz[b] : 0.0;
        s.rz[b] = s.rzn[b];
        break;
      default:
        s.beta[b] = s.act[b] != 0.0 ? -s.alpha[b] * s.zq[b] / s.rz[b] : 0.0;
        s.rz[b] = s.rzn[b];
        break;
    }
  }
}

// Second stage of every reduction: block b sums the K partials of
// configuration b in a fixed order into out[b].
__global__ __launch_bounds__(256) void k_sum_partials(int K, const double *__restrict__ partial, double *__restrict__ out) {
  __shared__ double red[256];
  partial += size_t(blockIdx.x) * K;
  // eight independent sums per thread keep eight loads in flight (one block
  // may read tens of thousands of partials); fixed order, so repeatable
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int i = threadIdx.x;
  for (; i + 7 * 256 < K; i += 8 * 256) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += partial[i + u * 256];
  }
  for (; i < K; i += 256) a[0] += partial[i];
  const double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  double t = block_sum(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// ----------------------------------------------------------------- launchers

namespace {
inline int grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  return int(g < kRedBlocks ? (g == 0 ? 1 : g) : kRedBlocks);
}
}  // namespace

int seg_blocks(int nb, size_t per) {
  const size_t cap = nb >= kRedBlocks ? 1 : size_t(kRedBlocks / nb);
  size_t g = (per + 255) / 256;
  if (g < 1) g = 1;
  return int(g < cap ? g : cap);
}
int row_blocks(int nb, int P) {
  const int cap = nb >= kRowBlocks ? 1 : kRowBlocks / nb;
  return P * P < cap ? P * P : cap;
}

int row_threads(int P) { return P >= 512 ? 512 : 64 * ((P + 63) / 64); }
int launch_load(hipStream_t s, int nb, int n, int p, const double *C, const double *gw, double *b, double *partial) {
  if (p != 5) return -1;
  const int K = row_blocks(nb, p * n);
  hipLaunchKernelGGL(k_load<5>, dim3(nb * K), dim3(row_threads(p * n)), 0, s, n, K, C, gw, b, partial);
  return K;
}
void launch_sum_partials(hipStream_t s, int K, const double *partial, double *out, int nb) {
  hipLaunchKernelGGL(k_sum_partials, dim3(nb), dim3(256), 0, s, K, partial, out);
}
int launch_sub_mass_ones(hipStream_t s, int nb, int n, int p, const double *w1, const double *scal, double *v) {
  const int K = row_blocks(nb, p * n);
  const dim3 g(nb * K), b(row_threads(p * n));
  switch (p) {
    case 3: hipLaunchKernelGGL(k_sub_mass_ones<3>, g, b, 0, s, n, K, w1, scal, v); return 0;
    case 4: hipLaunchKernelGGL(k_sub_mass_ones<4>, g, b, 0, s, n, K, w1, scal, v); return 0;
    case 5: hipLaunchKernelGGL(k_sub_mass_ones<5>, g, b, 0, s, n, K, w1, scal, v); return 0;
    case 6: hipLaunchKernelGGL(k_sub_mass_ones<6>, g, b, 0, s, n, K, w1, scal, v); return 0;
    default: return -1;
  }
}
int launch_mass_dot(hipStream_t s, int nb, int n, int p, const double *w1, const double *v, double *partial) {
  const int K = row_blocks(nb, p * n);
  const dim3 g(nb * K), b(row_threads(p * n));
  switch (p) {
    case 3: hipLaunchKernelGGL(k_mass_dot<3>, g, b, 0, s, n, K, w1, v, partial); return K;
    case 4: hipLaunchKernelGGL(k_mass_dot<4>, g, b, 0, s, n, K, w1, v, partial); return K;
    case 5: hipLaunchKernelGGL(k_mass_dot<5>, g, b, 0, s, n, K, w1, v, partial); return K;
    case 6: hipLaunchKernelGGL(k_mass_dot<6>, g, b, 0, s, n, K, w1, v, partial); return K;
    default: return -1;
  }
}
void launch_sub_const(hipStream_t s, int nb, size_t per, double invV, const double *scal, double *v) {
  const int K = seg_blocks(nb, per);
  hipLaunchKernelGGL(k_sub_const, dim3(nb * K), dim3(256), 0, s, per, K, invV, scal, v);
}

template <class T, int PO, int TE, int NT = 256>
static int apply_impl(hipStream_t s, int nb, const LevelOpT<T> &op, const T *x, const T *f, T *out, const T *d, T *xo,
                      T c1, T c2, int mode, double *partial, T s0) {
  const int tiles = (op.n + TE - 1) / TE;
  const int K = tiles * tiles * tiles;
  if (PO == 6 && !op.cg) return -1;   // the order-6 operator reads its coefficients from op.cg
  hipLaunchKernelGGL((k_apply<T, PO, TE, false, NT>), dim3(nb * K), dim3(NT), 0, s, op, x, f, out, d, xo, c1, c2,
                     mode, partial, s0, RestrictArgs<T>{}, op.cg);
  return K;
}

// Partial coarse values of the tiles (7^3 each) summed per coarse node: own
// tile, and for a node on a tile's lower face (local index 0 along an axis)
// also the upper-vertex value (index 6) of the tile below, in a fixed order.
template <class T>
__global__ __launch_bounds__(256) void k_restrict_sum(int Pc, int tiles, int K, const T *__restrict__ partall,
                                                      T *__restrict__ fcall) {
  const size_t total = size_t(Pc) * Pc * Pc;
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const T *part = partall + size_t(cfg) * tiles * tiles * tiles * 343;
  T *fc = fcall + size_t(cfg) * total;
  for (size_t g = size_t(kb) * blockDim.x + threadIdx.x; g < total; g += size_t(K) * blockDim.x) {
    const int gx = int(g % Pc), gy = int((g / Pc) % Pc), gz = int(g / (size_t(Pc) * Pc));
    int t[3][2], k[3][2], nn[3];
    const int gg[3] = {gx, gy, gz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      t[a][0] = gg[a] / 6;
      k[a][0] = gg[a] % 6;
      nn[a] = 1;
      if (k[a][0] == 0) {
        t[a][1] = t[a][0] == 0 ? tiles - 1 : t[a][0] - 1;
        k[a][1] = 6;
        nn[a] = 2;
      }
    }
    T s = T(0);
    for (int iz = 0; iz < nn[2]; ++iz)
      for (int iy = 0; iy < nn[1]; ++iy)
        for (int ix = 0; ix < nn[0]; ++ix) {
          const size_t tile = (size_t(t[2][iz]) * tiles + t[1][iy]) * tiles + t[0][ix];
          s += part[tile * 343 + (k[2][iz] * 7 + k[1][iy]) * 7 + k[0][ix]];
        }
    fc[g] = s;
  }
}

template <class T>
int launch_apply_restrict(hipStream_t s, int nb, const LevelOpT<T> &op, const TransferT<T> &tr, const T *x,
                          const T *f, T *part) {
  if (op.p != 5 || tr.pf != 5 || tr.pc != 3 || tr.r != 1 || op.n % 2 != 0) return -1;
  RestrictArgs<T> ra{};
  for (int i = 0; i < 20; ++i) ra.w[i] = tr.w[i];
  ra.part = part;
  const int tiles = op.n / 2;
  const int K = tiles * tiles * tiles;
  hipLaunchKernelGGL((k_apply<T, 5, 2, true>), dim3(nb * K), dim3(256), 0, s, op, x, f, nullptr, nullptr, nullptr,
                     T(0), T(0), int(kResidual), nullptr, T(0), ra, op.cg);
  return K;
}

template <class T>
void launch_restrict_sum(hipStream_t s, int nb, int n, const T *part, T *fc) {
  const int Pc = 3 * n;
  const int K = seg_blocks(nb, size_t(Pc) * Pc * Pc);
  hipLaunchKernelGGL(k_restrict_sum<T>, dim3(nb * K), dim3(256), 0, s, Pc, n / 2, K, part, fc);
}

template <class T>
int launch_apply(hipStream_t s, int nb, const LevelOpT<T> &op, const T *x, const T *f, T *out, const T *d, T *xo,
                 T c1, T c2, int mode, double *partial, T s0) {
  switch (op.p) {
    case 1: return apply_impl<T, 1, 8>(s, nb, op, x, f, out, d, xo, c1, c2, mode, partial, s0);
    case 2: return apply_impl<T, 2, 4>(s, nb, op, x, f, out, d, xo, c1, c2, mode, partial, s0);
    case 3: return apply_impl<T, 3, 4>(s, nb, op, x, f, out, d, xo, c1, c2, mode, partial, s0);
    case 4: return apply_impl<T, 4, 2>(s, nb, op, x, f, out, d, xo, c1, c2, mode, partial, s0);
    case 5: return apply_impl<T, 5, 2>(s, nb, op, x, f, out, d, xo, c1, c2, mode, partial, s0);
    case 6: return apply_impl<T, 6, 2, 384>(s, nb, op, x, f, out, d, xo, c1, c2, mode, partial, s0);
    default: return -1;
  }
}

int apply_blocks(const LevelOp &op) {
  int TE = op.p == 1 ? 8 : op.p == 2 ? 4 : op.p == 3 ? 4 : 2;
  int tiles = (op.n + TE - 1) / TE;
  return tiles * tiles * tiles;
}

template <class T>
void launch_cheb_first(hipStream_t s, int nb, const LevelOpT<T> &op, const T *f, T *x, T c2) {
  const size_t per = size_t(op.P) * op.P * op.P;
  const int K = seg_blocks(nb, per);
  hipLaunchKernelGGL(k_cheb_first<T>, dim3(nb * K), dim3(256), 0, s, op, K, f, x, c2);
}
template <class T, int PF, int PC, int R, int TE, int NT = 256>
static void restrict_impl(hipStream_t s, int nb, const TransferT<T> &tr, const T *in, T *out) {
  const int tiles = (tr.nc + TE - 1) / TE;
  hipLaunchKernelGGL((k_restrict<T, PF, PC, R, TE, NT>), dim3(nb * tiles * tiles * tiles), dim3(NT), 0, s, tr, in,
                     out);
}
template <class T, int PF, int PC, int R, int TE>
static void prolong_impl(hipStream_t s, int nb, const TransferT<T> &tr, const T *in, T *out) {
  const int tiles = (tr.nc + TE - 1) / TE;
  hipLaunchKernelGGL((k_prolong_add<T, PF, PC, R, TE>), dim3(nb * tiles * tiles * tiles), dim3(256), 0, s, tr, in,
                     out);
}

// Supported transfers: p 5 -> 3 and 3 -> 1 on one mesh, Q1 coarsening by 2 or 3.
template <class T>
int launch_transfer(hipStream_t s, int nb, const TransferT<T> &tr, const T *in, T *out, bool restrict_) {
  if (tr.pf == 5 && tr.pc == 3 && tr.r == 1) {
    if (restrict_) restrict_impl<T, 5, 3, 1, 2>(s, nb, tr, in, out);
    else prolong_impl<T, 5, 3, 1, 3>(s, nb, tr, in, out);
  } else if (tr.pf == 4 && tr.pc == 3 && tr.r == 1) {
    if (restrict_) restrict_impl<T, 4, 3, 1, 2>(s, nb, tr, in, out);
    else prolong_impl<T, 4, 3, 1, 3>(s, nb, tr, in, out);
  } else if (tr.pf == 6 && tr.pc == 3 && tr.r == 1) {
    if (restrict_) restrict_impl<T, 6, 3, 1, 2, 384>(s, nb, tr, in, out);
    else prolong_impl<T, 6, 3, 1, 2>(s, nb, tr, in, out);
  } else if (tr.pf == 3 && tr.pc == 1 && tr.r == 1) {
    if (restrict_) restrict_impl<T, 3, 1, 1, 4>(s, nb, tr, in, out);
    else prolong_impl<T, 3, 1, 1, 5>(s, nb, tr, in, out);
  } else if (tr.pf == 1 && tr.pc == 1 && tr.r == 2) {
    if (restrict_) restrict_impl<T, 1, 1, 2, 7>(s, nb, tr, in, out);
    else prolong_impl<T, 1, 1, 2, 8>(s, nb, tr, in, out);
  } else if (tr.pf == 1 && tr.pc == 1 && tr.r == 3) {
    if (restrict_) restrict_impl<T, 1, 1, 3, 4>(s, nb, tr, in, out);
    else prolong_impl<T, 1, 1, 3, 5>(s, nb, tr, in, out);
  } else {
    return -1;
  }
  return 0;
}
template <class T>
void launch_coarse_solve(hipStream_t s, int nb, int Pn, const double *V, const double *lam, const T *f, T *x) {
  hipLaunchKernelGGL(k_coarse_solve<T>, dim3(nb), dim3(256), 0, s, Pn, V, lam, f, x);
}

#define FEP3M_MESH_INSTANTIATE(T)                                                                                   \
  template int launch_apply<T>(hipStream_t, int, const LevelOpT<T> &, const T *, const T *, T *, const T *, T *, T, \
                               T, int, double *, T);                                                                \
  template void launch_cheb_first<T>(hipStream_t, int, const LevelOpT<T> &, const T *, T *, T);                     \
  template int launch_transfer<T>(hipStream_t, int, const TransferT<T> &, const T *, T *, bool);                    \
  template int launch_apply_restrict<T>(hipStream_t, int, const LevelOpT<T> &, const TransferT<T> &, const T *,       \
                                        const T *, T *);                                                              \
  template void launch_restrict_sum<T>(hipStream_t, int, int, const T *, T *);                                       \
  template void launch_coarse_solve<T>(hipStream_t, int, int, const double *, const double *, const T *, T *);
FEP3M_MESH_INSTANTIATE(double)
FEP3M_MESH_INSTANTIATE(float)
#undef FEP3M_MESH_INSTANTIATE

void launch_to_f32(hipStream_t s, size_t n, const double *a, float *b) {
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(256), 0, s, n, a, b);
}
int launch_dot2_f32(hipStream_t s, int nb, size_t per, const float *z, const double *r, const double *q,
                    double *partial) {
  const int K = seg_blocks(nb, per);
  hipLaunchKernelGGL(k_dot2_f32, dim3(nb * K), dim3(256), 0, s, per, K, z, r, q, partial);
  return K;
}
void launch_pcg_scalars(hipStream_t s, int nb, int step, double rtol, const PcgScalars &sc) {
  hipLaunchKernelGGL(k_pcg_scalars, dim3(1), dim3(64), 0, s, nb, step, rtol, sc);
}
int launch_dot(hipStream_t s, int nb, size_t per, const double *a, const double *b, double *partial) {
  const int K = seg_blocks(nb, per);
  hipLaunchKernelGGL(k_dot, dim3(nb * K), dim3(256), 0, s, per, K, a, b, partial);
  return K;
}
int launch_r_update(hipStream_t s, int nb, size_t per, const double *alphas, const double *q, const double *r_in,
                    double *r_out, double *partial, float *rf) {
  const int K = seg_blocks(nb, per);
  hipLaunchKernelGGL(k_r_update, dim3(nb * K), dim3(256), 0, s, per, K, alphas, q, r_in, r_out, rf, partial);
  return K;
}
template <class ZT>
void launch_xp_update(hipStream_t s, int nb, size_t per, const double *alphas, const double *betas, const ZT *z,
                      double *p, double *x, bool xinit) {
  const int K = int((per + 255) / 256);
  hipLaunchKernelGGL(k_xp_update<ZT>, dim3(nb * K), dim3(256), 0, s, per, K, alphas, betas, z, p, x, xinit ? 1 : 0);
}
template void launch_xp_update<double>(hipStream_t, int, size_t, const double *, const double *, const double *,
                                       double *, double *, bool);
template void launch_xp_update<float>(hipStream_t, int, size_t, const double *, const double *, const float *,
                                      double *, double *, bool);
template <class ZT>
void launch_p_init(hipStream_t s, int nb, size_t per, const ZT *z, double *p) {
  const int K = int((per + 255) / 256);
  hipLaunchKernelGGL(k_p_init<ZT>, dim3(nb * K), dim3(256), 0, s, per, K, z, p);
}
template void launch_p_init<double>(hipStream_t, int, size_t, const double *, double *);
template void launch_p_init<float>(hipStream_t, int, size_t, const float *, double *);
void launch_x_final(hipStream_t s, int nb, size_t per, const double *alphas, const double *p, double *x,
                    bool xinit) {
  const int K = int((per + 255) / 256);
  hipLaunchKernelGGL(k_x_final, dim3(nb * K), dim3(256), 0, s, per, K, alphas, p, x, xinit ? 1 : 0);
}
void launch_scale(hipStream_t s, size_t n, double sc, const double *a, double *b) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(256), 0, s, n, sc, a, b);
}
void launch_fdm_scale(hipStream_t s, size_t total, int P, int i0, const double *lam, double *X) {
  hipLaunchKernelGGL(k_fdm_scale, dim3(grid_for(total)), dim3(256), 0, s, total, P, i0, lam, X);
}
void launch_copy_f64(hipStream_t s, size_t n, const double *a, double *b) {
  hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(n)), dim3(256), 0, s, n, a, b);
}
void launch_hash_fill(hipStream_t s, size_t n, uint32_t seed, double *v) {
  hipLaunchKernelGGL(k_hash_fill, dim3(grid_for(n)), dim3(256), 0, s, n, seed, v);
}

}  // namespace fep3m
