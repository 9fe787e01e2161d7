// Particle-side kernels: periodic wrap and element binning, a deterministic
// counting sort by element, per-element screen moments, the near-pair 1/R
// sum, interpolation of the mesh field at the charges, and the energy.
//
// Positions are kept as g = n * frac(x / L) in element units: element
// e = floor(g) (clamped to n - 1) and local offset u = g - e - 1/2.
#include "kernels.hpp"
#include "pair_segments.hpp"

namespace fep3m {

__device__ __forceinline__ double block_sum_p(double v, double *red) {
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

// ----------------------------------------------------------------- binning

// Wrap, bin and count; K blocks per configuration, block (b, k) over the
// charges off[b] .. off[b+1]-1, which fall in elements b n^3 + e.
// Non-finite inputs raise flags[0] and are binned to the configuration's
// element 0 so every index stays in bounds.  Block partials of sum Q and
// sum |Q| go to partial[blockIdx] and partial[gridDim.x + blockIdx].
__global__ __launch_bounds__(256) void k_bin(int64_t N, int K, const int *__restrict__ off,
                                             const double *__restrict__ x, const double *__restrict__ Q, double L,
                                             int n, int box, double *__restrict__ gtmp, int *__restrict__ elem,
                                             int *__restrict__ slot, int *__restrict__ count, int *__restrict__ flags,
                                             double *__restrict__ partial) {
  __shared__ double red[256];
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const int64_t hi = off[cfg + 1];
  const int base = cfg * n * n * n;
  double sq = 0.0, sa = 0.0;
  for (int64_t i = off[cfg] + int64_t(kb) * blockDim.x + threadIdx.x; i < hi; i += int64_t(K) * blockDim.x) {
    int e[3];
    bool ok = true;
    double gv[3];
    for (int k = 0; k < 3; ++k) {
      const double xv = x[3 * i + k];
      if (!isfinite(xv)) ok = false;
      if (box && !(xv > 0.0 && xv < L)) atomicOr(flags, 2);   // outside the box (the run is refused)
      double s = xv / L;
      s = s - floor(s);
      double t = s * double(n);
      double ef = floor(t);
      if (ef > double(n - 1)) ef = double(n - 1);
      if (!(ef >= 0.0 && ef <= double(n - 1))) {  // NaN from an overflowing x / L
        ok = false;
        ef = 0.0;
      }
      gv[k] = t;
      e[k] = int(ef);
    }
    const double q = Q[i];
    if (!isfinite(q)) ok = false;
    if (!ok) {
      atomicOr(flags, 1);
      e[0] = e[1] = e[2] = 0;
      gv[0] = gv[1] = gv[2] = 0.5;
    }
    for (int k = 0; k < 3; ++k) gtmp[k * N + i] = gv[k];
    const int E = base + e[0] + n * (e[1] + n * e[2]);
    elem[i] = E;
    slot[i] = atomicAdd(count + E, 1);
    sq += ok ? q : 0.0;
    sa += ok ? fabs(q) : 0.0;
  }
  double t1 = block_sum_p(sq, red);
  double t2 = block_sum_p(sa, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = t1;
    partial[gridDim.x + blockIdx.x] = t2;
  }
}

// Exclusive scan of count[0..M) into start[0..M]; also the largest count.
// Exclusive scan of element counts (start[0..M], start[M] = total) and their
// maximum, in three passes: per-tile sums and maxima, a one-block scan of
// the tile sums, and a per-tile rescan with the tile's offset.  A tile is
// 256 threads x 8 consecutive counts.
constexpr int kScanPer = 8;
constexpr int kScanTile = 256 * kScanPer;

__device__ __forceinline__ void load8(const int *__restrict__ a, int M, int i0, int (&v)[kScanPer]) {
  if (i0 + kScanPer <= M) {
    const int4 p = *reinterpret_cast<const int4 *>(a + i0), q = *reinterpret_cast<const int4 *>(a + i0 + 4);
    v[0] = p.x; v[1] = p.y; v[2] = p.z; v[3] = p.w; v[4] = q.x; v[5] = q.y; v[6] = q.z; v[7] = q.w;
  } else {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) v[k] = i0 + k < M ? a[i0 + k] : 0;
  }
}

// exclusive block scan of one value per thread (256 threads); returns the total in *tot
__device__ __forceinline__ int block_exscan256(int v, int *sh, int *tot) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {   // inclusive Hillis-Steele scan
    const int u = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += u;
    __syncthreads();
  }
  const int inc = sh[t];
  *tot = sh[255];
  __syncthreads();
  return inc - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(int M, const int *__restrict__ count, int *__restrict__ bsum,
                                                     int *__restrict__ bmax) {
  __shared__ int ss[256], sm[256];
  const int t = threadIdx.x;
  int v[kScanPer];
  load8(count, M, blockIdx.x * kScanTile + t * kScanPer, v);
  int s = 0, m = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) { s += v[k]; m = max(m, v[k]); }
  ss[t] = s;
  sm[t] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) { ss[t] += ss[t + off]; sm[t] = max(sm[t], sm[t + off]); }
    __syncthreads();
  }
  if (t == 0) { bsum[blockIdx.x] = ss[0]; bmax[blockIdx.x] = sm[0]; }
}

// one block: exclusive scan of the B tile sums in place, start[M] = total,
// maxcount[0] = the largest count
__global__ __launch_bounds__(256) void k_scan_top(int B, int M, int *__restrict__ bsum, const int *__restrict__ bmax,
                                                  int *__restrict__ start, int *__restrict__ maxcount) {
  __shared__ int sh[256];
  const int t = threadIdx.x;
  const int chunk = (B + 255) / 256;
  const int b0 = min(B, t * chunk), b1 = min(B, b0 + chunk);
  int s = 0, m = 0;
  for (int i = b0; i < b1; ++i) { s += bsum[i]; m = max(m, bmax[i]); }
  int tot;
  int run = block_exscan256(s, sh, &tot);
  for (int i = b0; i < b1; ++i) { const int v = bsum[i]; bsum[i] = run; run += v; }
  sh[t] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) sh[t] = max(sh[t], sh[t + off]);
    __syncthreads();
  }
  if (t == 0) { start[M] = tot; maxcount[0] = sh[0]; }
}

__global__ __launch_bounds__(256) void k_scan_down(int M, const int *__restrict__ count, const int *__restrict__ boff,
                                                   int *__restrict__ start) {
  __shared__ int sh[256];
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * kScanTile + t * kScanPer;
  int v[kScanPer];
  load8(count, M, i0, v);
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) s += v[k];
  int tot;
  int run = boff[blockIdx.x] + block_exscan256(s, sh, &tot);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (i0 + k < M) start[i0 + k] = run;
    run += v[k];
  }
}

__global__ __launch_bounds__(256) void k_scatter(int64_t N, const int *__restrict__ elem, const int *__restrict__ slot,
                                                 const int *__restrict__ start, int *__restrict__ tmp) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x)
    tmp[start[elem[i]] + slot[i]] = int(i);
}

// Stable order inside each element: the rank of caller index i among its
// element's indices.  Gathers the sorted positions and charges.
__global__ __launch_bounds__(256) void k_rank(int64_t N, const int *__restrict__ tmp, const int *__restrict__ elem,
                                              const int *__restrict__ start, const double *__restrict__ gtmp,
                                              const double *__restrict__ Q, int *__restrict__ perm,
                                              double *__restrict__ sg, double *__restrict__ sQ) {
  for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < N; s += int64_t(gridDim.x) * blockDim.x) {
    const int i = tmp[s];
    const int E = elem[i];
    const int b = start[E], e = start[E + 1];
    int rank = 0;
    for (int j = b; j < e; ++j) rank += (tmp[j] < i);
    const int pos = b + rank;
    perm[pos] = i;
    for (int k = 0; k < 3; ++k) sg[k * N + pos] = gtmp[k * N + i];
    sQ[pos] = Q[i];
  }
}

// ----------------------------------------------------------------- moments

// C[E][a] = sum_{j in E} Q_j u_j^a, a = ax + 2 ay + 4 az (element units).
__global__ __launch_bounds__(256) void k_moments(int n, int MT, int64_t N, const int *__restrict__ start,
                                                 const double *__restrict__ sg, const double *__restrict__ sQ,
                                                 double *__restrict__ C) {
  const int M = n * n * n;
  for (int E = blockIdx.x * blockDim.x + threadIdx.x; E < MT; E += gridDim.x * blockDim.x) {
    const int El = E % M;
    const int ex = El % n, ey = (El / n) % n, ez = El / (n * n);
    double c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    auto add = [&](double q, double gx, double gy, double gz) {
      const double ux = gx - ex - 0.5, uy = gy - ey - 0.5, uz = gz - ez - 0.5;
      c[0] += q;
      c[1] += q * ux;
      c[2] += q * uy;
      c[3] += q * ux * uy;
      c[4] += q * uz;
      c[5] += q * ux * uz;
      c[6] += q * uy * uz;
      c[7] += q * ux * uy * uz;
    };
    // four charges' loads in flight before they are summed (a heavy
    // element's chain of dependent loads sets the kernel's time); the sum
    // runs over the charges in order either way
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
    for (int a = 0; a < 8; ++a) C[size_t(E) * 8 + a] = c[a];
  }
}

// ----------------------------------------------------------------- pair sum

// One wavefront per target element.  Sources are the charges of the
// (2 NSR + 1)^3 element block, walked as up to 2 (2 NSR + 1)^2 contiguous
// sorted segments (rows along x, split where the row wraps the periodic
// boundary); every lane takes a strided share of the flattened source list
// and accumulates for a chunk of up to 8 targets, then the wave reduces.
// Displacements are formed in the target's unwrapped frame in element
// units, so no minimum-image test is needed (n >= 2 NSR + 1).
// With FORCE the same pass also accumulates sum_j Q_j (g_j - g_i) / r^3
// (fpair, 3 x N sorted), the pair part of dU/dg_i divided by Q_i.
// One chunk of nt <= NT targets starting at sorted slot t0: every lane
// walks its strided share of the block's sources and accumulates for all NT
// targets in registers; the wave then reduces.
// 1 / sqrt(x) for a positive normal x: the hardware estimate refined by one
// Newton-Raphson step y <- y (3 - x y^2) / 2, written as y + y e / 2 with
// e = 1 - x y^2 (one step squares the estimate's relative error).
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

template <int NSR, bool FORCE, int NT>
__device__ __forceinline__ void pair_chunk(const PairSegments<NSR> &seg, int total, int lane, int64_t N, int t0,
                                           int nt, double nd, const double *__restrict__ sg,
                                           const double *__restrict__ sQ, double *__restrict__ phip,
                                           double *__restrict__ fpair) {
  double tx[NT], ty[NT], tz[NT], acc[NT], fx[NT], fy[NT], fz[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const int ti = t0 + (k < nt ? k : 0);
    tx[k] = sg[ti]; ty[k] = sg[N + ti]; tz[k] = sg[2 * N + ti];
    acc[k] = 0.0;
    fx[k] = fy[k] = fz[k] = 0.0;
  }
  int sp = 0;
  for (int f = lane; f < total; f += 64) {
    while (f >= seg.so[sp + 1]) ++sp;
    const int j = seg.sb[sp] + (f - seg.so[sp]);
    const int pk = seg.ss[sp];
    const double shx = double(seg.shift(pk, 0)) * nd, shy = double(seg.shift(pk, 1)) * nd,
                 shz = double(seg.shift(pk, 2)) * nd;
    const double jx = sg[j] + shx, jy = sg[N + j] + shy, jz = sg[2 * N + j] + shz;
    const double qj = sQ[j];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      // slots k >= nt repeat the first target and are discarded at the end;
      // the self pair gets r^2 = 2^1000, so its terms (below 2^-500) vanish
      // in the sums
      const double dx = jx - tx[k], dy = jy - ty[k], dz = jz - tz[k];
      double r2 = dx * dx + dy * dy + dz * dz;
      r2 = (j == t0 + k) ? 0x1p1000 : r2;
      const double ri = rsqrt_pos(r2);
      const double qr = qj * ri;
      acc[k] += qr;
      if (FORCE) {
        const double qr3 = qr * (ri * ri);
        fx[k] += qr3 * dx;
        fy[k] += qr3 * dy;
        fz[k] += qr3 * dz;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    acc[k] = v;
    if (FORCE) {
      double a = fx[k], b = fy[k], c = fz[k];
      for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
        c += __shfl_xor(c, off, 64);
      }
      fx[k] = a; fy[k] = b; fz[k] = c;
    }
  }
  if (lane == 0) {
    for (int k = 0; k < nt; ++k) {
      phip[t0 + k] = acc[k];
      if (FORCE) {
        fpair[t0 + k] = fx[k];
        fpair[N + t0 + k] = fy[k];
        fpair[2 * N + t0 + k] = fz[k];
      }
    }
  }
}

template <int NSR, bool FORCE>
__global__ __launch_bounds__(64) void k_pair(int n, int64_t N, const int *__restrict__ start,
                                             const double *__restrict__ sg, const double *__restrict__ sQ,
                                             double *__restrict__ phip, double *__restrict__ fpair) {
  __shared__ PairSegments<NSR> seg;
  const int lane = threadIdx.x;
  const int E = blockIdx.x;
  const int tb = start[E], te = start[E + 1];
  if (tb == te) return;  // uniform over the (single-wave) block
  const int M = n * n * n;
  const int total = build_segments<NSR>(seg, E % M, n, start + (E / M) * M, lane, 64);
  const double nd = double(n);
  // chunk width per pass: 8 while more than 4 targets remain, then 4 or 2,
  // so that sparsely occupied elements do not compute empty target slots
  for (int t0 = tb; t0 < te;) {
    const int rem = te - t0;
    if (rem > 4) {
      pair_chunk<NSR, FORCE, 8>(seg, total, lane, N, t0, min(rem, 8), nd, sg, sQ, phip, fpair);
      t0 += 8;
    } else if (rem > 2) {
      pair_chunk<NSR, FORCE, 4>(seg, total, lane, N, t0, rem, nd, sg, sQ, phip, fpair);
      t0 += 4;
    } else {
      pair_chunk<NSR, FORCE, 2>(seg, total, lane, N, t0, rem, nd, sg, sQ, phip, fpair);
      t0 += 2;
    }
  }
}

// Load-balanced form: work items (element, first target) of up to `titem`
// targets each, taken from a shared counter by persistent one-wave blocks
// until the list is exhausted (every wave reaches the exit test).  Heavy
// elements split into several items; per-target arithmetic is the same as
// in k_pair, so the results are identical.
__global__ __launch_bounds__(256) void k_items_count(int MT, int titem, const int *__restrict__ start,
                                                     int *__restrict__ nit) {
  for (int E = blockIdx.x * blockDim.x + threadIdx.x; E < MT; E += gridDim.x * blockDim.x)
    nit[E] = (start[E + 1] - start[E] + titem - 1) / titem;
}
__global__ __launch_bounds__(256) void k_items_fill(int MT, int titem, const int *__restrict__ start,
                                                    const int *__restrict__ item_start, int2 *__restrict__ items) {
  for (int E = blockIdx.x * blockDim.x + threadIdx.x; E < MT; E += gridDim.x * blockDim.x) {
    const int b = item_start[E], k = item_start[E + 1] - b;
    for (int j = 0; j < k; ++j) items[b + j] = make_int2(E, start[E] + j * titem);
  }
}
__global__ __launch_bounds__(64) void k_fill_int(int count, int value, int *__restrict__ p) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = value;
}

template <int NSR, bool FORCE>
__global__ __launch_bounds__(64) void k_pair_queue(int n, int64_t N, const int *__restrict__ start,
                                                   const int2 *__restrict__ items, const int *__restrict__ nitems,
                                                   int *__restrict__ counter, int titem,
                                                   const double *__restrict__ sg, const double *__restrict__ sQ,
                                                   double *__restrict__ phip, double *__restrict__ fpair) {
  __shared__ PairSegments<NSR> seg;
  __shared__ int cur;
  const int lane = threadIdx.x;
  const int total_items = *nitems;
  const int M = n * n * n;
  const double nd = double(n);
  for (;;) {
    if (lane == 0) cur = atomicAdd(counter, 1);
    __syncthreads();
    const int it = cur;
    if (it >= total_items) break;   // uniform over the wave
    const int2 w = items[it];
    const int E = w.x, te = min(w.y + titem, start[E + 1]);
    const int total = build_segments<NSR>(seg, E % M, n, start + (E / M) * M, lane, 64);
    for (int t0 = w.y; t0 < te;) {
      const int rem = te - t0;
      if (rem > 4) {
        pair_chunk<NSR, FORCE, 8>(seg, total, lane, N, t0, min(rem, 8), nd, sg, sQ, phip, fpair);
        t0 += 8;
      } else if (rem > 2) {
        pair_chunk<NSR, FORCE, 4>(seg, total, lane, N, t0, rem, nd, sg, sQ, phip, fpair);
        t0 += 4;
      } else {
        pair_chunk<NSR, FORCE, 2>(seg, total, lane, N, t0, rem, nd, sg, sQ, phip, fpair);
        t0 += 2;
      }
    }
    __syncthreads();   // the segment list and cur are rewritten for the next item
  }
}

// Phi_m at each sorted charge: sum_m W_E[m] u_m(u_i) (W = phi - Psi of its
// element, element units) by sum factorisation; then the combined
// potential (Phi_p + Phi_m) / h, scattered to caller order.
template <int PO>
__global__ __launch_bounds__(256) void k_interp(int n, int64_t N, int nb, const int *__restrict__ off, double inv_h,
                                                GllBasis bas, const double *__restrict__ sg,
                                                const double *__restrict__ Wel,
                                                const double *__restrict__ phip, const int *__restrict__ perm,
                                                double *__restrict__ phim_s, double *__restrict__ phi_s,
                                                double *__restrict__ Phi) {
  constexpr int Q1 = PO + 1;
  for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < N; s += int64_t(gridDim.x) * blockDim.x) {
    double l[3][Q1];
    int e[3];
    for (int k = 0; k < 3; ++k) {
      const double g = sg[k * N + s];
      double ef = floor(g);
      if (ef > double(n - 1)) ef = double(n - 1);
      e[k] = int(ef);
      const double u = g - ef - 0.5;
#pragma unroll
      for (int a = 0; a < Q1; ++a) {
        double v = bas.w[a];
#pragma unroll
        for (int j = 0; j < Q1; ++j)
          if (j != a) v *= (u - bas.x[j]);
        l[k][a] = v;
      }
    }
    const size_t E = size_t(cfg_of(off, nb, s)) * n * n * n + size_t(e[0]) + size_t(n) * (e[1] + size_t(n) * e[2]);
    const double *w = Wel + E * (Q1 * Q1 * Q1);
    double acc = 0.0;
#pragma unroll
    for (int mz = 0; mz < Q1; ++mz) {
      double sy = 0.0;
#pragma unroll
      for (int my = 0; my < Q1; ++my) {
        double sx = 0.0;
#pragma unroll
        for (int mx = 0; mx < Q1; ++mx) sx += l[0][mx] * w[(mz * Q1 + my) * Q1 + mx];
        sy += l[1][my] * sx;
      }
      acc += l[2][mz] * sy;
    }
    const double pm = acc * inv_h;
    const double tot = phip[s] * inv_h + pm;
    phim_s[s] = pm;
    phi_s[s] = tot;
    Phi[perm[s]] = tot;
  }
}

// Per-configuration block partials of sum_s Q_s Phi_s (K blocks per
// configuration over its sorted slots off[b] .. off[b+1]-1).
__global__ __launch_bounds__(256) void k_energy(int K, const int *__restrict__ off, const double *__restrict__ sQ,
                                                const double *__restrict__ phi_s, double *__restrict__ partial) {
  __shared__ double red[256];
  const int cfg = blockIdx.x / K, kb = blockIdx.x % K;
  const int64_t hi = off[cfg + 1];
  double acc = 0.0;
  for (int64_t s = off[cfg] + int64_t(kb) * blockDim.x + threadIdx.x; s < hi; s += int64_t(K) * blockDim.x)
    acc += sQ[s] * phi_s[s];
  double t = block_sum_p(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_half(int nb, const double *__restrict__ in, double *__restrict__ out) {
  for (int b = threadIdx.x; b < nb; b += blockDim.x) out[b] = 0.5 * in[b];
}

// out[perm[s]] = scale * in[s]
__global__ __launch_bounds__(256) void k_unpermute(int64_t N, double scale, const int *__restrict__ perm,
                                                   const double *__restrict__ in, double *__restrict__ out) {
  for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < N; s += int64_t(gridDim.x) * blockDim.x)
    out[perm[s]] = scale * in[s];
}

// Ordered near pairs: sum_E count_E * (sum over the block of counts) - N.
template <int NSR>
__global__ __launch_bounds__(256) void k_pair_count(int n, int MT, const int *__restrict__ start,
                                                    unsigned long long *__restrict__ out) {
  const int M = n * n * n;
  for (int E = blockIdx.x * blockDim.x + threadIdx.x; E < MT; E += gridDim.x * blockDim.x) {
    const int c = start[E + 1] - start[E];
    if (c == 0) continue;
    const int base = (E / M) * M, El = E % M;
    const int ex = El % n, ey = (El / n) % n, ez = El / (n * n);
    long long s = 0;
    for (int dz = -NSR; dz <= NSR; ++dz)
      for (int dy = -NSR; dy <= NSR; ++dy)
        for (int dx = -NSR; dx <= NSR; ++dx) {
          const int F = base + (ex + dx + n) % n + n * ((ey + dy + n) % n + n * ((ez + dz + n) % n));
          s += start[F + 1] - start[F];
        }
    atomicAdd(out, (unsigned long long)(c * s - c));
  }
}

// ----------------------------------------------------------------- launchers

namespace {
inline int grid_n(int64_t n, int maxb = 4096) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  return int(g < maxb ? g : maxb);
}
}  // namespace

int bin_grid(int64_t N, int nb) { return seg_blocks(nb, size_t((N + nb - 1) / nb)); }

int launch_bin(hipStream_t s, int nb, const int *off, int64_t N, const double *x, const double *Q, double L, int n,
               int box, double *gtmp, int *elem, int *slot, int *count, int *flags, double *partial) {
  const int K = bin_grid(N, nb);
  hipLaunchKernelGGL(k_bin, dim3(nb * K), dim3(256), 0, s, N, K, off, x, Q, L, n, box, gtmp, elem, slot, count,
                     flags, partial);
  return K;
}
void launch_scan(hipStream_t s, int M, const int *count, int *start, int *maxcount, int *scratch) {
  const int B = (M + kScanTile - 1) / kScanTile;
  int *bsum = scratch, *bmax = scratch + B;
  hipLaunchKernelGGL(k_scan_reduce, dim3(B), dim3(256), 0, s, M, count, bsum, bmax);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, B, M, bsum, bmax, start, maxcount);
  hipLaunchKernelGGL(k_scan_down, dim3(B), dim3(256), 0, s, M, count, bsum, start);
}
void launch_scatter(hipStream_t s, int64_t N, const int *elem, const int *slot, const int *start, int *tmp) {
  hipLaunchKernelGGL(k_scatter, dim3(grid_n(N)), dim3(256), 0, s, N, elem, slot, start, tmp);
}
void launch_rank(hipStream_t s, int64_t N, const int *tmp, const int *elem, const int *start, const double *gtmp,
                 const double *Q, int *perm, double *sg, double *sQ) {
  hipLaunchKernelGGL(k_rank, dim3(grid_n(N)), dim3(256), 0, s, N, tmp, elem, start, gtmp, Q, perm, sg, sQ);
}
void launch_moments(hipStream_t s, int nb, int n, int64_t N, const int *start, const double *sg, const double *sQ,
                    double *C) {
  const int MT = nb * n * n * n;
  hipLaunchKernelGGL(k_moments, dim3(grid_n(MT)), dim3(256), 0, s, n, MT, N, start, sg, sQ, C);
}
template <int NSR>
static void pair_impl(hipStream_t s, int nb, int n, int64_t N, const int *start, const double *sg, const double *sQ,
                      double *phip, double *fpair) {
  dim3 g(nb * n * n * n);
  if (fpair) hipLaunchKernelGGL((k_pair<NSR, true>), g, dim3(64), 0, s, n, N, start, sg, sQ, phip, fpair);
  else hipLaunchKernelGGL((k_pair<NSR, false>), g, dim3(64), 0, s, n, N, start, sg, sQ, phip, fpair);
}
int launch_pair(hipStream_t s, int nb, int n, int nsr, int64_t N, const int *start, const double *sg, const double *sQ,
                double *phip, double *fpair) {
  switch (nsr) {
    case 1: pair_impl<1>(s, nb, n, N, start, sg, sQ, phip, fpair); return 0;
    case 2: pair_impl<2>(s, nb, n, N, start, sg, sQ, phip, fpair); return 0;
    case 3: pair_impl<3>(s, nb, n, N, start, sg, sQ, phip, fpair); return 0;
    case 4: pair_impl<4>(s, nb, n, N, start, sg, sQ, phip, fpair); return 0;
    default: return -1;
  }
}
// Work list of items of up to `titem` targets; nit (MT + 1 ints) and
// item_start (MT + 1 ints) are scratch, items holds up to N entries, and
// item_start[MT] receives the item count.
void launch_items(hipStream_t s, int MT, int titem, const int *start, int *nit, int *item_start, int *scan_max,
                  int2 *items, int *scan_scratch) {
  hipLaunchKernelGGL(k_items_count, dim3(grid_n(MT)), dim3(256), 0, s, MT, titem, start, nit);
  launch_scan(s, MT, nit, item_start, scan_max, scan_scratch);
  hipLaunchKernelGGL(k_items_fill, dim3(grid_n(MT)), dim3(256), 0, s, MT, titem, start, item_start, items);
}
void launch_fill_int(hipStream_t s, int count, int value, int *p) {
  hipLaunchKernelGGL(k_fill_int, dim3((count + 63) / 64 < 1024 ? (count + 63) / 64 : 1024), dim3(64), 0, s, count,
                     value, p);
}
template <int NSR>
static void pair_queue_impl(hipStream_t s, int waves, int n, int64_t N, const int *start, const int2 *items,
                            const int *nitems, int *counter, int titem, const double *sg, const double *sQ,
                            double *phip, double *fpair) {
  if (fpair)
    hipLaunchKernelGGL((k_pair_queue<NSR, true>), dim3(waves), dim3(64), 0, s, n, N, start, items, nitems, counter,
                       titem, sg, sQ, phip, fpair);
  else
    hipLaunchKernelGGL((k_pair_queue<NSR, false>), dim3(waves), dim3(64), 0, s, n, N, start, items, nitems, counter,
                       titem, sg, sQ, phip, fpair);
}
int launch_pair_queue(hipStream_t s, int waves, int n, int nsr, int64_t N, const int *start, const int2 *items,
                      const int *nitems, int *counter, int titem, const double *sg, const double *sQ, double *phip,
                      double *fpair) {
  launch_fill_int(s, 1, 0, counter);
  switch (nsr) {
    case 1: pair_queue_impl<1>(s, waves, n, N, start, items, nitems, counter, titem, sg, sQ, phip, fpair); return 0;
    case 2: pair_queue_impl<2>(s, waves, n, N, start, items, nitems, counter, titem, sg, sQ, phip, fpair); return 0;
    case 3: pair_queue_impl<3>(s, waves, n, N, start, items, nitems, counter, titem, sg, sQ, phip, fpair); return 0;
    case 4: pair_queue_impl<4>(s, waves, n, N, start, items, nitems, counter, titem, sg, sQ, phip, fpair); return 0;
    default: return -1;
  }
}
int launch_pair_count(hipStream_t s, int nb, int n, int nsr, const int *start, unsigned long long *out) {
  const int MT = nb * n * n * n;
  switch (nsr) {
    case 1: hipLaunchKernelGGL(k_pair_count<1>, dim3(grid_n(MT)), dim3(256), 0, s, n, MT, start, out); return 0;
    case 2: hipLaunchKernelGGL(k_pair_count<2>, dim3(grid_n(MT)), dim3(256), 0, s, n, MT, start, out); return 0;
    case 3: hipLaunchKernelGGL(k_pair_count<3>, dim3(grid_n(MT)), dim3(256), 0, s, n, MT, start, out); return 0;
    case 4: hipLaunchKernelGGL(k_pair_count<4>, dim3(grid_n(MT)), dim3(256), 0, s, n, MT, start, out); return 0;
    default: return -1;
  }
}
int launch_interp(hipStream_t s, int nb, const int *off, int p, int n, int64_t N, double inv_h, const GllBasis &bas,
                  const double *sg, const double *Wel, const double *phip, const int *perm, double *phim_s,
                  double *phi_s, double *Phi) {
#define CALL(PO)                                                                                                 \
  hipLaunchKernelGGL(k_interp<PO>, dim3(grid_n(N)), dim3(256), 0, s, n, N, nb, off, inv_h, bas, sg, Wel, phip, perm, \
                     phim_s, phi_s, Phi)
  switch (p) {
    case 3: CALL(3); return 0;
    case 4: CALL(4); return 0;
    case 5: CALL(5); return 0;
    case 6: CALL(6); return 0;
    default: return -1;
  }
#undef CALL
}
int launch_energy(hipStream_t s, int nb, const int *off, int64_t N, const double *sQ, const double *phi_s,
                  double *partial) {
  const int K = energy_grid(N, nb);
  hipLaunchKernelGGL(k_energy, dim3(nb * K), dim3(256), 0, s, K, off, sQ, phi_s, partial);
  return K;
}
int energy_grid(int64_t N, int nb) { return seg_blocks(nb, size_t((N + nb - 1) / nb)); }
void launch_half(hipStream_t s, int nb, const double *in, double *out) {
  hipLaunchKernelGGL(k_half, dim3(1), dim3(256), 0, s, nb, in, out);
}
void launch_unpermute(hipStream_t s, int64_t N, double scale, const int *perm, const double *in, double *out) {
  hipLaunchKernelGGL(k_unpermute, dim3(grid_n(N)), dim3(256), 0, s, N, scale, perm, in, out);
}

}  // namespace fep3m
