// Mixed-precision particle kernels: the near-pair sum and the mesh-to-charge
// interpolation in float32 with Kahan-compensated per-charge sums, on a
// float32 copy of the sorted charges in element-local coordinates.  Every
// result leaves these kernels in float64 (pair potential and gradient,
// interpolated potential); the energy and the combination stay float64.
//
// Local coordinates: a charge at element units g = e + 1/2 + u keeps u in
// [-1/2, 1/2)^3 as float32 (for the interpolation) and as 29-bit fixed point
// iu = round(u 2^29) (for the pair sum), with its element (ex, ey, ez) packed
// as ex | ey << 10 | ez << 20.  A pair separation in units of 2^-29 element
// is then the exact int32 (element offset) 2^29 + iu_j - iu_i (|.| < 2^31
// for offsets up to 3), converted to float32 once: relative rounding 6e-8
// whatever the distance, where float32 coordinates would lose 3e-8 / r.
#include "kernels.hpp"
#include "pair_segments.hpp"

namespace fep3m {

namespace {

__device__ __forceinline__ void kahan_add(float &sum, float &comp, float v) {
  const float y = v - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace

// u (float32) and Q of every sorted charge, and its packed element.
constexpr double kFix = 536870912.0;   // 2^29
__global__ __launch_bounds__(256) void k_local_f32(int n, int64_t N, const double *__restrict__ sg,
                                                   const double *__restrict__ sQ, float4 *__restrict__ su,
                                                   int4 *__restrict__ si, int *__restrict__ sel) {
  for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < N; s += int64_t(gridDim.x) * blockDim.x) {
    int e[3], iu[3];
    float u[3];
    for (int k = 0; k < 3; ++k) {
      const double g = sg[k * N + s];
      double ef = floor(g);
      if (ef > double(n - 1)) ef = double(n - 1);
      e[k] = int(ef);
      const double ud = g - ef - 0.5;   // in [-1/2, 1/2]
      u[k] = float(ud);
      double fx = rint(ud * kFix);
      fx = fx > 268435455.0 ? 268435455.0 : (fx < -268435456.0 ? -268435456.0 : fx);
      iu[k] = int(fx);
    }
    const float q = float(sQ[s]);
    su[s] = make_float4(u[0], u[1], u[2], q);
    si[s] = make_int4(iu[0], iu[1], iu[2], __float_as_int(q));
    sel[s] = e[0] | (e[1] << 10) | (e[2] << 20);
  }
}

// Near-pair sum, one wavefront per target element as in the float64 kernel:
// each lane walks a strided share of the block's sources for a chunk of up
// to 8 targets, accumulating sum_j Q_j / r_ij (and, with FORCE, sum_j Q_j d_ij /
// r_ij^3) in float32 with Kahan compensation; the lanes' compensated sums
// are combined in float64.
template <int NSR, bool FORCE, int NT>
__device__ __forceinline__ void pair_chunk_f32(const PairSegments<NSR> &seg, int total, int lane, int64_t N, int t0,
                                               int nt, int n, int ex, int ey, int ez, const int4 *__restrict__ si,
                                               const int *__restrict__ sel, double *__restrict__ phip,
                                               double *__restrict__ fpair) {
  int tx[NT], ty[NT], tz[NT];
  float ps[NT], pc[NT];
  float fs[3][NT], fc[3][NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const int4 t = si[t0 + (k < nt ? k : 0)];
    tx[k] = t.x; ty[k] = t.y; tz[k] = t.z;
    ps[k] = pc[k] = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) fs[d][k] = fc[d][k] = 0.f;
  }
  int sp = 0;
  for (int f = lane; f < total; f += 64) {
    while (f >= seg.so[sp + 1]) ++sp;
    const int j = seg.sb[sp] + (f - seg.so[sp]);
    const int pk = seg.ss[sp];
    const int pe = sel[j];
    const int4 s = si[j];
    const float qj = __int_as_float(s.w);
    // source position relative to the target element centre, units of 2^-29 element
    const int jx = ((pe & 1023) + seg.shift(pk, 0) * n - ex) * (1 << 29) + s.x;
    const int jy = (((pe >> 10) & 1023) + seg.shift(pk, 1) * n - ey) * (1 << 29) + s.y;
    const int jz = ((pe >> 20) + seg.shift(pk, 2) * n - ez) * (1 << 29) + s.z;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const float dx = float(jx - tx[k]), dy = float(jy - ty[k]), dz = float(jz - tz[k]);
      const float r2 = dx * dx + dy * dy + dz * dz;
      const bool use = (k < nt) && (j != t0 + k);
      const float ri = use ? rsqrtf(r2) : 0.f;   // the skipped self pair has r = 0
      const float qr = qj * ri;
      kahan_add(ps[k], pc[k], qr);
      if (FORCE) {
        const float qr3 = qr * ri * ri;
        kahan_add(fs[0][k], fc[0][k], qr3 * dx);
        kahan_add(fs[1][k], fc[1][k], qr3 * dy);
        kahan_add(fs[2][k], fc[2][k], qr3 * dz);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    // sums in fixed-point units: 1/r carries 2^-29 and d/r^3 carries 2^-58
    const double p = wave_sum(double(ps[k]) - double(pc[k])) * kFix;
    double g[3] = {0.0, 0.0, 0.0};
    if (FORCE) {
#pragma unroll
      for (int d = 0; d < 3; ++d) g[d] = wave_sum(double(fs[d][k]) - double(fc[d][k])) * (kFix * kFix);
    }
    if (lane == 0 && k < nt) {
      phip[t0 + k] = p;
      if (FORCE) {
        fpair[t0 + k] = g[0];
        fpair[N + t0 + k] = g[1];
        fpair[2 * N + t0 + k] = g[2];
      }
    }
  }
}

template <int NSR, bool FORCE>
__global__ __launch_bounds__(64) void k_pair_f32(int n, int64_t N, const int *__restrict__ start,
                                                 const int4 *__restrict__ si, const int *__restrict__ sel,
                                                 double *__restrict__ phip, double *__restrict__ fpair) {
  __shared__ PairSegments<NSR> seg;
  const int lane = threadIdx.x;
  const int E = blockIdx.x;
  const int tb = start[E], te = start[E + 1];
  if (tb == te) return;  // uniform over the (single-wave) block
  const int M = n * n * n, El = E % M;
  const int total = build_segments<NSR>(seg, El, n, start + (E / M) * M, lane, 64);
  const int ex = El % n, ey = (El / n) % n, ez = El / (n * n);
  for (int t0 = tb; t0 < te;) {   // chunk widths 8, 4, 2 as in the float64 kernel
    const int rem = te - t0;
    if (rem > 4) {
      pair_chunk_f32<NSR, FORCE, 8>(seg, total, lane, N, t0, min(rem, 8), n, ex, ey, ez, si, sel, phip, fpair);
      t0 += 8;
    } else if (rem > 2) {
      pair_chunk_f32<NSR, FORCE, 4>(seg, total, lane, N, t0, rem, n, ex, ey, ez, si, sel, phip, fpair);
      t0 += 4;
    } else {
      pair_chunk_f32<NSR, FORCE, 2>(seg, total, lane, N, t0, rem, n, ex, ey, ez, si, sel, phip, fpair);
      t0 += 2;
    }
  }
}

// Load-balanced form over the work items of k_pair_queue (same items).
template <int NSR, bool FORCE>
__global__ __launch_bounds__(64) void k_pair_queue_f32(int n, int64_t N, const int *__restrict__ start,
                                                       const int2 *__restrict__ items, const int *__restrict__ nitems,
                                                       int *__restrict__ counter, int titem,
                                                       const int4 *__restrict__ si, const int *__restrict__ sel,
                                                       double *__restrict__ phip, double *__restrict__ fpair) {
  __shared__ PairSegments<NSR> seg;
  __shared__ int cur;
  const int lane = threadIdx.x;
  const int total_items = *nitems;
  const int M = n * n * n;
  for (;;) {
    if (lane == 0) cur = atomicAdd(counter, 1);
    __syncthreads();
    const int it = cur;
    if (it >= total_items) break;   // uniform over the wave
    const int2 w = items[it];
    const int E = w.x, El = E % M, te = min(w.y + titem, start[E + 1]);
    const int total = build_segments<NSR>(seg, El, n, start + (E / M) * M, lane, 64);
    const int ex = El % n, ey = (El / n) % n, ez = El / (n * n);
    for (int t0 = w.y; t0 < te;) {
      const int rem = te - t0;
      if (rem > 4) {
        pair_chunk_f32<NSR, FORCE, 8>(seg, total, lane, N, t0, min(rem, 8), n, ex, ey, ez, si, sel, phip, fpair);
        t0 += 8;
      } else if (rem > 2) {
        pair_chunk_f32<NSR, FORCE, 4>(seg, total, lane, N, t0, rem, n, ex, ey, ez, si, sel, phip, fpair);
        t0 += 4;
      } else {
        pair_chunk_f32<NSR, FORCE, 2>(seg, total, lane, N, t0, rem, n, ex, ey, ez, si, sel, phip, fpair);
        t0 += 2;
      }
    }
    __syncthreads();   // the segment list and cur are rewritten for the next item
  }
}

// Phi_m at each sorted charge from the float32 W of its element by sum
// factorisation in float32 (the outer sum compensated), combined with the
// pair term in float64 and scattered to caller order.
template <int PO>
__global__ __launch_bounds__(256) void k_interp_f32(int n, int64_t N, int nb, const int *__restrict__ off,
                                                    double inv_h, GllBasis bas,
                                                    const float4 *__restrict__ su, const int *__restrict__ sel,
                                                    const float *__restrict__ Wel, const double *__restrict__ phip,
                                                    const int *__restrict__ perm, double *__restrict__ phim_s,
                                                    double *__restrict__ phi_s, double *__restrict__ Phi) {
  constexpr int Q1 = PO + 1;
  float bx[Q1], bw[Q1];
#pragma unroll
  for (int a = 0; a < Q1; ++a) { bx[a] = float(bas.x[a]); bw[a] = float(bas.w[a]); }
  for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < N; s += int64_t(gridDim.x) * blockDim.x) {
    const float4 t = su[s];
    const int pe = sel[s];
    const float u[3] = {t.x, t.y, t.z};
    float l[3][Q1];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int a = 0; a < Q1; ++a) {
        float v = bw[a];
#pragma unroll
        for (int j = 0; j < Q1; ++j)
          if (j != a) v *= (u[k] - bx[j]);
        l[k][a] = v;
      }
    const size_t E = size_t(cfg_of(off, nb, s)) * n * n * n + size_t(pe & 1023) +
                     size_t(n) * (((pe >> 10) & 1023) + size_t(n) * (pe >> 20));
    const float *w = Wel + E * (Q1 * Q1 * Q1);
    float acc = 0.f, comp = 0.f;
#pragma unroll
    for (int mz = 0; mz < Q1; ++mz) {
      float sy = 0.f;
#pragma unroll
      for (int my = 0; my < Q1; ++my) {
        float sx = 0.f;
#pragma unroll
        for (int mx = 0; mx < Q1; ++mx) sx += l[0][mx] * w[(mz * Q1 + my) * Q1 + mx];
        sy += l[1][my] * sx;
      }
      kahan_add(acc, comp, l[2][mz] * sy);
    }
    const double pm = (double(acc) - double(comp)) * inv_h;
    const double tot = phip[s] * inv_h + pm;
    phim_s[s] = pm;
    phi_s[s] = tot;
    Phi[perm[s]] = tot;
  }
}

// ----------------------------------------------------------------- launchers

namespace {
inline int grid_m(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  return int(g < 4096 ? g : 4096);
}
}  // namespace

void launch_local_f32(hipStream_t s, int n, int64_t N, const double *sg, const double *sQ, float4 *su, int4 *si,
                      int *sel) {
  hipLaunchKernelGGL(k_local_f32, dim3(grid_m(N)), dim3(256), 0, s, n, N, sg, sQ, su, si, sel);
}

template <int NSR>
static void pair_f32_impl(hipStream_t s, int nb, int n, int64_t N, const int *start, const int4 *si, const int *sel,
                          double *phip, double *fpair) {
  dim3 g(nb * n * n * n);
  if (fpair) hipLaunchKernelGGL((k_pair_f32<NSR, true>), g, dim3(64), 0, s, n, N, start, si, sel, phip, fpair);
  else hipLaunchKernelGGL((k_pair_f32<NSR, false>), g, dim3(64), 0, s, n, N, start, si, sel, phip, fpair);
}
int launch_pair_f32(hipStream_t s, int nb, int n, int nsr, int64_t N, const int *start, const int4 *si,
                    const int *sel, double *phip, double *fpair) {
  // packed element coordinates hold 10 bits per axis; fixed-point separations
  // stay inside int32 for element offsets up to 3
  if (n > 1024 || nsr > 3) return -1;
  switch (nsr) {
    case 1: pair_f32_impl<1>(s, nb, n, N, start, si, sel, phip, fpair); return 0;
    case 2: pair_f32_impl<2>(s, nb, n, N, start, si, sel, phip, fpair); return 0;
    case 3: pair_f32_impl<3>(s, nb, n, N, start, si, sel, phip, fpair); return 0;
    default: return -1;
  }
}

template <int NSR>
static void pair_queue_f32_impl(hipStream_t s, int waves, int n, int64_t N, const int *start, const int2 *items,
                                const int *nitems, int *counter, int titem, const int4 *si, const int *sel,
                                double *phip, double *fpair) {
  if (fpair)
    hipLaunchKernelGGL((k_pair_queue_f32<NSR, true>), dim3(waves), dim3(64), 0, s, n, N, start, items, nitems,
                       counter, titem, si, sel, phip, fpair);
  else
    hipLaunchKernelGGL((k_pair_queue_f32<NSR, false>), dim3(waves), dim3(64), 0, s, n, N, start, items, nitems,
                       counter, titem, si, sel, phip, fpair);
}
int launch_pair_queue_f32(hipStream_t s, int waves, int n, int nsr, int64_t N, const int *start, const int2 *items,
                          const int *nitems, int *counter, int titem, const int4 *si, const int *sel, double *phip,
                          double *fpair) {
  if (n > 1024 || nsr > 3) return -1;
  launch_fill_int(s, 1, 0, counter);
  switch (nsr) {
    case 1: pair_queue_f32_impl<1>(s, waves, n, N, start, items, nitems, counter, titem, si, sel, phip, fpair); return 0;
    case 2: pair_queue_f32_impl<2>(s, waves, n, N, start, items, nitems, counter, titem, si, sel, phip, fpair); return 0;
    case 3: pair_queue_f32_impl<3>(s, waves, n, N, start, items, nitems, counter, titem, si, sel, phip, fpair); return 0;
    default: return -1;
  }
}

int launch_interp_f32(hipStream_t s, int nb, const int *off, int p, int n, int64_t N, double inv_h,
                      const GllBasis &bas, const float4 *su, const int *sel, const float *Wel, const double *phip,
                      const int *perm, double *phim_s, double *phi_s, double *Phi) {
  if (p != 5) return -1;
  hipLaunchKernelGGL(k_interp_f32<5>, dim3(grid_m(N)), dim3(256), 0, s, n, N, nb, off, inv_h, bas, su, sel, Wel,
                     phip, perm, phim_s, phi_s, Phi);
  return 0;
}

}  // namespace fep3m
