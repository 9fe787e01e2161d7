// Near-pair sum (float64) on rows of target elements: one workgroup (one
// wave) takes up to 64 consecutive sorted charges of one x-row of elements (fixed y, z),
// one charge per thread.  For each of the (2 NSR + 1)^2 source rows (dy, dz)
// of the near block the workgroup stages, once, the charges of the x-range
// its targets need (elements exA - NSR .. exB + NSR, unwrapped: a wrapped
// element appears with its periodic image shift) in LDS with the shift
// applied, and each thread walks the contiguous window of its own element,
// ex - NSR .. ex + NSR, with no segment search and no shift arithmetic per
// source.  Every staged source serves all the targets of the workgroup
// whose window holds it (up to about 7 Ntilde, Ntilde charges per element).
// A target may take SL lanes, each walking every SL-th source of its window
// (the autotuner picks SL = 1, 2 or 4); the central row (dy = dz = 0) skips
// the target itself.  Each target sums its pairs in a fixed order (rows, then
// sources in sorted order), so results are repeatable; the order differs
// from the one-wave-per-element kernels, hence results agree with them to
// rounding, not bit for bit.
#include "kernels.hpp"

namespace fep3m {
namespace {

constexpr int kRowTargets = 64;    // targets (threads) per workgroup: one wave
constexpr int kRowCap = 256;       // sources staged per LDS fill (8 KB)

__global__ __launch_bounds__(256) void k_row_starts(int RT, int n, const int *__restrict__ start,
                                                    int *__restrict__ rowstart) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r <= RT; r += gridDim.x * blockDim.x)
    rowstart[r] = start[size_t(r) * n];
}

__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// The staged x-range of one source row as up to three runs of sorted
// charges: unwrapped elements u < 0 (image shift -1), 0 .. n - 1, >= n (+1).
struct RowRuns {
  int b0, l0, b1, l1, b2, l2;   // first sorted slot and length of each run
  int u0;                       // first unwrapped element of the range
  const int *st;                // element starts of the row (st[x], x in 0 .. n)
  int n;
  // offset in the flattened range of the first charge of unwrapped element u
  __device__ int off(int u) const {
    if (u < 0) return st[u + n] - b0;
    if (u < n) return l0 + st[u] - b1;
    return l0 + l1 + st[u - n] - b2;
  }
};

// SL lanes per target (each walks every SL-th source of the target's
// window; their sums are added at the end in a fixed order), 64 / SL
// targets per wave.
// box: the near block is cut at the faces of [0, n)^3: rows outside are
// skipped (a block-uniform test) and the x-range is clipped, so no run is
// wrapped.
template <int NSR, bool FORCE, int SL>
__global__ __launch_bounds__(kRowTargets) void k_pair_rows(int n, int box, int64_t N, const int *__restrict__ start,
                                                           const int2 *__restrict__ items,
                                                           const int *__restrict__ nitems,
                                                           const double *__restrict__ sg,
                                                           const double *__restrict__ sQ, double *__restrict__ phip,
                                                           double *__restrict__ fpair) {
  constexpr int TPW = kRowTargets / SL;   // targets per wave
  __shared__ double4 S[kRowCap];
  if (int(blockIdx.x) >= *nitems) return;   // uniform over the block
  const int2 it = items[blockIdx.x];
  const int R = it.x, t0 = it.y;
  const int n2 = n * n;
  const int cfg = R / n2, rr = R % n2, ey = rr % n, ez = rr / n;
  const size_t M = size_t(n) * n2;
  const int *stc = start + cfg * M;   // element starts of this configuration
  const int rowbase = n * (ey + n * ez);
  const int te = min(t0 + TPW, start[cfg * M + rowbase + n]);
  const int tid = threadIdx.x;
  const int sl = tid % SL;
  const int t = t0 + tid / SL;
  const bool act = t < te;
  const double nd = double(n);
  // this lane's target and element; the block's element range
  double tx = 0.0, ty = 0.0, tz = 0.0;
  int ext = 0;
  if (act) {
    tx = sg[t];
    ty = sg[N + t];
    tz = sg[2 * N + t];
    ext = min(int(floor(tx)), n - 1);
  }
  auto elem_of = [&](int s) { return min(int(floor(sg[s])), n - 1); };
  const int exA = elem_of(t0), exB = elem_of(te - 1);
  const int uA = box ? max(exA - NSR, 0) : exA - NSR, uB = box ? min(exB + NSR, n - 1) : exB + NSR;
  double acc = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
  auto pair = [&](const double4 &q) {
    const double dx = q.x - tx, dyv = q.y - ty, dzv = q.z - tz;
    const double r2 = fma(dx, dx, fma(dyv, dyv, dzv * dzv));
    const double ri = rsqrt_pos(r2);
    const double qr = q.w * ri;
    acc += qr;
    if (FORCE) {
      const double qr3 = qr * (ri * ri);
      fx = fma(qr3, dx, fx);
      fy = fma(qr3, dyv, fy);
      fz = fma(qr3, dzv, fz);
    }
  };
  for (int dz = -NSR; dz <= NSR; ++dz) {
    int zz = ez + dz, sz = 0;
    if (box && (zz < 0 || zz >= n)) continue;
    if (zz < 0) { zz += n; sz = -1; } else if (zz >= n) { zz -= n; sz = 1; }
    for (int dy = -NSR; dy <= NSR; ++dy) {
      int yy = ey + dy, sy = 0;
      if (box && (yy < 0 || yy >= n)) continue;
      if (yy < 0) { yy += n; sy = -1; } else if (yy >= n) { yy -= n; sy = 1; }
      RowRuns rw;
      rw.st = stc + n * (yy + n * zz);
      rw.n = n;
      rw.u0 = uA;
      rw.b0 = uA < 0 ? rw.st[uA + n] : 0;
      rw.l0 = uA < 0 ? rw.st[n] - rw.b0 : 0;
      rw.b1 = rw.st[max(uA, 0)];
      rw.l1 = rw.st[min(uB, n - 1) + 1] - rw.b1;
      rw.b2 = rw.st[0];
      rw.l2 = uB >= n ? rw.st[uB - n + 1] - rw.b2 : 0;
      const int U = rw.l0 + rw.l1 + rw.l2;
      const double shy = double(sy) * nd, shz = double(sz) * nd;
      const bool central = dy == 0 && dz == 0;
      int lo = 0, hi = 0, self = -1;
      if (act) {
        const int wa = box ? max(ext - NSR, 0) : ext - NSR, wb = box ? min(ext + NSR, n - 1) : ext + NSR;
        lo = rw.off(wa) + sl;   // this lane's sources: lo, lo + SL, ...
        hi = rw.off(wb + 1);
        if (central) self = rw.off(ext) + (t - rw.st[ext]);
      }
      for (int c0 = 0; c0 < U; c0 += kRowCap) {
        const int cn = min(kRowCap, U - c0);
        __syncthreads();   // the previous fill has been consumed
        for (int i = tid; i < cn; i += kRowTargets) {
          const int f = c0 + i;
          int s;
          double shx;
          if (f < rw.l0) { s = rw.b0 + f; shx = -nd; }
          else if (f < rw.l0 + rw.l1) { s = rw.b1 + (f - rw.l0); shx = 0.0; }
          else { s = rw.b2 + (f - rw.l0 - rw.l1); shx = nd; }
          S[i] = make_double4(sg[s] + shx, sg[N + s] + shy, sg[2 * N + s] + shz, sQ[s]);
        }
        __syncthreads();
        // first source of this lane's stride at or after c0
        int j = lo;
        if (j < c0) j += ((c0 - j + SL - 1) / SL) * SL;
        const int je = min(hi, c0 + cn);
        if (central) {   // the window holds the target itself
          for (; j < je; j += SL)
            if (j != self) pair(S[j - c0]);
        } else {
          for (; j + SL < je; j += 2 * SL) {   // two independent chains per step
            const double4 qa = S[j - c0], qb = S[j + SL - c0];
            pair(qa);
            pair(qb);
          }
          if (j < je) pair(S[j - c0]);
        }
      }
    }
  }
  // the SL partial sums of each target, added in a fixed order
#pragma unroll
  for (int o = 1; o < SL; o <<= 1) {
    acc += __shfl_xor(acc, o, 64);
    if (FORCE) {
      fx += __shfl_xor(fx, o, 64);
      fy += __shfl_xor(fy, o, 64);
      fz += __shfl_xor(fz, o, 64);
    }
  }
  if (act && sl == 0) {
    phip[t] = acc;
    if (FORCE) {
      fpair[t] = fx;
      fpair[N + t] = fy;
      fpair[2 * N + t] = fz;
    }
  }
}

template <int NSR, int SL>
void pair_rows_impl(hipStream_t s, int grid, int n, int box, int64_t N, const int *start, const int2 *items,
                    const int *nitems, const double *sg, const double *sQ, double *phip, double *fpair) {
  if (fpair)
    hipLaunchKernelGGL((k_pair_rows<NSR, true, SL>), dim3(grid), dim3(kRowTargets), 0, s, n, box, N, start, items,
                       nitems, sg, sQ, phip, fpair);
  else
    hipLaunchKernelGGL((k_pair_rows<NSR, false, SL>), dim3(grid), dim3(kRowTargets), 0, s, n, box, N, start, items,
                       nitems, sg, sQ, phip, fpair);
}

template <int NSR>
int pair_rows_sl(hipStream_t s, int sl, int grid, int n, int box, int64_t N, const int *start, const int2 *items,
                 const int *nitems, const double *sg, const double *sQ, double *phip, double *fpair) {
  switch (sl) {
    case 1: pair_rows_impl<NSR, 1>(s, grid, n, box, N, start, items, nitems, sg, sQ, phip, fpair); return 0;
    case 2: pair_rows_impl<NSR, 2>(s, grid, n, box, N, start, items, nitems, sg, sQ, phip, fpair); return 0;
    case 4: pair_rows_impl<NSR, 4>(s, grid, n, box, N, start, items, nitems, sg, sQ, phip, fpair); return 0;
    default: return -1;
  }
}

}  // namespace

int pair_rows_items_max(int nb, int n, int64_t N) {   // for up to 64 targets per item (one lane each)
  return nb * n * n + int(N / 16) + 1;
}

int launch_pair_rows(hipStream_t s, int nb, int n, int nsr, int sl, int box, int64_t N, const int *start,
                     int *rowstart, int *rnit, int *ritem_start, int *rscan_max, int2 *ritems, int *scan_scratch,
                     const double *sg, const double *sQ, double *phip, double *fpair) {
  if (sl != 1 && sl != 2 && sl != 4) return -1;
  const int RT = nb * n * n, tpw = kRowTargets / sl;
  hipLaunchKernelGGL(k_row_starts, dim3((RT + 256) / 256), dim3(256), 0, s, RT, n, start, rowstart);
  launch_items(s, RT, tpw, rowstart, rnit, ritem_start, rscan_max, ritems, scan_scratch);
  const int grid = RT + int(N / tpw) + 1;
  switch (nsr) {
    case 1: return pair_rows_sl<1>(s, sl, grid, n, box, N, start, ritems, ritem_start + RT, sg, sQ, phip, fpair);
    case 2: return pair_rows_sl<2>(s, sl, grid, n, box, N, start, ritems, ritem_start + RT, sg, sQ, phip, fpair);
    case 3: return pair_rows_sl<3>(s, sl, grid, n, box, N, start, ritems, ritem_start + RT, sg, sQ, phip, fpair);
    default: return -1;
  }
}

}  // namespace fep3m
