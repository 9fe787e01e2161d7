// Source list of one target element's near block for the pair kernels.
//
// The (2 NSR + 1)^3 source elements of target element E are walked as
// 2 (2 NSR + 1)^2 contiguous runs of sorted charges: one run per (dy, dz)
// row of elements along x, split in two where the row wraps the periodic
// box.  Each run carries its periodic image shift (-1, 0, +1 per axis, in
// units of the box) and its offset in the flattened list, so that one wave
// can stride over every source of the block with unit-stride loads.
#pragma once

#include <hip/hip_runtime.h>

namespace fep3m {

template <int NSR>
struct PairSegments {
  static constexpr int W = 2 * NSR + 1;
  static constexpr int MAXSEG = 2 * W * W;
  int sb[MAXSEG];       // first sorted slot of the run
  int sl[MAXSEG];       // run length
  int so[MAXSEG + 1];   // offset of the run in the flattened list
  int ss[MAXSEG];       // packed image shifts (s + 1) per axis, 2 bits each

  __device__ static int shift(int pk, int axis) { return ((pk >> (2 * axis)) & 3) - 1; }
};

// Fill the runs of element E (called by every thread of one wave-sized
// block; contains the block's barriers).  Returns the flattened length.
template <int NSR>
__device__ int build_segments(PairSegments<NSR> &S, int E, int n, const int *__restrict__ start, int lane,
                              int nthreads) {
  constexpr int W = PairSegments<NSR>::W, MAXSEG = PairSegments<NSR>::MAXSEG;
  const int ex = E % n, ey = (E / n) % n, ez = E / (n * n);
  for (int row = lane; row < W * W; row += nthreads) {
    const int dy = row % W - NSR, dz = row / W - NSR;
    int yy = ey + dy, zz = ez + dz, sy = 0, sz = 0;
    if (yy < 0) { yy += n; sy = -1; } else if (yy >= n) { yy -= n; sy = 1; }
    if (zz < 0) { zz += n; sz = -1; } else if (zz >= n) { zz -= n; sz = 1; }
    const int rowE = n * (yy + n * zz);
    const int x0 = ex - NSR, x1 = ex + NSR;
    int bA, eA, shA, bB = 0, eB = 0, shB = 0;
    if (x0 < 0) {
      bA = start[rowE + x0 + n]; eA = start[rowE + n]; shA = -1;
      bB = start[rowE]; eB = start[rowE + x1 + 1]; shB = 0;
    } else if (x1 >= n) {
      bA = start[rowE + x0]; eA = start[rowE + n]; shA = 0;
      bB = start[rowE]; eB = start[rowE + x1 - n + 1]; shB = 1;
    } else {
      bA = start[rowE + x0]; eA = start[rowE + x1 + 1]; shA = 0;
    }
    const int pk = ((sy + 1) << 2) | ((sz + 1) << 4);
    S.sb[2 * row] = bA; S.sl[2 * row] = eA - bA; S.ss[2 * row] = pk | (shA + 1);
    S.sb[2 * row + 1] = bB; S.sl[2 * row + 1] = eB - bB; S.ss[2 * row + 1] = pk | (shB + 1);
  }
  __syncthreads();
  if (lane == 0) {
    int acc = 0;
    for (int k = 0; k < MAXSEG; ++k) { S.so[k] = acc; acc += S.sl[k]; }
    S.so[MAXSEG] = acc;
  }
  __syncthreads();
  return S.so[MAXSEG];
}

}  // namespace fep3m
