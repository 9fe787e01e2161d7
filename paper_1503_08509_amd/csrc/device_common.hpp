// Shared definitions for the gfx950 kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fep3m {

constexpr int kMaxP = 6;           // largest element order handled by the kernels
constexpr int kRedBlocks = 1024;   // fixed block count of every two-stage reduction
constexpr int kRowBlocks = 8192;   // block count of the row-wise mesh kernels (load, assembly, mass)
constexpr int kRedThreads = 256;

// 1-D element operator of one multigrid level, passed by value, in the
// arithmetic type T of the kernels that apply it.
template <class T>
struct LevelOpT {
  int p;                 // element order
  int n;                 // elements per axis (periodic)
  int P;                 // DOFs per axis = p * n
  T ke[(kMaxP + 1) * (kMaxP + 1)];  // element stiffness, row-major (p+1)^2
  T me[(kMaxP + 1) * (kMaxP + 1)];  // element mass
  T dk[kMaxP];           // diagonal of assembled K1 at local index k (k = 0: vertex)
  T dm[kMaxP];           // diagonal of assembled M1
  const T *cg = nullptr; // device copy of me then ke (p = 6 levels: read through scalar loads)

  template <class U>
  LevelOpT<U> cast() const {
    LevelOpT<U> o{};
    o.p = p; o.n = n; o.P = P;
    for (int i = 0; i < (kMaxP + 1) * (kMaxP + 1); ++i) { o.ke[i] = U(ke[i]); o.me[i] = U(me[i]); }
    for (int i = 0; i < kMaxP; ++i) { o.dk[i] = U(dk[i]); o.dm[i] = U(dm[i]); }
    return o;
  }
};
using LevelOp = LevelOpT<double>;
using LevelOpF = LevelOpT<float>;

// Prolongation weights from a coarse level (pc, nc) to a fine level (pf, nf):
// fine nodes inside one coarse element are numbered s = 0 .. r*pf - 1
// (r = nf / nc); w[s * (pc+1) + j] is coarse basis j at fine node s.
template <class T>
struct TransferT {
  int pf, nf, Pf;
  int pc, nc, Pc;
  int r;                  // fine elements per coarse element per axis
  int ns;                 // r * pf
  T w[3 * kMaxP * (kMaxP + 1)];   // ns <= 3 * kMaxP

  template <class U>
  TransferT<U> cast() const {
    TransferT<U> o{};
    o.pf = pf; o.nf = nf; o.Pf = Pf; o.pc = pc; o.nc = nc; o.Pc = Pc; o.r = r; o.ns = ns;
    for (int i = 0; i < 3 * kMaxP * (kMaxP + 1); ++i) o.w[i] = U(w[i]);
    return o;
  }
};
using Transfer = TransferT<double>;
using TransferF = TransferT<float>;

// Batches: nb independent configurations that share the mesh and the
// method's parameters.  Element ids are configuration-major (b * n^3 + e),
// mesh vectors are nb consecutive P^3 blocks, and the charges of
// configuration b occupy caller (and sorted) indices off[b] .. off[b+1]-1.
// Per-configuration reductions use K blocks per configuration: block
// (b, k) = blockIdx b * K + k strides over configuration b's range.
__device__ __forceinline__ int cfg_of(const int *__restrict__ off, int nb, int64_t i) {
  int lo = 0, hi = nb;   // off[lo] <= i < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  For a grid of `total` blocks walking a linear (x fastest) order of
// tiles, give XCD k the k-th contiguous eighth of that order, so the tiles
// resident together on one XCD are spatial neighbours that share halo data
// in its L2.  Identity when total is not a multiple of 8.
__device__ __forceinline__ int xcd_linear(int b, int total) {
  if (total % 8) return b;
  return (b & 7) * (total >> 3) + (b >> 3);
}

// Device arrays (nb values each) of the per-configuration PCG scalars.
struct PcgScalars {
  double *bn2, *rz, *rzn, *pq, *rr, *zq, *alpha, *beta, *act, *rel;
};

enum PcgStep : int { kPcgStart = 0, kPcgAlpha = 1, kPcgResid = 2, kPcgBeta = 3, kPcgBetaPR = 4 };

enum ApplyMode : int {
  kApply = 0,      // out = K x
  kResidual = 1,   // out = f - K x
  kCheb = 2,       // xo = x + c1 (x - xprev) + c2 D^-1 (f - K x)   (xo may alias xprev)
  kApplyDot = 3,   // out = K x, block partial of x . (K x)
  kDinvApply = 4,  // out = D^-1 K x
  // Second and third Chebyshev steps after a zero start, whose first step
  // x1 = s0 D^-1 f is never stored:
  kChebZ2 = 5,     // as kCheb with x = s0 D^-1 f (built from f on the fly) and x_prev = 0
  kChebZ3 = 6,     // as kCheb with x_prev = s0 D^-1 f
  kResidualRestrict = 7,  // f - K x restricted to the next level, not stored (launch_apply_restrict)
  kChebDot = 8     // as kCheb, and block partials of x_new . f
};

}  // namespace fep3m
