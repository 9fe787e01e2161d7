// Shared definitions for the gfx950 kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fep3m {

constexpr int kMaxP = 6;           // largest element order handled by the kernels
constexpr int kRedBlocks = 1024;   // fixed block count of every two-stage reduction
constexpr int kRedThreads = 256;

// 1-D element operator of one multigrid level, passed by value.
struct LevelOp {
  int p;                 // element order
  int n;                 // elements per axis (periodic)
  int P;                 // DOFs per axis = p * n
  double ke[(kMaxP + 1) * (kMaxP + 1)];  // element stiffness, row-major (p+1)^2
  double me[(kMaxP + 1) * (kMaxP + 1)];  // element mass
  double dk[kMaxP];      // diagonal of assembled K1 at local index k (k = 0: vertex)
  double dm[kMaxP];      // diagonal of assembled M1
};

// Prolongation weights from a coarse level (pc, nc) to a fine level (pf, nf):
// fine nodes inside one coarse element are numbered s = 0 .. r*pf - 1
// (r = nf / nc); w[s * (pc+1) + j] is coarse basis j at fine node s.
struct Transfer {
  int pf, nf, Pf;
  int pc, nc, Pc;
  int r;                  // fine elements per coarse element per axis
  int ns;                 // r * pf
  double w[3 * kMaxP * (kMaxP + 1)];   // ns <= 3 * kMaxP
};

enum ApplyMode : int {
  kApply = 0,      // out = K x
  kResidual = 1,   // out = f - K x
  kCheb = 2,       // xo = x + c1 (x - xprev) + c2 D^-1 (f - K x)   (xo may alias xprev)
  kApplyDot = 3,   // out = K x, block partial of x . (K x)
  kDinvApply = 4   // out = D^-1 K x
};

}  // namespace fep3m
