// Host launchers of the gfx950 kernels (one declaration per launcher).
#pragma once

#include "device_common.hpp"

namespace fep3m {

// Order-p GLL Lagrange basis on [-1/2, 1/2] in product form:
// l_a(u) = w[a] * prod_{j != a} (u - x[j]).
struct GllBasis {
  double x[kMaxP + 1];
  double w[kMaxP + 1];
};

// particles (k_particles.hip)
int bin_grid(int64_t N);
int energy_grid(int64_t N);
void launch_bin(hipStream_t s, int64_t N, const double *x, const double *Q, double L, int n, double *gtmp, int *elem,
                int *slot, int *count, int *flags, double *partial);
void launch_scan(hipStream_t s, int M, const int *count, int *start, int *maxcount);
void launch_scatter(hipStream_t s, int64_t N, const int *elem, const int *slot, const int *start, int *tmp);
void launch_rank(hipStream_t s, int64_t N, const int *tmp, const int *elem, const int *start, const double *gtmp,
                 const double *Q, int *perm, double *sg, double *sQ);
void launch_moments(hipStream_t s, int n, int64_t N, const int *start, const double *sg, const double *sQ, double *C);
int launch_pair(hipStream_t s, int n, int nsr, int64_t N, const int *start, const double *sg, const double *sQ,
                double *phip, double *fpair);
int launch_pair_count(hipStream_t s, int n, int nsr, const int *start, unsigned long long *out);
int launch_interp(hipStream_t s, int p, int n, int64_t N, double inv_h, const GllBasis &bas, const double *sg,
                  const double *Wel, const double *phip, const int *perm, double *phim_s, double *phi_s, double *Phi);
void launch_energy(hipStream_t s, int64_t N, const double *sQ, const double *phi_s, double *partial);
void launch_half(hipStream_t s, const double *in, double *out);
void launch_unpermute(hipStream_t s, int64_t N, double scale, const int *perm, const double *in, double *out);

// adjoint (k_adjoint.hip)
int launch_deposit(hipStream_t s, int p, int n, int64_t N, const GllBasis &bas, const int *start, const double *sg,
                   const double *sQ, double *gE);
int launch_assemble(hipStream_t s, int p, int n, const double *gE, double *G, double *partial);
int launch_adj_moments(hipStream_t s, int p, int n, int nsr, const double *gE, const double *Tt, const double *lam,
                       const double *gw, double *A);
int launch_forces(hipStream_t s, int p, int n, int64_t N, double inv_h, const GllBasis &bas, const double *sg,
                  const double *sQ, const double *Wel, const double *A, const double *fpair, const double *phip,
                  const double *phim_s, const int *perm, double *F, double *dUdQ);

// near field (k_near.hip)
int launch_psi(hipStream_t s, int n, int nsr, int p, const double *C, const double *T, const double *phi, double *Wel);

// mesh (k_mesh.hip)
int red_grid(size_t n);
void launch_load(hipStream_t s, int n, int p, const double *C, const double *gw, double *b, double *partial);
void launch_sum_partials(hipStream_t s, int count, const double *partial, double *out);
void launch_sub_mass_ones(hipStream_t s, int n, int p, const double *w1, const double *scal, double *v);
void launch_mass_dot(hipStream_t s, int n, int p, const double *w1, const double *v, double *partial);
void launch_sub_const(hipStream_t s, size_t total, double invV, const double *scal, double *v);
int launch_apply(hipStream_t s, const LevelOp &op, const double *x, const double *f, double *out,
                 const double *xprev, double *xo, double c1, double c2, int mode, double *partial);
int apply_blocks(const LevelOp &op);
void launch_cheb_first(hipStream_t s, const LevelOp &op, const double *f, double *xprev, double *x, double c2);
int launch_transfer(hipStream_t s, const Transfer &tr, const double *in, double *out, bool restrict_);
void launch_restrict(hipStream_t s, const Transfer &tr, const double *rf, double *fc);
void launch_prolong_add(hipStream_t s, const Transfer &tr, const double *ec, double *xf);
void launch_coarse_solve(hipStream_t s, int Pn, const double *V, const double *lam, const double *f, double *x);
void launch_dot(hipStream_t s, size_t n, const double *a, const double *b, double *partial);
void launch_cg_update(hipStream_t s, size_t n, double alpha, const double *p, const double *q, double *x, double *r,
                      double *partial);
void launch_xpay(hipStream_t s, size_t n, double beta, const double *z, double *p);
void launch_scale(hipStream_t s, size_t n, double sc, const double *a, double *b);
void launch_hash_fill(hipStream_t s, size_t n, uint32_t seed, double *v);

}  // namespace fep3m
