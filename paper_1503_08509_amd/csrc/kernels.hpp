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

// particles (k_particles.hip).  nb configurations: charges of configuration
// b are caller (and sorted) indices off[b] .. off[b+1]-1 (off on the device)
// and fall in elements b n^3 .. (b+1) n^3 - 1.
int bin_grid(int64_t N, int nb);
int energy_grid(int64_t N, int nb);
// box: positions must lie strictly inside [0, L)^3 (flags bit 2 otherwise);
// else they wrap periodically.
int launch_bin(hipStream_t s, int nb, const int *off, int64_t N, const double *x, const double *Q, double L, int n,
               int box, double *gtmp, int *elem, int *slot, int *count, int *flags, double *partial);
// scratch: 2 ceil(M / 2048) ints (tile sums and maxima)
void launch_scan(hipStream_t s, int M, const int *count, int *start, int *maxcount, int *scratch);
void launch_scatter(hipStream_t s, int64_t N, const int *elem, const int *slot, const int *start, int *tmp);
void launch_rank(hipStream_t s, int64_t N, const int *tmp, const int *elem, const int *start, const double *gtmp,
                 const double *Q, int *perm, double *sg, double *sQ);
void launch_moments(hipStream_t s, int nb, int n, int64_t N, const int *start, const double *sg, const double *sQ,
                    double *C);
int launch_pair(hipStream_t s, int nb, int n, int nsr, int64_t N, const int *start, const double *sg, const double *sQ,
                double *phip, double *fpair);
int launch_pair_count(hipStream_t s, int nb, int n, int nsr, const int *start, unsigned long long *out);
// Load-balanced pair sums: a work list of (element, first target) items of
// up to titem targets (item_start[MT] = item count; items up to N entries),
// consumed by `waves` persistent one-wave blocks through *counter.
void launch_items(hipStream_t s, int MT, int titem, const int *start, int *nit, int *item_start, int *scan_max,
                  int2 *items, int *scan_scratch);
void launch_fill_int(hipStream_t s, int count, int value, int *p);
int launch_pair_queue(hipStream_t s, int waves, int n, int nsr, int64_t N, const int *start, const int2 *items,
                      const int *nitems, int *counter, int titem, const double *sg, const double *sQ, double *phip,
                      double *fpair);
// Near-pair sum on rows of target elements (k_pair_rows.hip, float64):
// one-wave workgroups of up to 64 targets of one x-row, LDS-staged source rows.
// Work arrays: rowstart, ritem_start nb n^2 + 1 ints, rnit nb n^2,
// rscan_max 4, ritems pair_rows_items_max() int2, scan_scratch as launch_scan.
int pair_rows_items_max(int nb, int n, int64_t N);
// sl: lanes per target (1, 2 or 4; 64 / sl targets per wave); box: the near
// block is cut at the faces of [0, n)^3 (no periodic images)
int launch_pair_rows(hipStream_t s, int nb, int n, int nsr, int sl, int box, int64_t N, const int *start,
                     int *rowstart, int *rnit, int *ritem_start, int *rscan_max, int2 *ritems, int *scan_scratch,
                     const double *sg, const double *sQ, double *phip, double *fpair);
int launch_interp(hipStream_t s, int nb, const int *off, int p, int n, int64_t N, double inv_h, const GllBasis &bas,
                  const double *sg, const double *Wel, const double *phip, const int *perm, double *phim_s,
                  double *phi_s, double *Phi);
int launch_energy(hipStream_t s, int nb, const int *off, int64_t N, const double *sQ, const double *phi_s,
                  double *partial);
void launch_half(hipStream_t s, int nb, const double *in, double *out);
void launch_unpermute(hipStream_t s, int64_t N, double scale, const int *perm, const double *in, double *out);

// mixed precision (k_mixed.hip): float32 local coordinates and charges
// (su = {ux, uy, uz, Q}), the same offsets in 2^-29 fixed point with the
// charge's float bits (si), packed elements sel = ex | ey << 10 | ez << 20
void launch_local_f32(hipStream_t s, int n, int64_t N, const double *sg, const double *sQ, float4 *su, int4 *si,
                      int *sel);
int launch_pair_f32(hipStream_t s, int nb, int n, int nsr, int64_t N, const int *start, const int4 *si,
                    const int *sel, double *phip, double *fpair);
int launch_pair_queue_f32(hipStream_t s, int waves, int n, int nsr, int64_t N, const int *start, const int2 *items,
                          const int *nitems, int *counter, int titem, const int4 *si, const int *sel, double *phip,
                          double *fpair);
int launch_interp_f32(hipStream_t s, int nb, const int *off, int p, int n, int64_t N, double inv_h,
                      const GllBasis &bas, const float4 *su, const int *sel, const float *Wel, const double *phip,
                      const int *perm, double *phim_s, double *phi_s, double *Phi);

// adjoint (k_adjoint.hip)
int launch_deposit(hipStream_t s, int nb, int p, int n, int64_t N, const GllBasis &bas, const int *start,
                   const double *sg, const double *sQ, double *gE);
// returns the partial count K per configuration (-1: unsupported order)
int launch_assemble(hipStream_t s, int nb, int p, int n, const double *gE, double *G, double *partial);
// box = 1: no source outside [0, n)^3 and lam on the (p n + 1)^3 nodes of the
// box (launch_psi likewise: no source outside, phi on the box's nodes; a null
// phi gives W = -Psi).  A null lam writes the near part alone (A = -B); p = 3
// (the 27-element q = 1 screen) takes only that form.
int launch_adj_moments(hipStream_t s, int nb, int p, int n, int nsr, int box, const double *gE, const double *Tt,
                       const double *lam, const double *gw, double *A);
// W of the forward pass in float64, or float32 on the mixed-precision path
// (nl moments per axis; the screen families' (p, nl) pairs are instantiated)
template <class WT>
int launch_forces(hipStream_t s, int nb, const int *off, int p, int n, int nl, int64_t N, double inv_h,
                  const GllBasis &bas, const double *sg, const double *sQ, const WT *Wel, const double *A,
                  const double *fpair, const double *phip, const double *phim_s, const int *perm, double *F,
                  double *dUdQ);

// screen families other than the one-element q = 3 screen (k_screens.hip),
// float64: nl moments per axis, p the order, span 1 or 3 elements per axis;
// gw the load weights [nl][span p + 1].  The load returns its partial count
// per configuration (-1: unsupported combination), the others 0 or -1.
int launch_moments_g(hipStream_t s, int nb, int n, int nl, int64_t N, const int *start, const double *sg,
                     const double *sQ, double *C);
// box = 1: the grounded box [0, n]^3 (no wrap, (p n + 1)^3 nodes per
// configuration; span 1 only); a null phi makes the near field W = -Psi.
int launch_load_g(hipStream_t s, int nb, int n, int p, int span, int nl, int box, const double *C, const double *gw,
                  double *b, double *partial, double *sep = nullptr);
// scratch (doubles) of the separable load and lambda passes (periodic screen families; sep above)
size_t load_sep_scratch(int nb, int n, int p, int nl);
int launch_psi_g(hipStream_t s, int nb, int n, int nsr, int p, int nl, int box, const double *C, const double *T,
                 const double *phi, double *W);
int launch_adj_g(hipStream_t s, int nb, int n, int nsr, int p, int span, int nl, int box, const double *gE,
                 const double *Tt, const double *lam, const double *gw, double *A, double *sep = nullptr);   // Tt: tables as [D][m][a]

// grounded box (k_box.hip): mesh vectors of (p n + 1)^3 nodes per
// configuration, P = p n + 1.
struct BoxNodes {
  double x[8];   // GLL nodes of the element (p + 1 used) on [-1/2, 1/2]
};
// face quadrature of the insulating box: kBoxNQ Gauss-Legendre points per
// direction on [-1/2, 1/2], the order-p Lagrange values there and the
// basis derivatives at the element ends (-1/2, +1/2)
constexpr int kBoxNQ = 10;
struct BoxQuad {
  double xq[kBoxNQ], wq[kBoxNQ];
  double lq[kBoxNQ][8];
  double dend[2][8];
};
// phi_B = -Phi_sr on the boundary nodes (only those are written); Wneg the
// near field -Psi per element (launch_psi_g with box = 1 and no phi)
int launch_box_bvals(hipStream_t s, int nb, int n, int nsr, int p, int64_t N, const BoxNodes &nodes, const int *start,
                     const double *sg, const double *sQ, const double *Wneg, double *phiB);
// y = K v on every node of the box (K = Kx My Mz + Mx Ky Mz + Mx My Kz) by
// three banded 1-D passes; Kc, Mc the 1-D matrices as (p + 2) x (2 p + 1)
// tables of class rows (row o: class o mod p inside, p for o = 0, p + 1 for
// o = P - 1; entry d is column o - p + d); t1..t4 work vectors of nb P^3
int launch_box_apply(hipStream_t s, int P, int nb, int p, const double *Kc, const double *Mc, const double *v,
                     double *t1, double *t2, double *t3, double *t4, double *y);
// interior nodes of the box <-> contiguous (P - 2)^3 blocks
void launch_box_interior(hipStream_t s, int P, int nb, bool to_interior, const double *src, double *dst);
// y = c y + a x (c = 0: y is not read); fill y = v
void launch_box_axpby(hipStream_t s, size_t total, double a, const double *x, double c, double *y);
void launch_box_fill(hipStream_t s, size_t total, double v, double *y);
int launch_box_addphi(hipStream_t s, int nb, int n, int p, const double *phi, double *W);
// reverse pass: box assembly of element-local values; the boundary part of
// the per-charge gradients (F += Q bp / (2 h^2), dU/dQ -= bq / (2 h), added
// to what launch_forces wrote); mu on the boundary nodes of a box vector
int launch_box_assemble(hipStream_t s, int nb, int n, int p, const double *gE, double *G);
// gE[e(B)][m_B] -= mu_B: the boundary part then rides in the near part of
// the moment adjoint (launch_adj_g)
int launch_box_mu_slots(hipStream_t s, int nb, int n, int p, const double *mu, double *gE);
int launch_box_charge_bnd(hipStream_t s, int nb, int n, int nsr, int p, int64_t N, const int *off, double inv_h,
                          const BoxNodes &nodes, const double *sg, const double *sQ, const double *mu, const int *perm,
                          double *F, double *dUdQ);
// returns K: partial[0, nb K) holds the squares of b - y (y null: zero),
// [nb K, 2 nb K) those of b (plain: b itself), over the interior nodes or all
int launch_box_resid(hipStream_t s, int P, int nb, bool interior, bool plain, const double *b, const double *y,
                     double *partial);
// insulating box: f += surface load (tF: nb 6 n^2 (p + 1)^2 face values);
// f -= (sums / V) w1 (x) w1 (x) w1 (compatibility projection)
int launch_box_flux(hipStream_t s, int nb, int n, int nsr, int p, int64_t N, const BoxQuad &qd, const int *start,
                    const double *sg, const double *sQ, const double *Wneg, double *tF, double *f);
void launch_box_sub_mass(hipStream_t s, int P, int nb, double invV, const double *w1, const double *sums, double *f);
// insulating box, reverse pass: per face Lw (nb 6 n^2 kBoxNQ^2) and hF
// (nb 6 n^2 (p + 1)^3); gE -= the faces' hF per element; the per-charge
// face terms added to F and dU/dQ (after launch_forces)
int launch_box_flux_adj(hipStream_t s, int nb, int n, int p, const BoxQuad &qd, const double *lam, double *Lw,
                        double *hF);
int launch_box_h_slots(hipStream_t s, int nb, int n, int p, const double *hF, double *gE);
int launch_box_flux_charge(hipStream_t s, int nb, int n, int nsr, int p, int64_t N, const int *off, double inv_h,
                           const BoxQuad &qd, const double *sg, const double *sQ, const double *Lw, const int *perm,
                           double *F, double *dUdQ);

// near field (k_near.hip)
// T = double, or float (float32 tables, compensated slab sums, float32 W)
template <class T>
int launch_psi(hipStream_t s, int nb, int n, int nsr, int p, int box, const double *C, const T *Tab, const double *phi,
               T *Wel);
// the same on the matrix cores for the other screen families of order <= 5
// (nl moments per axis; -1 for (p, nl) it does not cover), float64
int launch_psi_mfma_g(hipStream_t s, int nb, int n, int nsr, int p, int nl, int box, const double *C, const double *Tab,
                      const double *phi, double *Wel);
// near part of the moment adjoint (A = -sum_D <g_{E+D}, T[.][D]>) on the
// matrix cores for the families with 27 or more moments (-1 otherwise)
int launch_adj_near_mfma(hipStream_t s, int nb, int n, int nsr, int p, int nl, int box, const double *gE,
                         const double *Tt, double *A);

// near field and its transpose by 3-D FFTs of the element lattice (k_fft.hip);
// n a power of two in [8, 64], p = 5.  S: table spectrum at the
// spec_freqs(n) = (n/2 + 1)^3 octant frequencies x 8 x (p+1)^3 complex;
// tw: exp(-2 pi i j / n), j < n.  Work arrays: zc, za nb n^3 x 4 complex;
// zpsi, zg nb n^3 x (p+1)^3 / 2 complex.
bool fft_size_ok(int n);
size_t spec_freqs(int n);
void launch_spec_build(hipStream_t s, int n, int nsr, int p, const double *T, const double2 *twf, double2 *S);
// transforms of C (if given) and of the deposits gE (if given), the spectrum
// products (one read of S for both), the inverse transform of the moment
// adjoint's near part (left in za as [E][8] doubles); Psi^ is left in zpsi.
int launch_near_fft(hipStream_t s, int nb, int n, int p, const double *C, const double *gE, const double2 *S,
                    const double2 *tw, double2 *zc, double2 *zpsi, double2 *zg, double2 *za);
// inverse transform of Psi^ and W = phi - Psi into Wel
template <class WT>
int launch_psi_fft_finish(hipStream_t s, int nb, int n, int p, const double2 *tw, const double *phi, double2 *zpsi,
                          WT *Wel);
// A = 4 pi G^T lambda - (near part in za)
int launch_adj_fft_finish(hipStream_t s, int nb, int n, int p, const double *lam, const double *gw, const double2 *za,
                          double *A);

// exact periodic solve by Fourier analysis over the element lattice
// (k_fdm.hip): nsys real systems (pairs share one complex work system),
// n a power of two in [8, 64], p = 3..6.  Z: ceil(nsys / 2) n^3 p^3
// complex; W, lam from periodic_fourier_eigen; tw: exp(-2 pi i j / n).
int launch_fs_solve(hipStream_t s, int nsys, int n, int p, const double *rhs, double *out, double2 *Z,
                    const double2 *tw, const double2 *W, const double *lam);
// the same solve on any mesh size (k_fdm.hip): the dense 1-D transform of
// the pencil's eigenvectors V (P x P, column-major, node i of mode j at
// V[i + j P]) along one axis (0 x, 1 y, 2 z) of nsys P^3 arrays; to_modes:
// V^T, else V.
void launch_axis_transform(hipStream_t s, int P, int axis, int nsys, const double *V, bool to_modes, const double *in,
                           double *out);
// in-place 3-D FFT of [nb][z][y][x][nch] complex arrays, nch = p^3 (k_fft.hip)
int launch_fft3_nodes(hipStream_t s, int nb, int n, int nch, double2 *z, const double2 *tw, bool inverse);

// mesh (k_mesh.hip).  nb configurations; per-configuration reductions
// write nb * K block partials (K = seg_blocks(nb, per) unless a launcher
// returns its own K) that launch_sum_partials folds into out[0 .. nb).
int seg_blocks(int nb, size_t per);
// block count per configuration and block size (whole waves, up to 512
// threads, one row of P nodes per pass) of the row-wise mesh kernels
int row_blocks(int nb, int P);
int row_threads(int P);
int launch_load(hipStream_t s, int nb, int n, int p, const double *C, const double *gw, double *b, double *partial);
void launch_sum_partials(hipStream_t s, int K, const double *partial, double *out, int nb = 1);
int launch_sub_mass_ones(hipStream_t s, int nb, int n, int p, const double *w1, const double *scal, double *v);
int launch_mass_dot(hipStream_t s, int nb, int n, int p, const double *w1, const double *v, double *partial);
void launch_sub_const(hipStream_t s, int nb, size_t per, double invV, const double *scal, double *v);
// Multigrid kernels in the arithmetic type T (double, or float for the
// mixed-precision preconditioner); instantiated for both in k_mesh.hip.
// launch_apply returns its blocks per configuration (the K of kApplyDot);
// s0 is the first-step coefficient of the kChebZ2 / kChebZ3 modes.
template <class T>
int launch_apply(hipStream_t s, int nb, const LevelOpT<T> &op, const T *x, const T *f, T *out, const T *xprev, T *xo,
                 T c1, T c2, int mode, double *partial, T s0 = T(0));
int apply_blocks(const LevelOp &op);
template <class T>
void launch_cheb_first(hipStream_t s, int nb, const LevelOpT<T> &op, const T *f, T *x, T c2);
// Fine-level residual f - K x restricted from p = 5 to p = 3 without storing
// it: the operator tiles (2^3 elements, n even) write 7^3 partial coarse
// values each into part (nb n^3 / 8 * 343 values); launch_restrict_sum adds
// them into the coarse right side fc.  Returns -1 when the level or the
// transfer is not the supported pair.
template <class T>
int launch_apply_restrict(hipStream_t s, int nb, const LevelOpT<T> &op, const TransferT<T> &tr, const T *x,
                          const T *f, T *part);
template <class T>
void launch_restrict_sum(hipStream_t s, int nb, int n, const T *part, T *fc);
template <class T>
int launch_transfer(hipStream_t s, int nb, const TransferT<T> &tr, const T *in, T *out, bool restrict_);
template <class T>
void launch_coarse_solve(hipStream_t s, int nb, int Pn, const double *V, const double *lam, const T *f, T *x);
void launch_to_f32(hipStream_t s, size_t n, const double *a, float *b);
// partial[0, nb K): block sums of z.r; partial[nb K, 2 nb K): z.q (0 if q is null); returns K
int launch_dot2_f32(hipStream_t s, int nb, size_t per, const float *z, const double *r, const double *q,
                    double *partial);
void launch_pcg_scalars(hipStream_t s, int nb, int step, double rtol, const PcgScalars &sc);
int launch_dot(hipStream_t s, int nb, size_t per, const double *a, const double *b, double *partial);
// PCG updates.  r_out = r_in - alpha q with block partials of r_out . r_out
// (returns K); x += alpha p (x = alpha p unless xinit) fused with the next
// direction p = z + beta p; p = z; the last x update after the loop.
int launch_r_update(hipStream_t s, int nb, size_t per, const double *alphas, const double *q, const double *r_in,
                    double *r_out, double *partial, float *rf = nullptr);   // rf: float32 copy of r_out (or null)
template <class ZT>
void launch_xp_update(hipStream_t s, int nb, size_t per, const double *alphas, const double *betas, const ZT *z,
                      double *p, double *x, bool xinit);
template <class ZT>
void launch_p_init(hipStream_t s, int nb, size_t per, const ZT *z, double *p);
void launch_x_final(hipStream_t s, int nb, size_t per, const double *alphas, const double *p, double *x, bool xinit);
void launch_scale(hipStream_t s, size_t n, double sc, const double *a, double *b);
void launch_hash_fill(hipStream_t s, size_t n, uint32_t seed, double *v);
void launch_fdm_scale(hipStream_t s, size_t total, int P, int i0, const double *lam, double *X);
void launch_copy_f64(hipStream_t s, size_t n, const double *a, double *b);

}  // namespace fep3m
