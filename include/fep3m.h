/*
 * fep3m.h - C ABI of the MI355X finite-element P3M library.
 *
 * Computes periodic 1/R potentials and energies of N point charges in the
 * cube [0, L]^3 by the finite-element P3M method of Beams, Olson & Freund
 * ("A Finite Element Based P3M Method for N-body Problems"):
 *
 *   Phi_i = sum_n sum'_j Q_j / |x_i - x_j + n L|            (eq. potential)
 *   U     = 1/2 sum_i Q_i Phi_i                             (eq. potentialenergy)
 *
 * split as Phi = Phi_sr + Phi_sm (eq. phisplit) with polynomial screens
 * (Section 2.1): a near-field pair sum minus the potential of the screens in
 * the (2 n_sr + 1)^3 block of elements around each charge (eq. sc, the
 * self term of Section 2.5 included), plus an order-p finite element
 * solution of the periodic Poisson problem for the screens (Section 2.2),
 * evaluated at the charges (eq. evalsmooth).  The screen is the
 * one-element-support variant of the Discussion (Section 5) with degree q;
 * the mesh uses order p = q + 2.  Screen-potential tables are order-p
 * Dirichlet finite element solutions on a larger box (Remark, Section 4).
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer on the context's device,
 *     owned by the caller; the library never frees or retains it.
 *   - x is N x 3, xyz interleaved (x[3 i + k]); Q, Phi are length N;
 *     F is N x 3 interleaved.  Outputs are in the caller's particle order.
 *   - Positions may be any finite reals; they are wrapped periodically.
 *   - Charges must be neutral: |sum Q| <= 1e-10 sum |Q| (the periodic
 *     problem is only solvable for neutral charge, Section 2.2).
 *   - Calls are ordered on the context's stream (default: the null stream)
 *     and have completed when they return.
 *   - A context is not thread safe; use one context per stream.
 *   - Functions return FEP3M_OK (0) or a negative status; no exception
 *     crosses the ABI.  fep3m_last_error() gives a message for the last
 *     failure on a context.
 */
#ifndef FEP3M_H
#define FEP3M_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fep3m_ctx fep3m_ctx;

enum {
  FEP3M_OK = 0,
  FEP3M_ERR_ARG = -1,           /* invalid argument (size, pointer, option)        */
  FEP3M_ERR_NOT_NEUTRAL = -2,   /* |sum Q| > 1e-10 sum |Q|                         */
  FEP3M_ERR_NONFINITE = -3,     /* NaN or Inf in x or Q                            */
  FEP3M_ERR_NOT_CONVERGED = -4, /* mesh solve missed mg_rtol within mg_max_iter     */
  FEP3M_ERR_DEVICE = -5,        /* HIP runtime error                               */
  FEP3M_ERR_OOM = -6,           /* device allocation failed                        */
  FEP3M_ERR_UNSUPPORTED = -7    /* valid request the library does not implement     */
};

enum {
  FEP3M_PRECISION_FP64 = 0,     /* every stage in float64                          */
  FEP3M_PRECISION_MIXED = 1     /* float32: the near-pair sum and its gradient,
                                   the interpolation (both with Kahan-compensated
                                   per-charge sums), the near-screen field (slab
                                   sums compensated) and the multigrid V-cycle
                                   that preconditions the mesh solve; float64:
                                   the PCG iteration around it (operator apply,
                                   updates, residual norms), the coarse-grid
                                   solve, the mean-zero projections, the moments,
                                   the moment adjoint and every reduction to U.
                                   Results agree with FP64 to about 1e-6
                                   relative RMS (Phi, U, F, dU/dQ).               */
};

/* Mesh solvers (Section 2.2 leaves the solver open; the paper uses an
 * AMG-preconditioned Krylov method). */
enum {
  FEP3M_SOLVER_MG = 0,   /* PCG with a p/h multigrid V-cycle (Chebyshev-Jacobi
                            smoothing), iterated to mg_rtol                     */
  FEP3M_SOLVER_FDM = 1   /* exact periodic solve by fast diagonalisation.  On
                            meshes whose edge is a power of two in [8, 64]:
                            the 1-D operators are block circulant over the
                            element index, so a DFT over the element lattice
                            leaves p x p Hermitian pencils per frequency,
                            diagonalised once at create; each solve gathers
                            the vector into element-major channels (two real
                            systems per complex one), runs 3-D FFTs, divides
                            by lam_x + lam_y + lam_z in each frequency's
                            eigenbasis and transforms back.  Other meshes: the
                            P x P pencil K1 v = lam M1 v (host, about 2 s for
                            320 nodes per axis) and dense tiled transforms
                            along x, y, z.  float64 in both precisions;
                            mg_rtol is not used (the achieved residual is
                            still measured and must be <= 1e-9).            */
};

/* Screen supports (Section 2.1 and the Discussion, Section 5). */
enum {
  FEP3M_SUPPORT_ONE = 0,  /* screens interior to the charge's element: degree q
                             cancels d = q - 2 moments per axis (R^-q decay) */
  FEP3M_SUPPORT_27 = 1    /* the order-q Lagrange functions of the nodes of the
                             closed element (equispaced order-q nodes): support
                             of 3^3 elements, d = q moments per axis cancelled
                             (R^-(q+2) decay)                                 */
};

/* Boundary conditions (Section 2.6). */
enum {
  FEP3M_BOUNDARY_PERIODIC = 0,  /* the periodic cube (the method's main case) */
  FEP3M_BOUNDARY_GROUNDED = 1,  /* Phi = 0 on the faces of the box [0, L]^3: the
                             mesh potential takes the boundary values -Phi_sr
                             of the charges of the near block (eq. bcadjust with
                             g = 0), the near block is cut at the faces and
                             nothing wraps.  Charges must lie strictly inside
                             the box (else the call returns FEP3M_ERR_ARG); the
                             net charge is free.  Needs one-element screens
                             (q = 2..4), float64, solver = FEP3M_SOLVER_FDM
                             (the interior pencil diagonalised by dense
                             transforms) and near_field DIRECT or AUTO; no
                             use_graph, no static storage (else create returns
                             FEP3M_ERR_UNSUPPORTED).  Forces and dU/dQ come
                             from the adjoint with two more terms: the
                             boundary values depend on the moments (tables)
                             and on the positions (near pairs).  Charges
                             within about half an element of a face are
                             resolved poorly: their images lie within h of the
                             face, where the mesh cannot follow them.        */
  FEP3M_BOUNDARY_INSULATED = 2  /* dPhi/dn = 0 on the faces of the box [0, L]^3:
                             the mesh potential has the normal derivative
                             -dPhi_sr/dn there, a surface load on the faces'
                             nodes (tensor Gauss rule of 10 x 10 points per
                             element face, the near sums of the face's element
                             and its screen field differentiated exactly); the
                             load is projected on the compatible subspace and
                             the pure-Neumann system solved on every node with
                             the constant mode dropped (int phi = 0): Phi is
                             defined up to a constant, U of neutral charges is
                             not.  Charges must be neutral and strictly inside
                             the box; the same restrictions as GROUNDED.
                             Forces and dU/dQ by the adjoint with the surface
                             load's dependence on the moments and positions  */
};

/* Evaluation of the near-screen field and of its transpose in the moment
 * adjoint (Section 3, eq. sc with the Remark's tables).  Both are periodic
 * convolutions over the element lattice with the table as the kernel. */
enum {
  FEP3M_NEAR_AUTO = 0,    /* FFT when the mesh allows it (n a power of two,
                             8 <= n <= 64), else DIRECT                         */
  FEP3M_NEAR_DIRECT = 1,  /* the table sums themselves: 2 * 8 * (p+1)^3 FLOP per
                             element and near offset (matrix cores forward,
                             vector units for the transpose)                    */
  FEP3M_NEAR_FFT = 2      /* the same linear maps through the convolution
                             theorem: 3-D FFTs of the moments and node fields,
                             products with the tables' spectrum (computed at
                             create for one octant of frequencies, the tables
                             being symmetric under axis reflections:
                             (n/2 + 1)^3 x 8 x (p+1)^3 complex float64, 0.99 GB
                             at n = 64).  float64 in both precisions;
                             n must be a power of two in [8, 64] (else create
                             returns FEP3M_ERR_UNSUPPORTED).  Agrees with
                             DIRECT to about 1e-14 relative (Phi, F).           */
};

typedef struct {
  int32_t n_sr;          /* near block radius in elements (default 3: 7^3 block,
                            the paper's short-range list, Section 4)             */
  int32_t precision;     /* FEP3M_PRECISION_*                                    */
  double  mg_rtol;       /* relative residual target of the mesh solve (1e-7,
                            the single-precision level the paper's example
                            calculations solve to, Section 4)                   */
  int32_t mg_max_iter;   /* PCG iteration cap (60)                               */
  int32_t cheb_degree;   /* Chebyshev smoothing degree per V-cycle side (3)      */
  int32_t table_box;     /* elements per axis of the table domain, odd,
                            > 2 n_sr + 1 (default 2 n_sr + 9)                    */
  int32_t autotune;      /* 1 (default): the first evaluation times the pair
                            sum's work decompositions (one wave per element;
                            persistent waves over a queue of target chunks of
                            several sizes and grid sizes; in float64 also
                            workgroups of up to 256 targets of one row of
                            elements against LDS-staged source rows) and
                            keeps the fastest; 0: one wave per element; 2:
                            the row form (float64 only).  The first two give
                            bit-identical results, the row form sums each
                            charge's pairs in another order (equal to
                            rounding).                                         */
  int32_t use_graph;     /* 1: run each evaluation as one captured hipGraph
                            replay on an internal stream ordered after the
                            caller's stream, on context copies of the inputs
                            and outputs (copied in and out around the replay).
                            The graph is captured after an eager call and
                            reused while the same outputs are requested; each
                            mesh solve runs the iteration
                            count of that eager call (a configuration that
                            converges earlier stops changing), and after each
                            replay the input checks and the final residuals are
                            read back: a replay that falls short of mg_rtol is
                            redone eagerly and the graph captured again.
                            Results are identical to eager calls.  0 (default):
                            eager launches.  Not used while profiling is on,
                            nor with solver = FEP3M_SOLVER_FDM.                */
  int32_t solver;        /* FEP3M_SOLVER_* (default: multigrid-preconditioned CG) */
  int32_t near_field;    /* FEP3M_NEAR_* (default AUTO)                          */
  int32_t pair_stream;   /* 1 (default): on meshes of at least 2^16 elements
                            the near-pair sum of a tuned context runs on a
                            second stream beside the assignment and the mesh
                            solve; 0: every launch on the caller's stream      */
  int32_t support;       /* FEP3M_SUPPORT_* (default ONE).  Every family but the
                            one-element q = 3 screen runs in float64 with the
                            direct near field (matrix cores from 8 moments per
                            element, vector units for one); create returns
                            FEP3M_ERR_UNSUPPORTED for precision = MIXED or
                            near_field = FFT there, and for element orders
                            above 6 (one-element q = 5, 6)                     */
  int32_t boundary;      /* FEP3M_BOUNDARY_* (default PERIODIC)                  */
} fep3m_options;

typedef struct {
  int32_t mg_iterations;     /* PCG iterations of the last mesh solve            */
  double  mg_rel_residual;   /* ||b - K phi|| / ||b|| reached                     */
  int64_t near_pairs;        /* ordered near pairs (i, j), j != i, of the last call */
  int32_t max_per_element;   /* largest element occupancy of the last call        */
  int32_t adj_iterations;    /* PCG iterations of the second (adjoint) mesh solve */
  int32_t mg_levels;         /* levels of the multigrid hierarchy                */
  double  create_seconds;    /* wall time of create (tables, hierarchy)           */
  int64_t generation;        /* successful potential/energy/energy_forces calls
                                on this context; names the state fep3m_backward
                                reuses                                            */
  int32_t pair_variant;      /* pair-sum decomposition in use: 0 one wave per
                                element, 1 persistent waves over a work queue     */
  int32_t pair_item_targets; /* targets per work item (variant 1)                 */
  int32_t pair_waves;        /* persistent waves launched (variant 1)             */
  double  tune_ms_best;      /* device time of the chosen variant when tuned      */
  double  tune_ms_default;   /* device time of one wave per element when tuned    */
  int64_t graph_replays;     /* evaluations served by a graph replay (use_graph)  */
  int32_t near_fft;          /* 1: the near field and its transpose run as FFTs   */
  int64_t device_bytes;      /* device memory the context holds                   */
} fep3m_stats;

/* Profile slots: stages of one call, the fine-level operator launches, and
 * the whole call.  `work` holds the algorithmic work of the slot: floating
 * point operations for NEAR and ADJ_NEAR on the direct path (2 * 8 * (p+1)^3
 * per element and near offset) and PAIR (11 per ordered near pair, 20 when
 * forces are accumulated in the same pass); bytes that must cross HBM for
 * NEAR and ADJ_NEAR on the FFT path (what each of their launches reads and
 * writes: the table spectrum once per product, every FFT pass's array in and
 * out) and for FINE_APPLY (the vectors each launch reads and writes, 8 bytes
 * per DOF each) and for MOMENTS (sorted positions and charges in, 32 bytes
 * per charge, the element starts and moments), LOAD (the moments in, the
 * load vector out), DEPOSIT (positions and charges in, the per-element
 * deposits out and back in, the assembled vector out) and INTERP_KERNEL
 * (per charge its position, pair potential and slot in and three potentials
 * out, 60 bytes, plus the element field once); 0 elsewhere. */
enum {
  FEP3M_PROF_SORT = 0,        /* wrap, bin, counting sort, gather          */
  FEP3M_PROF_ASSIGN = 1,      /* element moments, load assembly, projection */
  FEP3M_PROF_SOLVE = 2,       /* multigrid-PCG mesh solve and gauge        */
  FEP3M_PROF_NEAR = 3,        /* near-screen field (one launch per call)    */
  FEP3M_PROF_PAIR = 4,        /* near-pair sum (one launch per call)        */
  FEP3M_PROF_INTERP = 5,      /* interpolation, combination, energy         */
  FEP3M_PROF_FINE_APPLY = 6,  /* every fine-level operator launch           */
  FEP3M_PROF_TOTAL = 7,       /* whole call                                 */
  FEP3M_PROF_ADJ_SOLVE = 8,   /* forces: deposit, assembly, second mesh solve */
  FEP3M_PROF_ADJ_NEAR = 9,    /* forces: moment adjoint (transposed near field) */
  FEP3M_PROF_FORCES = 10,     /* forces: per-charge gradient and dU/dQ      */
  FEP3M_PROF_FINE_APPLY_F32 = 11, /* fine-level operator launches in float32
                                     (mixed-precision preconditioner)     */
  FEP3M_PROF_MOMENTS = 12,    /* element moments kernel (inside ASSIGN)   */
  FEP3M_PROF_LOAD = 13,       /* load assembly kernel (inside ASSIGN)     */
  FEP3M_PROF_DEPOSIT = 14,    /* forces: charge deposit and its assembly  */
  FEP3M_PROF_INTERP_KERNEL = 15, /* interpolation kernel (inside INTERP)  */
  FEP3M_PROF_SLOTS = 16
};

typedef struct {
  double  ms[FEP3M_PROF_SLOTS];     /* accumulated device time (hipEvents)     */
  int64_t count[FEP3M_PROF_SLOTS];  /* calls (stage slots) or kernel launches  */
  double  work[FEP3M_PROF_SLOTS];   /* accumulated algorithmic work (above)    */
} fep3m_profile;

/* Fill *opt with the defaults listed above.  Returns FEP3M_ERR_ARG on NULL. */
int fep3m_default_options(fep3m_options *opt);

/* Create a context for N charges in the periodic cube [0, L]^3 meshed by
 * dims[0] x dims[1] x dims[2] elements (cubic meshes only: all three equal),
 * screens of degree q with the support of opt->support, mesh order
 * p = q + 2: one-element screens (Section 5) for q = 2..4 (q = 3, the lowest
 * degree that cancels monopole and dipole, is the default and the fastest
 * path), 27-element screens (Section 2.1) for q = 1..4.
 * Precomputes the 1-D element matrices, screens, near-field tables and the
 * multigrid hierarchy, and allocates every device buffer the evaluation
 * needs.  Errors: FEP3M_ERR_ARG for L <= 0 or non-finite, N < 2,
 * dims < 2 n_sr + 1 or unequal, q out of range for the support (2..6 one
 * element, 1..4 27 elements), bad options; FEP3M_ERR_UNSUPPORTED as listed
 * under fep3m_options.support;
 * FEP3M_ERR_OOM, FEP3M_ERR_DEVICE.  *out is NULL on failure. */
int fep3m_create(double L, int64_t N, const int32_t dims[3], int32_t q, fep3m_ctx **out);
int fep3m_create_ex(double L, int64_t N, const int32_t dims[3], int32_t q,
                    const fep3m_options *opt, fep3m_ctx **out);

/* A batch of nconf independent configurations that share L, the mesh and
 * the options (spec extension: many small systems in one pass).
 * Configuration b holds N_per_conf[b] >= 2 charges; every array argument of
 * the evaluation calls concatenates the configurations in order (x is
 * (sum N) x 3, Phi, Q and dUdQ have sum N entries, F (sum N) x 3), and U
 * receives nconf energies, U[b] for configuration b.  Each configuration
 * must be neutral on its own.  Every kernel launch covers all
 * configurations; the mesh solves of all configurations iterate together
 * and each stops changing once its own residual reaches mg_rtol.
 * 1 <= nconf <= 1024, nconf * dims^3 <= 2^28.  fep3m_create_ex is the
 * nconf = 1 case.  Errors as fep3m_create_ex. */
int fep3m_create_batch(double L, int32_t nconf, const int64_t *N_per_conf, const int32_t dims[3], int32_t q,
                       const fep3m_options *opt, fep3m_ctx **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): fep3m_create_ex
 * for one configuration with every device buffer placed in a static device
 * array of 192 MiB that the library holds on each GPU it runs on until the
 * process ends (enough for 16^3 elements and about 10^5 charges; the
 * context's need is fep3m_stats.device_bytes of a fep3m_create_ex context).
 * No hipMalloc, hipFree, pinned host allocation, stream, event or library
 * handle is created, at create or in any evaluation call on the context;
 * host-side setup uses ordinary heap memory.  Evaluation calls behave as on
 * a fep3m_create_ex context with autotune = 0 (one wave per element for the
 * pair sum, on the caller's stream only).  One static context per device at
 * a time: the array keeps the last context's contents and is cleared at
 * create; while a static context lives, fep3m_create_static on the same
 * device returns FEP3M_ERR_ARG, and fep3m_destroy releases it.  Calls on
 * static contexts of different threads must not overlap.  Errors:
 * FEP3M_ERR_ARG when the context needs more than the array holds (the
 * message names the buffer) or the array is held, FEP3M_ERR_UNSUPPORTED for
 * use_graph = 1 or solver = FEP3M_SOLVER_FDM, else as fep3m_create_ex. */
int fep3m_create_static(double L, int64_t N, const int32_t dims[3], int32_t q, const fep3m_options *opt,
                        fep3m_ctx **out);

/* Order subsequent calls on the given hipStream_t (NULL: null stream).
 * Inside a call (eager, or a graph replay) the near-pair sum may run on a
 * second stream that the context owns (default priority), forked from and
 * joined back into this stream before the call's later work, so every output
 * is ordered on this stream when the call returns. */
int fep3m_set_stream(fep3m_ctx *ctx, void *hip_stream);

/* Phi[i] for every charge (eq. potential evaluated by the method). */
int fep3m_potential(fep3m_ctx *ctx, const double *x, const double *Q, double *Phi);

/* Phi as above and U = 1/2 sum Q_i Phi_i written to U[0] (device pointer,
 * one double per configuration of a batch); the sum is a fixed-order
 * float64 tree. */
int fep3m_energy(fep3m_ctx *ctx, const double *x, const double *Q, double *Phi, double *U);

/* Energy and forces (spec extension; the paper evaluates potentials
 * only, Section 5).  U[0] = 1/2 sum Q_i Phi_i as in fep3m_energy, and the
 * exact gradient of that discrete energy: F[3 i + k] = -dU/dx_ik (the
 * near-pair term is recomputed in the pair pass, the mesh terms come from a
 * deposit of the charges on the order-p basis, a second mesh solve and the
 * transposed near-screen correlation).  The method's operators are not
 * symmetric (no exact momentum conservation, Section 5), so sum_i F_i is
 * not exactly zero and dU/dQ differs from Phi; U is discontinuous where a
 * charge crosses an element face, and F is the gradient inside elements.
 * Phi (length N) and dUdQ (length N) may be NULL.  All device pointers. */
int fep3m_energy_forces(fep3m_ctx *ctx, const double *x, const double *Q, double *U, double *F);
int fep3m_energy_forces_ex(fep3m_ctx *ctx, const double *x, const double *Q, double *Phi, double *U,
                           double *F, double *dUdQ);

/* Reverse pass of the last successful fep3m_potential / fep3m_energy /
 * fep3m_energy_forces call on ctx, for callers that split the forward
 * evaluation from the gradient (an autograd backward): F[3 i + k] = -dU/dx_ik
 * and dUdQ[i] = dU/dQ_i exactly as fep3m_energy_forces_ex would return them
 * for that call's x and Q.  It reuses that call's bins, sorted charges, mesh
 * potential and per-element mesh-minus-near-screen field, recomputes the
 * near-pair gradients (they are not kept by the forward call), and runs the
 * deposit, second mesh solve and moment adjoint.  `generation` must equal
 * fep3m_stats.generation read right after that call: any later call
 * overwrites the state, and FEP3M_ERR_ARG is returned then (and when the
 * last call failed, or both outputs are NULL).  F (N x 3) or dUdQ (N) may
 * be NULL.  Device pointers, caller-owned. */
int fep3m_backward(fep3m_ctx *ctx, int64_t generation, double *F, double *dUdQ);

/* Copy an internal stage of the last evaluation to the device buffer `out`
 * of `out_bytes` bytes (test and diagnostic use).  Stages:
 *   0 perm     int32  [N]        caller index of each sorted slot
 *   1 start    int32  [n^3 + 1]  first sorted slot of each element
 *   2 C        double [n^3 * (d + 1)^3]  element screen moments (element
 *                                units; (d + 1)^3 = 8 for the default screen)
 *   3 b        double [(p n)^3]  load vector after projection ([z][y][x]);
 *                                in a box [(p n + 1)^3]: the volume load
 *                                (insulating box: plus the surface load,
 *                                projected on the compatible subspace)
 *   4 phi      double [(p n)^3]  mesh potential, zero mean (element units);
 *                                in a box [(p n + 1)^3] with its boundary
 *                                values (grounded) or int phi = 0 (insulating)
 *   5 Phi_p    double [N]        near pair sum, caller order, physical units
 *   6 Phi_m    double [N]        mesh minus near-screen term, caller order
 *   7 T        double [8 * (2 n_sr + 1)^3 * (p + 1)^3]  tables (element units)
 * Returns FEP3M_ERR_ARG when out_bytes is too small or the stage unknown. */
int fep3m_debug_stage(fep3m_ctx *ctx, int32_t stage, void *out, int64_t out_bytes);

/* Number of bytes fep3m_debug_stage needs for a stage (0 if unknown). */
int64_t fep3m_stage_bytes(const fep3m_ctx *ctx, int32_t stage);

/* Turn per-stage device timing on (1) or off (0) and clear the profile.
 * While on, every call records hipEvents on the context's stream around
 * each stage and each fine-level operator launch.  When the near-pair sum
 * runs on the second stream (tuned calls, one wave per element) its time
 * overlaps that of ASSIGN, SOLVE and NEAR, which then include the slowdown
 * from sharing the GPU, and TOTAL is less than the sum of the stages. */
int fep3m_set_profiling(fep3m_ctx *ctx, int32_t on);

/* Accumulated profile since the last fep3m_set_profiling. */
int fep3m_get_profile(const fep3m_ctx *ctx, fep3m_profile *prof);

/* Counters of the last call. */
int fep3m_get_stats(const fep3m_ctx *ctx, fep3m_stats *stats);

void fep3m_destroy(fep3m_ctx *ctx);

/* Message of the last failure on ctx ("" if none); valid until the next call. */
const char *fep3m_last_error(const fep3m_ctx *ctx);

/* Static description of a status code. */
const char *fep3m_status_string(int status);

/* The create-time near-field tables on the host (no device needed), for
 * inspection and tests: order-p Dirichlet FE solutions of the basis screens
 * on a box of `box` elements (Remark, Section 4), element units, layout as
 * debug stage 7: T[a][D][m], a = ax + nl ay + nl^2 az with nl = d + 1 moments
 * per axis (d = q - 2 for support FEP3M_SUPPORT_ONE, q for
 * FEP3M_SUPPORT_27), D the target-minus-source element offset in
 * [-n_sr, n_sr]^3 (x fastest), m the node of the order p = q + 2 element
 * (x fastest).  out (host memory, caller-owned) must hold
 * out_len >= nl^3 (2 n_sr + 1)^3 (q + 3)^3 doubles.  Returns FEP3M_ERR_ARG
 * for a degree outside 2..6 (one element) or 1..4 (27 elements), an unknown
 * support, n_sr outside 1..3, an even box or box <= 2 n_sr + 1, or a short
 * buffer. */
int fep3m_host_tables(int32_t q, int32_t support, int32_t n_sr, int32_t box, double *out, int64_t out_len);

#ifdef __cplusplus
}
#endif

#endif /* FEP3M_H */
