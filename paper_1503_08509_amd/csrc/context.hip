// Context, pipeline orchestration and the C ABI (include/fep3m.h).
//
// Per call (Algorithm 1): bin and sort the charges by element, form the
// per-element screen moments, assemble the load, solve the periodic mesh
// problem by multigrid-preconditioned conjugate gradients, then evaluate
// the near-screen field, the near-pair sum and the interpolation, and
// combine.  Every buffer is allocated at create; a call allocates nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "fep3m.h"
#include "host_fe.hpp"
#include "host_tables.hpp"

#include "kernels.hpp"

using namespace fep3m;

namespace {

struct Status : std::runtime_error {
  int code;
  Status(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory) throw Status(FEP3M_ERR_OOM, std::string(what) + ": out of device memory");
  if (e != hipSuccess) throw Status(FEP3M_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
T *dalloc(size_t count, const char *what) {
  void *p = nullptr;
  hip_check(hipMalloc(&p, count * sizeof(T) + 64), what);
  return static_cast<T *>(p);
}

// Device-time profile (hipEvents on the context stream).
struct Profiler {
  bool on = false;
  hipEvent_t stage_ev[2 * FEP3M_PROF_SLOTS] = {};
  std::vector<hipEvent_t> kev;   // begin/end pairs for fine-level operator launches
  std::vector<double> kwork;     // bytes of each recorded launch
  std::vector<int> kslot;        // profile slot of each recorded launch
  int kused = 0;
  unsigned marked = 0;        // slots recorded in the current call
  bool pair_forces = false;   // the current call's pair pass accumulated gradients
  bool near_both = false;     // the near-field stage also transformed the deposits (FFT path)
  bool adj_full = false;      // the moment-adjoint stage ran the deposits' transforms itself
  fep3m_profile acc{};
  void begin_call() {
    kused = 0;
    marked = 0;
  }
};

// Vectors of one multigrid level in one arithmetic type.
template <class T>
struct LevelVecs {
  T *x = nullptr, *x2 = nullptr, *f = nullptr, *r = nullptr;
};

struct MGLevel {
  LevelOp op{};
  LevelOpF opf{};           // float32 copy (mixed-precision preconditioner)
  size_t ndof = 0;
  LevelVecs<double> vd;
  LevelVecs<float> vf;
  double *d = nullptr;      // power-iteration work vector
  double lmax = 0.0;
  template <class T> LevelVecs<T> &vec();
  template <class T> const LevelOpT<T> &oper() const;
};
template <> LevelVecs<double> &MGLevel::vec<double>() { return vd; }
template <> LevelVecs<float> &MGLevel::vec<float>() { return vf; }
template <> const LevelOp &MGLevel::oper<double>() const { return op; }
template <> const LevelOpF &MGLevel::oper<float>() const { return opf; }

}  // namespace

// Device storage of contexts made by fep3m_create_static: one array per
// GPU the library runs on, held until the process ends.  Its device address
// comes from hipGetSymbolAddress (the array's name is only a host-side
// stand-in), taken once per device with that device current and kept in
// g_static_ptr; one static context may hold a device's array at a time.
constexpr size_t kStaticBytes = size_t(192) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};
bool g_static_busy[kMaxDevices] = {};
}  // namespace

// Per-configuration scalar slots (nb values each).
enum CfgScalar : int {
  kCsQ = 0,        // sum Q
  kCsQabs = 1,     // sum |Q|
  kCsLoad = 2,     // sum b (compatibility projection of the load)
  kCsSpare = 3,    // unused (the gauge integrals have a buffer of 2 nb values)
  kCsEnergy = 4,   // sum Q Phi
  kCsAdjLoad = 5,  // sum G (compatibility projection of the deposit)
  kCsPcg = 6,      // 10 PCG scalars from here
  kCsFwdRel = 16,  // final relative residual of the forward mesh solve
  kCsAdjRel = 17,  // final relative residual of the adjoint mesh solve
  kCsSlots = 18
};

struct fep3m_ctx {
  // configuration
  double L = 1.0, h = 1.0;
  int64_t N = 0;                // charges in the whole batch
  int nb = 1;                   // independent configurations (same mesh and parameters)
  std::vector<int> off_h;       // first charge of each configuration (nb + 1 entries)
  int *off_d = nullptr;
  double *cs = nullptr, *host_cs = nullptr;   // per-configuration scalars (device, pinned mirror)
  // Systems in the current mesh solve: nb, or 2 nb when the forward and the
  // adjoint systems of every configuration are solved together (the adjoint
  // right side does not depend on phi).  Their vectors are consecutive
  // blocks: b then G, phi then lambda.
  int nbs = 1;
  PcgScalars pcs{};                 // 2 nb values per scalar
  double *gauge = nullptr;          // 2 nb integrals of the solutions (gauge)
  bool lam_ready = false;           // the last forward call also solved for lambda
  bool adj_near_ready = false;      // ... and transformed the moment adjoint's near part (FFT path)
  double *cfgs(int slot) const { return cs + size_t(slot) * nb; }
  int n = 0, q = 3, p = 5, d = 1, nsr = 3, B = 15;
  // screens: nl = d + 1 moments per axis, na = nl^3, span elements per axis
  // of an element's screens; `generic` for every family but the one-element
  // q = 3 screen (their float64 kernels are in k_screens.hip)
  int nl = 2, na = 8, span = 1;
  bool generic = false;
  // boxes (boundary = FEP3M_BOUNDARY_GROUNDED or _INSULATED, Section 2.6):
  // mesh vectors of Pb = p n + 1 nodes per axis ([z][y][x] per
  // configuration), the 1-D stiffness and mass of the box as class-row band
  // tables, and the eigenbasis of the interior pencil
  // (K1_II V = M1_II V Lambda, V^T M1_II V = I)
  bool box = false;
  bool insulated = false;   // boundary = FEP3M_BOUNDARY_INSULATED (else grounded)
  int Pb = 0;
  double *bxb = nullptr, *bxphi = nullptr, *bxy = nullptr, *bxt1 = nullptr, *bxt2 = nullptr, *bxt3 = nullptr;
  double *bxg = nullptr, *bxlam = nullptr;   // reverse pass: assembled deposit, adjoint potential
  // insulating box: eigenbasis of the whole box pencil (its constant mode
  // at index bx_i0), the mass row sums, the face quadrature and face values
  double *bxVf = nullptr, *bxLamf = nullptr, *bxw1 = nullptr, *bxtF = nullptr;
  double *bxLw = nullptr, *bxhF = nullptr;   // reverse pass: face weights of lambda, face adjoint weights
  int bx_i0 = 0;
  BoxQuad bxquad{};
  double *bxV = nullptr, *bxLam = nullptr;
  double *bxKb = nullptr, *bxMb = nullptr, *bxt4 = nullptr;   // the 1-D matrices as bands; operator work vector
  BoxNodes bxnodes{};
  fep3m_options opt{};
  hipStream_t stream = nullptr;
  std::string err;
  fep3m_stats stats{};
  uint64_t generation = 0;   // successful evaluations so far
  bool fwd_valid = false;    // buffers hold the state of evaluation `generation`
  std::vector<void *> allocs;
  size_t dev_bytes = 0;        // device memory the context holds
  // static contexts: every device buffer is carved from the device's static
  // array (no hipMalloc), host mirrors are ordinary host memory (no pinned
  // allocation)
  unsigned char *arena = nullptr;
  size_t arena_used = 0;
  int arena_dev = -1;
  std::vector<double> host_cs_buf, host_scal_buf;
  Profiler prof;

  // precompute
  std::vector<double> T_host;
  double *T = nullptr, *Tt = nullptr, *gw = nullptr, *w1 = nullptr;
  GllBasis bas{};
  // near field by FFTs: table spectrum, twiddles exp(-2 pi i j / n), the
  // transformed moments / moment adjoint (4 complex channels), near-screen
  // field and deposits (108 complex channels)
  bool near_fft = false;
  double2 *spec = nullptr, *twd = nullptr, *zc = nullptr, *za = nullptr, *zpsi = nullptr, *zg = nullptr;

  // particles
  double *gtmp = nullptr, *sg = nullptr, *sQ = nullptr;
  int *elem = nullptr, *slot = nullptr, *count = nullptr, *start = nullptr, *tmp = nullptr, *perm = nullptr;
  int *scan_scr = nullptr;   // tile sums and maxima of the counting-sort scans
  int *flags = nullptr, *maxcount = nullptr;
  unsigned long long *paircount = nullptr;
  double *C = nullptr, *Wel = nullptr, *phip_s = nullptr, *phim_s = nullptr, *phi_s = nullptr;
  double *lsep = nullptr;   // scratch of the separable load and adjoint passes (periodic screen families)
  // mixed precision: float32 tables, element field, local coordinates
  float *Tf = nullptr, *Welf = nullptr;
  float4 *su = nullptr;
  int4 *si = nullptr;
  int *sel = nullptr;
  double *partial = nullptr, *scal = nullptr;
  size_t partial_len = 0;
  double *host_scal = nullptr;  // pinned

  // mesh
  std::vector<MGLevel> lv;
  std::vector<Transfer> tr;
  std::vector<TransferF> trf;
  // fine-level residual restricted inside the operator (p 5 -> 3, n even):
  // per-tile partial coarse values, float64 or float32 like the V-cycle
  bool fuse_rr = false;
  double *rrp_d = nullptr;
  float *rrp_f = nullptr;
  template <class T> T *rr_part() const;
  bool mixed = false;        // float32 V-cycle, float32 near field and interpolation
  template <class T> const TransferT<T> &transfer(int l) const;
  double *dot_scr = nullptr; // two-dot partials of the mixed PCG
  double *coarseV = nullptr, *coarseLam = nullptr;
  int coarseP = 0;
  double *b = nullptr, *sol = nullptr, *rr = nullptr, *pv = nullptr, *qv = nullptr;
  // fast-diagonalisation solver: 1-D eigenvectors (column-major, V[i + j P]:
  // node i, mode j, M1-orthonormal) and eigenvalues of the fine pencil
  double *fdmV = nullptr, *fdmLam = nullptr;
  int fdm_i0 = 0;
  // the same solve by Fourier analysis over the element lattice (meshes
  // whose edge is a power of two): per-frequency eigenvectors of the 1-D
  // blocks, twiddles, and the element-major complex work array
  bool fs_ready = false;
  double2 *fsW = nullptr, *fsTw = nullptr, *fsZ = nullptr;
  double *fsL = nullptr;
  // pair-sum work decomposition (autotuned): kind 0 one wave per element,
  // kind 1 persistent waves over items of `titem` targets, kind 2 workgroups
  // over rows of elements with LDS-staged source rows (float64)
  struct PairPlan {
    int kind = 0, titem = 0, waves = 0;
  };
  PairPlan plan;
  bool tuned = false;
  // The near-pair sum depends only on the sorted charges and is
  // instruction-bound, the mesh solve is memory-bound: once tuning is done the
  // pair pass runs on a second stream forked after the sort and joined before
  // the interpolation, overlapping the assignment, solve and near field.
  // Under graph capture the fork and the join become graph dependencies.
  // Default priority, like every stream here.
  hipStream_t pstream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  void side_stream() {   // created before any capture begins
    if (pstream) return;
    hip_check(hipStreamCreateWithFlags(&pstream, hipStreamNonBlocking), "pair stream");
    hip_check(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming), "event");
    hip_check(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming), "event");
  }
  // graph mode: the whole evaluation captured once per set of argument
  // pointers on an internal stream, then replayed
  hipStream_t gstream = nullptr;
  // the graph reads and writes context buffers; callers' arrays are copied
  // in before and out after each replay
  double *gx = nullptr, *gQ = nullptr, *gPhi = nullptr, *gU = nullptr, *gF = nullptr, *gD = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool graph_ready = false, capturing = false;
  int gmask = -1;               // outputs the captured graph produces (Phi, U, F, dUdQ bits)
  int cap_iters[2] = {0, 0};    // PCG iterations of the forward and adjoint solves in the graph
  int64_t replays = 0;
  int items_titem = -1;         // item size the current work list was built for
  int cus = 256;                // compute units of the device
  int *nit = nullptr, *item_start = nullptr, *icounter = nullptr, *iscan_max = nullptr;
  int2 *items = nullptr;
  // pair sum on rows of target elements (kind 2): row starts and work items
  int *rowstart = nullptr, *rnit = nullptr, *ritem_start = nullptr, *riscan_max = nullptr;
  int2 *ritems = nullptr;
  // adjoint
  double *gE = nullptr, *Gv = nullptr, *lam = nullptr, *Aadj = nullptr, *fpair = nullptr, *Phi_int = nullptr;

  template <class T>
  T *alloc(size_t count, const char *what) {
    const size_t bytes = count * sizeof(T) + 64;
    dev_bytes += bytes;
    if (arena) {
      const size_t at = (arena_used + 255) & ~size_t(255);
      if (at + bytes > kStaticBytes)
        throw Status(FEP3M_ERR_ARG, std::string("static storage of ") + std::to_string(kStaticBytes >> 20) +
                                        " MiB exceeded at " + what + " (the context needs more; use fep3m_create_ex)");
      arena_used = at + bytes;
      return reinterpret_cast<T *>(arena + at);
    }
    T *p = dalloc<T>(count, what);
    allocs.push_back(p);
    return p;
  }
  // host mirror of `count` doubles: pinned, or ordinary memory for static contexts
  double *host_mirror(size_t count, std::vector<double> &buf, const char *what) {
    if (arena) {
      buf.assign(count, 0.0);
      return buf.data();
    }
    double *p = nullptr;
    hip_check(hipHostMalloc(reinterpret_cast<void **>(&p), count * sizeof(double), hipHostMallocDefault), what);
    return p;
  }
  ~fep3m_ctx() {
    for (hipEvent_t e : prof.stage_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : prof.kev) (void)hipEventDestroy(e);
    for (void *p : allocs) (void)hipFree(p);
    if (!arena) {
      if (host_scal) (void)hipHostFree(host_scal);
      if (host_cs) (void)hipHostFree(host_cs);
    } else {
      std::lock_guard<std::mutex> lk(g_static_mu);
      g_static_busy[arena_dev] = false;
    }
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gstream) (void)hipStreamDestroy(gstream);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (pstream) (void)hipStreamDestroy(pstream);
  }
  void check_launch(const char *what) { hip_check(hipGetLastError(), what); }
  void sync(const char *what) { hip_check(hipStreamSynchronize(stream), what); }

  // reduce `count` partials to scal[slot] and return it on the host
  double reduce_host(int count, const double *part, int slot_) {
    launch_sum_partials(stream, count, part, scal + slot_);
    hip_check(hipMemcpyAsync(host_scal, scal + slot_, sizeof(double), hipMemcpyDeviceToHost, stream), "copy scalar");
    sync("reduce");
    return host_scal[0];
  }

  void build(double L_, const std::vector<int64_t> &Ns, int n_, int q_, const fep3m_options &o);
  void stage_mark(int slot, bool begin) {
    if (!prof.on) return;
    hip_check(hipEventRecord(prof.stage_ev[2 * slot + (begin ? 0 : 1)], stream), "event");
    if (begin) prof.marked |= 1u << slot;
  }
  // fine-level operator launch, bracketed by events when profiling
  template <class T>
  int apply0(const T *x, const T *f, T *out, const T *d, T *xo, T c1, T c2, int mode, double *part, T s0 = T(0)) {
    const bool rec = prof.on && prof.kused < int(prof.kev.size()) / 2;
    if (rec) hip_check(hipEventRecord(prof.kev[2 * prof.kused], stream), "event");
    const int K = mode == kResidualRestrict
                      ? launch_apply_restrict<T>(stream, nbs, lv[0].oper<T>(), transfer<T>(0), x, f, rr_part<T>())
                      : launch_apply<T>(stream, nbs, lv[0].oper<T>(), x, f, out, d, xo, c1, c2, mode, part, s0);
    if (K < 0) throw Status(FEP3M_ERR_UNSUPPORTED, "fine-level operator variant");
    if (rec) {
      hip_check(hipEventRecord(prof.kev[2 * prof.kused + 1], stream), "event");
      // vectors read + written: x, f, x_prev (when read) and x_new; f and x_new (x built from f);
      // x, f and x_new (x_prev built from f); x, f, r; x, Kx
      const double vec = (mode == kCheb || mode == kChebDot) ? ((c1 != T(0) && d) ? 4.0 : 3.0)
                         : (mode == kChebZ2 || mode == kResidualRestrict) ? 2.0
                         : (mode == kChebZ3 || mode == kResidual) ? 3.0 : 2.0;
      prof.kwork[prof.kused] = vec * double(sizeof(T)) * double(lv[0].ndof) * nbs;
      prof.kslot[prof.kused] = sizeof(T) == 8 ? FEP3M_PROF_FINE_APPLY : FEP3M_PROF_FINE_APPLY_F32;
      ++prof.kused;
    }
    return K;
  }
  void profile_collect();
  void forward(const double *x, const double *Q, double *Phi, double *U, bool pair_forces);
  void pair_pass(bool pair_forces);
  int pair_launch(const PairPlan &pl, bool pair_forces);
  void tune_pairs(bool pair_forces);
  void reverse(double *F, double *dUdQ);
  void finish(bool count_pairs);
  void check_inputs() {   // flags and per-configuration charge sums, already on the host
    int fl;
    std::memcpy(&fl, host_scal + 4, sizeof(int));
    if (fl & 1) throw Status(FEP3M_ERR_NONFINITE, "non-finite position or charge");
    if (fl & 2) throw Status(FEP3M_ERR_ARG, "positions must lie inside the box (0, L)^3");
    for (int bb = 0; bb < nb && !(box && !insulated); ++bb) {   // a grounded box takes any net charge
      const double sq = host_cs[kCsQ * nb + bb], sa = host_cs[kCsQabs * nb + bb];
      if (std::fabs(sq) > 1e-10 * sa)
        throw Status(FEP3M_ERR_NOT_NEUTRAL, "charges are not neutral: sum Q = " + std::to_string(sq) +
                                                (nb > 1 ? " in configuration " + std::to_string(bb) : std::string()));
    }
  }
  void backward(int64_t gen, double *F, double *dUdQ);
  void build_mg();
  void estimate_spectra();
  template <class T> int vcycle(int l, const T *f, double *dot_part = nullptr);
  template <class T> int cheb_smooth(int l, const T *f, bool zero_start, double *dot_part = nullptr);
  void solve(const double *rhs, double *out, int which);
  void fdm_solve(const double *rhs, double *out, int which);
  void build_fdm();
  void build_box();
  void box_apply(const double *v, double *y);
  void box_solve(const double *rhs, double *sol, int which, bool zero_boundary = false);
  // the one-element q = 3 screen (p = 5, 2 moments per axis), which has
  // kernels of its own for the near field and the moment adjoint
  bool std_screen() const { return p == 5 && nl == 2 && span == 1; }
  // moment adjoint in a box (near part from the deposit gE, mesh part from bxlam)
  int box_adjoint_moments() {
    return std_screen() ? launch_adj_moments(stream, nb, p, n, nsr, 1, gE, Tt, bxlam, gw, Aadj)
                        : launch_adj_g(stream, nb, n, nsr, p, span, nl, 1, gE, Tt, bxlam, gw, Aadj);
  }
  void box_solve_neumann(double *f, double *sol, int which);
  void forward_box(double *Phi, double *U, bool pair_forces);
  void reverse_box(double *F, double *dUdQ);
  void build_near_fft();
  void mesh_solve(double *rhs, double *out, int which, int nsys = 1);
  void adjoint_rhs();
  void store_rel(int which);
  void run_once(const double *x, const double *Qc, double *Phi, double *U, double *F, double *dUdQ);
  void finish_host();
  void evaluate_graph(const double *x, const double *Qc, double *Phi, double *U, double *F, double *dUdQ);
  void evaluate(const double *x, const double *Qc, double *Phi, double *U, double *F = nullptr,
                double *dUdQ = nullptr);
};

// ----------------------------------------------------------------- create

void fep3m_ctx::build(double L_, const std::vector<int64_t> &Ns, int n_, int q_, const fep3m_options &o) {
  auto t0 = std::chrono::steady_clock::now();
  L = L_;
  nb = int(Ns.size());
  off_h.assign(1, 0);
  for (int64_t v : Ns) off_h.push_back(off_h.back() + int(v));
  N = off_h.back();
  n = n_;
  q = q_;
  p = q + 2;
  opt = o;
  nsr = o.n_sr;
  B = o.table_box;
  h = L / n;
  mixed = o.precision == FEP3M_PRECISION_MIXED;

  Screen1D scr = make_screen(q, o.support);
  d = scr.d;
  nl = d + 1;
  na = nl * nl * nl;
  span = scr.span;
  generic = !(o.support == FEP3M_SUPPORT_ONE && q == 3);
  box = o.boundary != FEP3M_BOUNDARY_PERIODIC;
  insulated = o.boundary == FEP3M_BOUNDARY_INSULATED;
  if (box) {   // the box runs on the float64 table-sum kernels, the pair sum on rows of elements
    generic = true;
    plan = PairPlan{2, 2, 0};
    tuned = true;
  }
  compute_tables(p, scr, nsr, B, T_host);
  Mat g = load_weights(p, scr);
  Mat ke, me;
  element_matrices(p, ke, me);
  const int ks = span * p + 1;   // support nodes per axis
  std::vector<double> gwh(size_t(nl) * ks), w1h(p);
  for (int l = 0; l < nl; ++l)
    for (int k = 0; k < ks; ++k) gwh[l * ks + k] = g(l, k);
  for (int k = 0; k < p; ++k) {  // (M1 1) at local index k (k = 0 collects both elements)
    double s = 0.0;
    for (int j = 0; j <= p; ++j) s += me(k, j);
    if (k == 0)
      for (int j = 0; j <= p; ++j) s += me(p, j);
    w1h[k] = s;
  }
  Vec nodes = gll_nodes(p);
  for (int a = 0; a <= p; ++a) {
    double den = 1.0;
    for (int j = 0; j <= p; ++j)
      if (j != a) den *= (nodes[a] - nodes[j]);
    bas.x[a] = nodes[a];
    bas.w[a] = 1.0 / den;
  }

  const int M = n * n * n;
  off_d = alloc<int>(off_h.size(), "configuration offsets");
  hip_check(hipMemcpy(off_d, off_h.data(), off_h.size() * sizeof(int), hipMemcpyHostToDevice), "upload offsets");
  nbs = nb;
  cs = alloc<double>(size_t(kCsSlots) * nb, "configuration scalars");
  host_cs = host_mirror(size_t(kCsSlots) * nb, host_cs_buf, "pinned configuration scalars");
  {
    double **slots[] = {&pcs.bn2, &pcs.rz, &pcs.rzn, &pcs.pq, &pcs.rr, &pcs.zq, &pcs.alpha, &pcs.beta, &pcs.act, &pcs.rel};
    double *pbuf = alloc<double>(size_t(10) * 2 * nb, "pcg scalars");
    for (int k = 0; k < 10; ++k) *slots[k] = pbuf + size_t(k) * 2 * nb;
    gauge = alloc<double>(size_t(2) * nb, "gauge integrals");
  }
  T = alloc<double>(T_host.size(), "tables");
  gw = alloc<double>(gwh.size(), "load weights");
  w1 = alloc<double>(w1h.size(), "mass ones");
  hip_check(hipMemcpy(T, T_host.data(), T_host.size() * sizeof(double), hipMemcpyHostToDevice), "upload tables");
  {  // transposed copy Tt[D][m][a] for the reverse pass
    const size_t ND = size_t(2 * nsr + 1) * (2 * nsr + 1) * (2 * nsr + 1), NM = size_t(p + 1) * (p + 1) * (p + 1);
    const size_t NA = size_t(na);
    std::vector<double> tt(T_host.size());
    for (size_t a = 0; a < NA; ++a)
      for (size_t iD = 0; iD < ND; ++iD)
        for (size_t m = 0; m < NM; ++m) tt[(iD * NM + m) * NA + a] = T_host[(a * ND + iD) * NM + m];
    Tt = alloc<double>(tt.size(), "transposed tables");
    hip_check(hipMemcpy(Tt, tt.data(), tt.size() * sizeof(double), hipMemcpyHostToDevice), "upload tables");
  }
  hip_check(hipMemcpy(gw, gwh.data(), gwh.size() * sizeof(double), hipMemcpyHostToDevice), "upload weights");
  hip_check(hipMemcpy(w1, w1h.data(), w1h.size() * sizeof(double), hipMemcpyHostToDevice), "upload weights");

  gtmp = alloc<double>(3 * size_t(N), "positions");
  sg = alloc<double>(3 * size_t(N), "sorted positions");
  sQ = alloc<double>(size_t(N), "sorted charges");
  elem = alloc<int>(size_t(N), "elements");
  slot = alloc<int>(size_t(N), "slots");
  tmp = alloc<int>(size_t(N), "sort scratch");
  perm = alloc<int>(size_t(N), "permutation");
  count = alloc<int>(size_t(nb) * M, "counts");
  start = alloc<int>(size_t(nb) * M + 1, "element starts");
  flags = alloc<int>(4, "flags");
  scan_scr = alloc<int>(2 * ((size_t(nb) * M + 2047) / 2048) + 16, "scan scratch");
  maxcount = alloc<int>(4, "max count");
  paircount = alloc<unsigned long long>(2, "pair count");
  C = alloc<double>(size_t(nb) * M * na, "moments");
  if (generic && !box && (span == 3 || nl > 1)) lsep = alloc<double>(load_sep_scratch(nb, n, p, nl), "load passes");
  if (!mixed) {
    Wel = alloc<double>(size_t(nb) * M * (p + 1) * (p + 1) * (p + 1), "element field");
  } else {
    std::vector<float> tf(T_host.begin(), T_host.end());
    Tf = alloc<float>(tf.size(), "tables (f32)");
    hip_check(hipMemcpy(Tf, tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice), "upload tables");
    Welf = alloc<float>(size_t(nb) * M * (p + 1) * (p + 1) * (p + 1), "element field (f32)");
    su = alloc<float4>(size_t(N), "local coordinates (f32)");
    si = alloc<int4>(size_t(N), "local coordinates (fixed point)");
    sel = alloc<int>(size_t(N), "packed elements");
  }
  nit = alloc<int>(size_t(nb) * M + 1, "items per element");
  item_start = alloc<int>(size_t(nb) * M + 1, "item starts");
  items = alloc<int2>(size_t(N), "pair work items");
  icounter = alloc<int>(4, "item counter");
  iscan_max = alloc<int>(4, "item scan max");
  if (!mixed) {
    const size_t RT = size_t(nb) * n * n;
    rowstart = alloc<int>(RT + 1, "row starts");
    rnit = alloc<int>(RT, "row items");
    ritem_start = alloc<int>(RT + 1, "row item starts");
    riscan_max = alloc<int>(4, "row item scan max");
    ritems = alloc<int2>(size_t(pair_rows_items_max(nb, n, N)), "row work items");
  }
  {
    int dev = 0;
    hip_check(hipGetDevice(&dev), "device");
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, dev), "device properties");
    cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  }
  phip_s = alloc<double>(size_t(N), "pair potential");
  phim_s = alloc<double>(size_t(N), "mesh potential");
  phi_s = alloc<double>(size_t(N), "potential");
  partial_len = size_t(4 * kRedBlocks) + 64;
  scal = alloc<double>(64, "scalars");
  host_scal = host_mirror(64, host_scal_buf, "pinned scalars");

  build_mg();
  if (box) build_box();
  else if (opt.solver == FEP3M_SOLVER_FDM) build_fdm();
  // partials serve every two-stage reduction: the fixed reduction grids and
  // the per-tile partials of the fine-level operator
  partial_len = std::max(partial_len, size_t(2) * nb * apply_blocks(lv[0].op) + 64);
  // row-wise mesh kernels: nb K <= max(kRowBlocks, nb) partials (nb <= 2048 systems)
  partial_len = std::max(partial_len, size_t(kRowBlocks) + 64);
  partial = alloc<double>(partial_len, "partials");
  estimate_spectra();
  near_fft = !generic && (opt.near_field == FEP3M_NEAR_FFT || (opt.near_field == FEP3M_NEAR_AUTO && fft_size_ok(n)));
  if (near_fft) build_near_fft();
  stats.near_fft = near_fft ? 1 : 0;
  auto t1 = std::chrono::steady_clock::now();
  stats.create_seconds = std::chrono::duration<double>(t1 - t0).count();
  stats.mg_levels = int(lv.size());
  stats.device_bytes = int64_t(dev_bytes);
}

// Operator of a level whose elements are H fine elements wide: in fine
// element units K1 scales as 1/H and M1 as H, so K = K1 M1 M1 + ... scales
// as H (the coarse spaces are nested in the fine one, and the rediscretised
// operator equals the Galerkin product P^T K P only with this scaling).
static LevelOp make_levelop(int p, int n, double H) {
  LevelOp op{};
  op.p = p;
  op.n = n;
  op.P = p * n;
  Mat ke, me;
  element_matrices(p, ke, me);
  for (int a = 0; a <= p; ++a)
    for (int b = 0; b <= p; ++b) {
      ke(a, b) /= H;
      me(a, b) *= H;
    }
  for (int a = 0; a <= p; ++a)
    for (int b = 0; b <= p; ++b) {
      op.ke[a * (p + 1) + b] = ke(a, b);
      op.me[a * (p + 1) + b] = me(a, b);
    }
  for (int k = 0; k < p; ++k) {
    op.dk[k] = ke(k, k) + (k == 0 ? ke(p, p) : 0.0);
    op.dm[k] = me(k, k) + (k == 0 ? me(p, p) : 0.0);
  }
  return op;
}

static Transfer make_transfer(int pf, int nf, int pc, int nc) {
  Transfer t{};
  t.pf = pf; t.nf = nf; t.Pf = pf * nf;
  t.pc = pc; t.nc = nc; t.Pc = pc * nc;
  t.r = nf / nc;
  t.ns = t.r * pf;
  Vec gf = gll_nodes(pf), gc = gll_nodes(pc);
  std::vector<double> l(pc + 1);
  for (int s = 0; s < t.ns; ++s) {
    const int fe = s / pf, k = s % pf;
    const double pos = (fe + 0.5 + gf[k]) / t.r - 0.5;
    lagrange(gc, pos, l.data(), nullptr);
    for (int j = 0; j <= pc; ++j) t.w[s * (pc + 1) + j] = (std::fabs(l[j]) < 1e-15 ? 0.0 : l[j]);
  }
  return t;
}

template <> const Transfer &fep3m_ctx::transfer<double>(int l) const { return tr[l]; }
template <> const TransferF &fep3m_ctx::transfer<float>(int l) const { return trf[l]; }
template <> double *fep3m_ctx::rr_part<double>() const { return rrp_d; }
template <> float *fep3m_ctx::rr_part<float>() const { return rrp_f; }

void fep3m_ctx::build_mg() {
  std::vector<std::pair<int, int>> hier;
  hier.push_back({p, n});
  if (p > 3) hier.push_back({3, n});
  hier.push_back({1, n});
  int nc = n;
  while (nc > 4 && nc % 2 == 0) { nc /= 2; hier.push_back({1, nc}); }
  while (nc > 6 && nc % 3 == 0) { nc /= 3; hier.push_back({1, nc}); }
  if (size_t(nc) * nc * nc > 4096)
    throw Status(FEP3M_ERR_UNSUPPORTED, "mesh size leaves a coarse grid above 16^3 elements (n must coarsen by 2 or 3)");
  for (auto &pr : hier) {
    MGLevel L_;
    L_.op = make_levelop(pr.first, pr.second, double(n) / pr.second);
    L_.ndof = size_t(L_.op.P) * L_.op.P * L_.op.P;
    lv.push_back(L_);
  }
  for (size_t i = 0; i + 1 < hier.size(); ++i)
    tr.push_back(make_transfer(hier[i].first, hier[i].second, hier[i + 1].first, hier[i + 1].second));
  for (size_t i = 0; i < lv.size(); ++i) {
    MGLevel &L_ = lv[i];
    const size_t nv = L_.ndof * 2 * nb;   // one block of the level per system (forward and adjoint)
    L_.vd.x = alloc<double>(nv, "mg x");
    if (i + 1 < lv.size()) L_.d = alloc<double>(L_.ndof, "mg d");
    if (!mixed) {
      L_.vd.f = (i == 0) ? nullptr : alloc<double>(nv, "mg f");
      if (i + 1 < lv.size()) {
        L_.vd.x2 = alloc<double>(nv, "mg x2");
        L_.vd.r = alloc<double>(nv, "mg r");
      }
    } else {
      // float32 hierarchy; the fine level also holds the float32 copy of the residual
      L_.opf = L_.op.cast<float>();
      L_.vf.x = alloc<float>(nv, "mg x (f32)");
      L_.vf.f = alloc<float>(nv, "mg f (f32)");
      if (i + 1 < lv.size()) {
        L_.vf.x2 = alloc<float>(nv, "mg x2 (f32)");
        L_.vf.r = alloc<float>(nv, "mg r (f32)");
      }
    }
    if (L_.op.p == 6) {   // the order-6 operator reads its band coefficients from device memory
      constexpr int Q2 = 49;
      std::vector<double> cd(2 * Q2);
      for (int k = 0; k < Q2; ++k) {
        cd[k] = L_.op.me[k];
        cd[Q2 + k] = L_.op.ke[k];
      }
      double *g = alloc<double>(cd.size(), "order-6 operator coefficients");
      hip_check(hipMemcpy(g, cd.data(), cd.size() * sizeof(double), hipMemcpyHostToDevice), "upload coefficients");
      L_.op.cg = g;
      if (mixed) {
        std::vector<float> cf(cd.size());
        for (size_t k = 0; k < cf.size(); ++k) cf[k] = k < Q2 ? L_.opf.me[k] : L_.opf.ke[k - Q2];
        float *gf = alloc<float>(cf.size(), "order-6 operator coefficients (f32)");
        hip_check(hipMemcpy(gf, cf.data(), cf.size() * sizeof(float), hipMemcpyHostToDevice), "upload coefficients");
        L_.opf.cg = gf;
      }
    }
  }
  fuse_rr = lv.size() > 1 && lv[0].op.p == 5 && lv[1].op.p == 3 && n % 2 == 0;
  if (fuse_rr) {
    const size_t np = size_t(2) * nb * (n / 2) * (n / 2) * (n / 2) * 343;   // per system and tile
    if (mixed) rrp_f = alloc<float>(np, "restriction partials (f32)");
    else rrp_d = alloc<double>(np, "restriction partials");
  }
  if (mixed) {
    for (const Transfer &t : tr) trf.push_back(t.cast<float>());
    dot_scr = alloc<double>(2 * kRedBlocks, "two-dot partials");
  }
  const size_t nd0 = lv[0].ndof * nb;
  gE = alloc<double>(size_t(nb) * n * n * n * (p + 1) * (p + 1) * (p + 1), "deposit");
  b = alloc<double>(2 * nd0, "load, adjoint load");
  Gv = b + nd0;
  sol = alloc<double>(2 * nd0, "phi, lambda");
  lam = sol + nd0;
  Aadj = alloc<double>(size_t(nb) * n * n * n * na, "moment adjoint");
  fpair = alloc<double>(3 * size_t(N), "pair forces");
  Phi_int = alloc<double>(size_t(N), "potential (caller order)");
  rr = alloc<double>(2 * nd0, "pcg r");
  pv = alloc<double>(2 * nd0, "pcg p");
  qv = alloc<double>(2 * nd0, "pcg q");
  // coarse level: 1-D periodic pencil K1 V = M1 V Lambda
  {
    const LevelOp &op = lv.back().op;
    Mat K1, M1;
    assemble_1d(op.p, op.n, true, K1, M1);
    const double H = double(n) / op.n;
    for (double &v : K1.a) v /= H;
    for (double &v : M1.a) v *= H;
    Vec lam;
    Mat V;
    sym_gen_eig(K1, M1, lam, V);
    lam[0] = 0.0;
    coarseP = op.P;
    coarseV = alloc<double>(V.a.size(), "coarse V");
    coarseLam = alloc<double>(lam.size(), "coarse lambda");
    hip_check(hipMemcpy(coarseV, V.a.data(), V.a.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
    hip_check(hipMemcpy(coarseLam, lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
  }
}

// Spectrum of the tables at the octant frequencies (create time, on the
// device) and the FFT work arrays.
void fep3m_ctx::build_near_fft() {
  const size_t M = size_t(n) * n * n, NM = size_t(p + 1) * (p + 1) * (p + 1);
  std::vector<double2> tw(n);
  for (int j = 0; j < n; ++j) {
    const double t = 2.0 * M_PI * double(j) / double(n);
    tw[j] = make_double2(std::cos(t), -std::sin(t));
  }
  twd = alloc<double2>(size_t(n), "FFT twiddles");
  hip_check(hipMemcpy(twd, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice), "upload twiddles");
  spec = alloc<double2>(spec_freqs(n) * 8 * NM, "table spectrum");
  zc = alloc<double2>(size_t(nb) * M * 4, "transformed moments");
  za = alloc<double2>(size_t(nb) * M * 4, "transformed moment adjoint");
  zpsi = alloc<double2>(size_t(nb) * M * NM / 2, "transformed near-screen field");
  zg = alloc<double2>(size_t(nb) * M * NM / 2, "transformed deposits");
  launch_spec_build(stream, n, nsr, p, T, twd, spec);
  check_launch("table spectrum");
  hip_check(hipStreamSynchronize(stream), "table spectrum");
}

void fep3m_ctx::build_fdm() {
  if (fft_size_ok(n)) {
    Vec wr, wi, lamf;
    periodic_fourier_eigen(p, n, wr, wi, lamf);
    std::vector<double2> w(wr.size()), tw(n);
    for (size_t i = 0; i < wr.size(); ++i) w[i] = make_double2(wr[i], wi[i]);
    for (int j = 0; j < n; ++j) {
      const double t = 2.0 * M_PI * double(j) / double(n);
      tw[j] = make_double2(std::cos(t), -std::sin(t));
    }
    fsW = alloc<double2>(w.size(), "Fourier block eigenvectors");
    fsL = alloc<double>(lamf.size(), "Fourier block eigenvalues");
    fsTw = alloc<double2>(tw.size(), "FFT twiddles");
    // two real systems per complex one: the forward and adjoint systems of
    // every configuration
    fsZ = alloc<double2>(size_t(nb) * n * n * n * (p * p * p), "Fourier solve work array");
    hip_check(hipMemcpy(fsW, w.data(), w.size() * sizeof(double2), hipMemcpyHostToDevice), "upload");
    hip_check(hipMemcpy(fsL, lamf.data(), lamf.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
    hip_check(hipMemcpy(fsTw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice), "upload");
    fs_ready = true;
    return;
  }
  const LevelOp &op = lv[0].op;
  Mat K1, M1;
  assemble_1d(op.p, op.n, true, K1, M1);
  Vec lamv;
  Mat V;
  sym_gen_eig(K1, M1, lamv, V);
  const int P = op.P;
  fdm_i0 = 0;
  for (int i = 1; i < P; ++i)
    if (std::fabs(lamv[i]) < std::fabs(lamv[fdm_i0])) fdm_i0 = i;
  lamv[fdm_i0] = 0.0;   // the constant mode of the periodic pencil
  std::vector<double> vcm(size_t(P) * P);
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < P; ++j) vcm[i + size_t(j) * P] = V(i, j);
  fdmV = alloc<double>(vcm.size(), "fdm eigenvectors");
  fdmLam = alloc<double>(size_t(P), "fdm eigenvalues");
  hip_check(hipMemcpy(fdmV, vcm.data(), vcm.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
  hip_check(hipMemcpy(fdmLam, lamv.data(), size_t(P) * sizeof(double), hipMemcpyHostToDevice), "upload");
}


// Exact periodic solve by fast diagonalisation of the Kronecker sum
// K = K1 (x) M1 (x) M1 + M1 (x) K1 (x) M1 + M1 (x) M1 (x) K1 with
// K1 V = M1 V diag(lam), V^T M1 V = I:  out = (V (x) V (x) V) D^+ (V (x) V (x) V)^T rhs,
// D = lam_i + lam_j + lam_k.  On meshes whose edge is a power of two the
// same solve runs by Fourier analysis over the element lattice (k_fdm.hip:
// FFTs and p x p blocks per frequency); otherwise the 1-D transforms are
// dense tiled kernels over the whole batch.  The achieved relative residual
// is measured with one operator apply, as for the iterative solver.
void fep3m_ctx::fdm_solve(const double *rhs, double *sol, int which) {
  const int P = lv[0].op.P;
  const size_t per = lv[0].ndof, nd = per * nbs;
  if (fs_ready) {
    if (launch_fs_solve(stream, nbs, n, p, rhs, sol, fsZ, fsTw, fsW, fsL) != 0)
      throw Status(FEP3M_ERR_UNSUPPORTED, "Fourier solve variant");
  } else {
    // dense transforms of the pencil's eigenvectors along x, y, z (the PCG
    // buffers serve as the two work vectors), the eigenvalue division, back
    double *A = rr, *B = pv;
    launch_axis_transform(stream, P, 0, nbs, fdmV, true, rhs, A);
    launch_axis_transform(stream, P, 1, nbs, fdmV, true, A, B);
    launch_axis_transform(stream, P, 2, nbs, fdmV, true, B, A);
    launch_fdm_scale(stream, nd, P, fdm_i0, fdmLam, A);
    launch_axis_transform(stream, P, 2, nbs, fdmV, false, A, B);
    launch_axis_transform(stream, P, 1, nbs, fdmV, false, B, A);
    launch_axis_transform(stream, P, 0, nbs, fdmV, false, A, sol);
  }
  // achieved residual, per configuration
  launch_sum_partials(stream, launch_dot(stream, nbs, per, rhs, rhs, partial), partial, pcs.bn2, nbs);
  apply0<double>(sol, rhs, qv, nullptr, nullptr, 0.0, 0.0, kResidual, nullptr);
  launch_sum_partials(stream, launch_dot(stream, nbs, per, qv, qv, partial), partial, pcs.rr, nbs);
  launch_pcg_scalars(stream, nbs, kPcgStart, 0.0, pcs);
  launch_pcg_scalars(stream, nbs, kPcgResid, 0.0, pcs);
  store_rel(which);
  check_launch("fdm solve");
  if (capturing) return;
  hip_check(hipMemcpyAsync(host_cs, pcs.rel, nbs * sizeof(double), hipMemcpyDeviceToHost, stream), "copy residuals");
  sync("fdm residual");
  double relmax = 0.0;
  for (int bb = 0; bb < nbs; ++bb) relmax = std::max(relmax, host_cs[bb]);
  stats.mg_iterations = 0;
  stats.mg_rel_residual = relmax;
  if (!(relmax <= 1e-9))
    throw Status(FEP3M_ERR_NOT_CONVERGED, "fast-diagonalisation solve reached relative residual " +
                                              std::to_string(relmax));
}

void fep3m_ctx::estimate_spectra() {
  // largest eigenvalue of D^-1 K per smoothed level (power iteration)
  for (size_t i = 0; i + 1 < lv.size(); ++i) {
    MGLevel &L_ = lv[i];
    double *xw = L_.vd.x;
    launch_hash_fill(stream, L_.ndof, 12345u + uint32_t(i), xw);
    double lam = 0.0;
    // every configuration has the same operator: iterate on configuration 0
    double nx = std::sqrt(reduce_host(launch_dot(stream, 1, L_.ndof, xw, xw, partial), partial, 0));
    for (int it = 0; it < 24; ++it) {
      launch_apply<double>(stream, 1, L_.op, xw, nullptr, L_.d, nullptr, nullptr, 0.0, 0.0, kDinvApply, nullptr);
      double nd = std::sqrt(reduce_host(launch_dot(stream, 1, L_.ndof, L_.d, L_.d, partial), partial, 0));
      lam = nd / nx;
      launch_scale(stream, L_.ndof, 1.0 / nd, L_.d, xw);
      nx = 1.0;
    }
    check_launch("power iteration");
    L_.lmax = lam;
  }
}

// ----------------------------------------------------------------- multigrid

// Chebyshev(deg)-Jacobi smoothing on level l in arithmetic type T, targeting
// the interval [lmax / 12, 1.1 lmax] of D^-1 K.
// With dot_part, the last step also writes block partials of x_new . f
// (returns their count per system).
template <class T>
int fep3m_ctx::cheb_smooth(int l, const T *f, bool zero_start, double *dot_part) {
  int Kd = 0;
  MGLevel &L_ = lv[l];
  LevelVecs<T> &V = L_.vec<T>();
  const LevelOpT<T> &op = L_.oper<T>();
  const double bmax = 1.1 * L_.lmax, amin = bmax / 12.0;
  const double theta = 0.5 * (bmax + amin), delta = 0.5 * (bmax - amin), sigma = theta / delta;
  double rho = 1.0 / sigma;
  const int deg = opt.cheb_degree;
  double s0 = 0.0;   // first-step coefficient: x1 = s0 D^-1 f after a zero start
  for (int s = 0; s < deg; ++s) {
    double c1, c2;
    if (s == 0) {
      c1 = 0.0;
      c2 = 1.0 / theta;
    } else {
      const double rn = 1.0 / (2.0 * sigma - rho);
      c1 = rn * rho;
      c2 = 2.0 * rn / delta;
      rho = rn;
    }
    if (s == 0 && zero_start) {
      s0 = c2;
      // with later steps, the operator rebuilds x1 from f where it needs it
      if (deg == 1) launch_cheb_first<T>(stream, nbs, op, f, V.x, T(c2));   // x = c2 D^-1 f
    } else {
      // x2 holds x_prev on entry and receives x_new; then the two swap.
      // Steps 2 and 3 after a zero start take x1 (step 2: x; step 3: x_prev)
      // as s0 D^-1 f instead of reading it.
      int mode = !zero_start ? kCheb : s == 1 ? kChebZ2 : s == 2 ? kChebZ3 : kCheb;
      const bool dot = dot_part && s == deg - 1 && mode == kCheb;
      if (dot) mode = kChebDot;
      const T *xin = mode == kChebZ2 ? nullptr : V.x;
      const T *xprev = (mode == kCheb || mode == kChebDot) ? V.x2 : nullptr;
      double *part = dot ? dot_part : nullptr;
      const int K = l == 0 ? apply0<T>(xin, f, nullptr, xprev, V.x2, T(c1), T(c2), mode, part, T(s0))
                           : launch_apply<T>(stream, nbs, op, xin, f, nullptr, xprev, V.x2, T(c1), T(c2), mode, part,
                                             T(s0));
      if (dot) Kd = K;
      std::swap(V.x, V.x2);
    }
  }
  return Kd;
}

// One V-cycle for K x = f on level l (x from zero), in arithmetic type T;
// with dot_part, block partials of x . f from the last smoothing step
// (returns their count per system).
template <class T>
int fep3m_ctx::vcycle(int l, const T *f, double *dot_part) {
  MGLevel &L_ = lv[l];
  LevelVecs<T> &V = L_.vec<T>();
  if (l + 1 == int(lv.size())) {
    launch_coarse_solve<T>(stream, nbs, coarseP, coarseV, coarseLam, f, V.x);
    return 0;
  }
  const LevelOpT<T> &op = L_.oper<T>();
  LevelVecs<T> &Vc = lv[l + 1].vec<T>();
  cheb_smooth<T>(l, f, true);
  if (l == 0 && fuse_rr) {   // residual restricted in the operator's epilogue, never stored
    apply0<T>(V.x, f, nullptr, nullptr, nullptr, T(0), T(0), kResidualRestrict, nullptr);
    launch_restrict_sum<T>(stream, nbs, n, rr_part<T>(), Vc.f);
  } else {
    if (l == 0) apply0<T>(V.x, f, V.r, nullptr, nullptr, T(0), T(0), kResidual, nullptr);
    else launch_apply<T>(stream, nbs, op, V.x, f, V.r, nullptr, nullptr, T(0), T(0), kResidual, nullptr);
    launch_transfer<T>(stream, nbs, transfer<T>(l), V.r, Vc.f, true);
  }
  vcycle<T>(l + 1, Vc.f);
  launch_transfer<T>(stream, nbs, transfer<T>(l), Vc.x, V.x, false);
  return cheb_smooth<T>(l, f, false, dot_part);
}

// Boxes: the 1-D stiffness and mass on the p n + 1 nodes of an axis
// (non-periodic assembly) as class-row band tables for the operator, the
// generalised eigenbasis of the interior pencil (and, insulating box, of the
// whole pencil), the GLL nodes, the face quadrature and the box vectors.
void fep3m_ctx::build_box() {
  Pb = p * n + 1;
  const int Pi = Pb - 2;
  const size_t nv = size_t(Pb) * Pb * Pb * nb;
  bxb = alloc<double>(nv, "box load");
  bxphi = alloc<double>(nv, "box potential");
  bxy = alloc<double>(nv, "box operator output");
  bxt1 = alloc<double>(nv, "box work");
  bxt2 = alloc<double>(nv, "box work");
  bxt3 = alloc<double>(nv, "box work");
  bxt4 = alloc<double>(nv, "box work");
  bxg = alloc<double>(nv, "box assembled deposit");
  bxlam = alloc<double>(nv, "box adjoint potential");
  Mat K1, M1;
  assemble_1d(p, n, false, K1, M1);
  // class rows of the bands of half-width p: row o holds A(o, o - p .. o + p)
  // and equals the row of its class (o mod p inside, p for o = 0, p + 1 for
  // o = P - 1); every entry outside the band must be zero (elements couple
  // nodes at most p apart) and every row must equal its class row
  const int W = 2 * p + 1;
  std::vector<double> kb(size_t(p + 2) * W, 0.0), mb(size_t(p + 2) * W, 0.0);
  auto cls = [&](int o) { return o == 0 ? p : (o == Pb - 1 ? p + 1 : o % p); };
  std::vector<char> seen(p + 2, 0);
  for (int i = 0; i < Pb; ++i) {
    const int c = cls(i);
    for (int j = 0; j < Pb; ++j) {
      const int d = j - i + p;
      if (d < 0 || d >= W) {
        if (K1(i, j) != 0.0 || M1(i, j) != 0.0) throw Status(FEP3M_ERR_UNSUPPORTED, "box matrices wider than their band");
        continue;
      }
      double &kc = kb[size_t(c) * W + d], &mc = mb[size_t(c) * W + d];
      if (!seen[c]) {
        kc = K1(i, j);
        mc = M1(i, j);
      } else if (std::fabs(kc - K1(i, j)) > 1e-12 * std::fabs(K1(i, i)) ||
                 std::fabs(mc - M1(i, j)) > 1e-12 * std::fabs(M1(i, i))) {
        throw Status(FEP3M_ERR_UNSUPPORTED, "box matrix rows differ within a class");
      }
    }
    seen[c] = 1;
  }
  bxKb = alloc<double>(kb.size(), "box stiffness class rows");
  bxMb = alloc<double>(mb.size(), "box mass class rows");
  hip_check(hipMemcpy(bxKb, kb.data(), kb.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
  hip_check(hipMemcpy(bxMb, mb.data(), mb.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
  Mat Ki(Pi, Pi), Mi(Pi, Pi);
  for (int i = 0; i < Pi; ++i)
    for (int j = 0; j < Pi; ++j) {
      Ki(i, j) = K1(i + 1, j + 1);
      Mi(i, j) = M1(i + 1, j + 1);
    }
  Vec lamv;
  Mat V;
  sym_gen_eig(Ki, Mi, lamv, V);
  std::vector<double> vc(size_t(Pi) * Pi);
  for (int i = 0; i < Pi; ++i)
    for (int j = 0; j < Pi; ++j) vc[i + size_t(j) * Pi] = V(i, j);
  bxV = alloc<double>(vc.size(), "box interior eigenvectors");
  bxLam = alloc<double>(size_t(Pi), "box interior eigenvalues");
  hip_check(hipMemcpy(bxV, vc.data(), vc.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
  hip_check(hipMemcpy(bxLam, lamv.data(), size_t(Pi) * sizeof(double), hipMemcpyHostToDevice), "upload");
  const Vec nodes = gll_nodes(p);
  for (int a = 0; a <= p; ++a) bxnodes.x[a] = nodes[a];
  if (!insulated) return;
  // the whole pencil K1 V = M1 V Lambda (one zero eigenvalue: the constants)
  Vec lf;
  Mat Vf;
  sym_gen_eig(K1, M1, lf, Vf);
  bx_i0 = 0;
  for (int i = 1; i < Pb; ++i)
    if (std::fabs(lf[i]) < std::fabs(lf[bx_i0])) bx_i0 = i;
  lf[bx_i0] = 0.0;
  std::vector<double> vf(size_t(Pb) * Pb), w1(Pb);
  for (int i = 0; i < Pb; ++i) {
    double r = 0.0;
    for (int j = 0; j < Pb; ++j) {
      vf[i + size_t(j) * Pb] = Vf(i, j);
      r += M1(i, j);
    }
    w1[i] = r;
  }
  bxVf = alloc<double>(vf.size(), "box pencil eigenvectors");
  bxLamf = alloc<double>(size_t(Pb), "box pencil eigenvalues");
  bxw1 = alloc<double>(size_t(Pb), "box mass row sums");
  bxtF = alloc<double>(size_t(nb) * 6 * n * n * (p + 1) * (p + 1), "box face loads");
  bxLw = alloc<double>(size_t(nb) * 6 * n * n * kBoxNQ * kBoxNQ, "box face adjoint weights");
  bxhF = alloc<double>(size_t(nb) * 6 * n * n * (p + 1) * (p + 1) * (p + 1), "box face adjoint moments");
  hip_check(hipMemcpy(bxVf, vf.data(), vf.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
  hip_check(hipMemcpy(bxLamf, lf.data(), size_t(Pb) * sizeof(double), hipMemcpyHostToDevice), "upload");
  hip_check(hipMemcpy(bxw1, w1.data(), size_t(Pb) * sizeof(double), hipMemcpyHostToDevice), "upload");
  Vec xq, wq;
  gauss_legendre(kBoxNQ, xq, wq);
  std::vector<double> l(p + 1), dl(p + 1);
  for (int qi = 0; qi < kBoxNQ; ++qi) {
    bxquad.xq[qi] = xq[qi];
    bxquad.wq[qi] = wq[qi];
    lagrange(nodes, xq[qi], l.data(), nullptr);
    for (int k = 0; k <= p; ++k) bxquad.lq[qi][k] = l[k];
  }
  for (int sd = 0; sd < 2; ++sd) {
    lagrange(nodes, sd ? 0.5 : -0.5, l.data(), dl.data());
    for (int k = 0; k <= p; ++k) bxquad.dend[sd][k] = dl[k];
  }
}

// Pure-Neumann solve of the insulating box on every node: f projected on
// the compatible subspace (f -= (1^T f / V) M 1), then K^+ f by fast
// diagonalisation of the whole box pencil with the constant mode dropped
// (gauge int phi = 0).  The residual against f is checked as for the other
// exact solves.
void fep3m_ctx::box_solve_neumann(double *f, double *sol, int which) {
  int K = launch_box_resid(stream, Pb, nb, false, true, f, nullptr, partial);
  launch_sum_partials(stream, K, partial + size_t(nb) * K, pcs.zq, nb);   // 1^T f per configuration
  launch_box_sub_mass(stream, Pb, nb, 1.0 / (double(n) * n * n), bxw1, pcs.zq, f);
  launch_axis_transform(stream, Pb, 0, nb, bxVf, true, f, bxt1);
  launch_axis_transform(stream, Pb, 1, nb, bxVf, true, bxt1, bxt2);
  launch_axis_transform(stream, Pb, 2, nb, bxVf, true, bxt2, bxt1);
  launch_fdm_scale(stream, size_t(Pb) * Pb * Pb * nb, Pb, bx_i0, bxLamf, bxt1);
  launch_axis_transform(stream, Pb, 2, nb, bxVf, false, bxt1, bxt2);
  launch_axis_transform(stream, Pb, 1, nb, bxVf, false, bxt2, bxt1);
  launch_axis_transform(stream, Pb, 0, nb, bxVf, false, bxt1, sol);
  K = launch_box_resid(stream, Pb, nb, false, false, f, nullptr, partial);
  launch_sum_partials(stream, K, partial, pcs.bn2, nb);
  box_apply(sol, bxy);
  K = launch_box_resid(stream, Pb, nb, false, false, f, bxy, partial);
  launch_sum_partials(stream, K, partial, pcs.rr, nb);
  launch_pcg_scalars(stream, nb, kPcgStart, 0.0, pcs);
  launch_pcg_scalars(stream, nb, kPcgResid, 0.0, pcs);
  store_rel(which);
  check_launch("box solve");
  hip_check(hipMemcpyAsync(host_cs, pcs.rel, nb * sizeof(double), hipMemcpyDeviceToHost, stream), "copy residuals");
  sync("box residual");
  double relmax = 0.0;
  for (int bb = 0; bb < nb; ++bb) relmax = std::max(relmax, host_cs[bb]);
  if (which == 0) {
    stats.mg_iterations = 0;
    stats.mg_rel_residual = relmax;
  } else {
    stats.adj_iterations = 0;
  }
  if (!(relmax <= 1e-9))
    throw Status(FEP3M_ERR_NOT_CONVERGED, "box solve left relative residual " + std::to_string(relmax));
}

// y = K v on the box (all nodes; the rows of the interior nodes are those of
// the Dirichlet problem): K = Kx My Mz + Mx Ky Mz + Mx My Kz by banded 1-D
// passes, y = Kx (My Mz v) + Mx (Ky Mz v + My Kz v).  Uses bxt1, bxt2, bxt3
// and bxt4.
void fep3m_ctx::box_apply(const double *v, double *y) {
  if (launch_box_apply(stream, Pb, nb, p, bxKb, bxMb, v, bxt1, bxt2, bxt3, bxt4, y) != 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "box operator variant");
}

// Interior solve of the box: sol holds phi_B on the boundary and zero
// inside; K_II phi_I = rhs_I - K_IB phi_B by fast diagonalisation of the
// interior pencil, phi_I written into sol.  The relative residual of the
// interior equations (against the norm of their right side) is measured
// with one more operator apply; above 1e-9 the call fails.  which: 0 the
// forward solve, 1 the adjoint one (their statistics slots).
// zero_boundary: sol is zero on the boundary too (K_IB phi_B = 0, no apply).
void fep3m_ctx::box_solve(const double *rhs, double *sol, int which, bool zero_boundary) {
  const int Pi = Pb - 2;
  const size_t nv = size_t(Pb) * Pb * Pb * nb, ni = size_t(Pi) * Pi * Pi * nb;
  int K;
  if (zero_boundary) {
    K = launch_box_resid(stream, Pb, nb, true, false, rhs, nullptr, partial);
    launch_sum_partials(stream, K, partial, pcs.bn2, nb);   // |rhs_I|^2
    launch_box_interior(stream, Pb, nb, true, rhs, bxt1);
  } else {
    box_apply(sol, bxy);                                      // K phi_B
    K = launch_box_resid(stream, Pb, nb, true, false, rhs, bxy, partial);
    launch_sum_partials(stream, K, partial, pcs.bn2, nb);     // |rhs_I - K_IB phi_B|^2
    launch_box_axpby(stream, nv, 1.0, rhs, -1.0, bxy);        // r = rhs - K phi_B
    launch_box_interior(stream, Pb, nb, true, bxy, bxt1);
  }
  launch_axis_transform(stream, Pi, 0, nb, bxV, true, bxt1, bxt2);
  launch_axis_transform(stream, Pi, 1, nb, bxV, true, bxt2, bxt1);
  launch_axis_transform(stream, Pi, 2, nb, bxV, true, bxt1, bxt2);
  launch_fdm_scale(stream, ni, Pi, -1, bxLam, bxt2);        // no null mode
  launch_axis_transform(stream, Pi, 2, nb, bxV, false, bxt2, bxt1);
  launch_axis_transform(stream, Pi, 1, nb, bxV, false, bxt1, bxt2);
  launch_axis_transform(stream, Pi, 0, nb, bxV, false, bxt2, bxt3);
  launch_box_interior(stream, Pb, nb, false, bxt3, sol);
  box_apply(sol, bxy);
  K = launch_box_resid(stream, Pb, nb, true, false, rhs, bxy, partial);
  launch_sum_partials(stream, K, partial, pcs.rr, nb);
  launch_pcg_scalars(stream, nb, kPcgStart, 0.0, pcs);
  launch_pcg_scalars(stream, nb, kPcgResid, 0.0, pcs);
  store_rel(which);
  check_launch("box solve");
  hip_check(hipMemcpyAsync(host_cs, pcs.rel, nb * sizeof(double), hipMemcpyDeviceToHost, stream), "copy residuals");
  sync("box residual");
  double relmax = 0.0;
  for (int bb = 0; bb < nb; ++bb) relmax = std::max(relmax, host_cs[bb]);
  if (which == 0) {
    stats.mg_iterations = 0;
    stats.mg_rel_residual = relmax;
  } else {
    stats.adj_iterations = 0;
  }
  if (!(relmax <= 1e-9))
    throw Status(FEP3M_ERR_NOT_CONVERGED, "box solve left relative residual " + std::to_string(relmax));
}

// Forward pass in the grounded box (after binning and sorting): moments,
// load, the near field without phi (W = -Psi), the near pairs, the
// boundary values -Phi_sr (eq. bcadjust with g = 0), the interior solve,
// W = phi_E - Psi, interpolation and energy.
void fep3m_ctx::forward_box(double *Phi, double *U, bool pair_forces) {
  stage_mark(FEP3M_PROF_ASSIGN, true);
  stage_mark(FEP3M_PROF_MOMENTS, true);
  if (launch_moments_g(stream, nb, n, nl, N, start, sg, sQ, C) != 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "moments variant");
  stage_mark(FEP3M_PROF_MOMENTS, false);
  stage_mark(FEP3M_PROF_LOAD, true);
  if (launch_load_g(stream, nb, n, p, span, nl, 1, C, gw, bxb, partial) < 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "load variant");
  stage_mark(FEP3M_PROF_LOAD, false);
  stage_mark(FEP3M_PROF_ASSIGN, false);
  stage_mark(FEP3M_PROF_NEAR, true);
  // on the matrix cores where the screen family has a kernel there, else by the generic table sums
  if (launch_psi_mfma_g(stream, nb, n, nsr, p, nl, 1, C, T, nullptr, Wel) != 0 &&
      launch_psi_g(stream, nb, n, nsr, p, nl, 1, C, T, nullptr, Wel) != 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "near field variant");
  stage_mark(FEP3M_PROF_NEAR, false);
  pair_pass(pair_forces);
  stage_mark(FEP3M_PROF_SOLVE, true);
  if (insulated) {   // surface load of -dPhi_sr/dn, then the pure-Neumann solve
    if (launch_box_flux(stream, nb, n, nsr, p, N, bxquad, start, sg, sQ, Wel, bxtF, bxb) != 0)
      throw Status(FEP3M_ERR_UNSUPPORTED, "surface load variant");
    box_solve_neumann(bxb, bxphi, 0);
  } else {           // boundary values -Phi_sr, then the interior solve
    launch_box_fill(stream, size_t(Pb) * Pb * Pb * nb, 0.0, bxphi);
    if (launch_box_bvals(stream, nb, n, nsr, p, N, bxnodes, start, sg, sQ, Wel, bxphi) != 0)
      throw Status(FEP3M_ERR_UNSUPPORTED, "boundary values variant");
    box_solve(bxb, bxphi, 0);
  }
  stage_mark(FEP3M_PROF_SOLVE, false);
  if (launch_box_addphi(stream, nb, n, p, bxphi, Wel) != 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "element field variant");
  stage_mark(FEP3M_PROF_INTERP, true);
  stage_mark(FEP3M_PROF_INTERP_KERNEL, true);
  if (launch_interp(stream, nb, off_d, p, n, N, 1.0 / h, bas, sg, Wel, phip_s, perm, phim_s, phi_s, Phi) != 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "interpolation variant");
  stage_mark(FEP3M_PROF_INTERP_KERNEL, false);
  if (U) {
    const int Ke = launch_energy(stream, nb, off_d, N, sQ, phi_s, partial);
    launch_sum_partials(stream, Ke, partial, cfgs(kCsEnergy), nb);
    launch_half(stream, nb, cfgs(kCsEnergy), U);
  }
  stage_mark(FEP3M_PROF_INTERP, false);
}

// Reverse pass in the grounded box.  With G the assembled deposit,
// lambda = K_II^-1 G_I (zero on the boundary) and mu = G - K lambda on the
// boundary nodes, the gradients of U are the periodic ones (moment adjoint
// from lambda and the near deposits, cut at the faces) plus the terms of
// the boundary values: A[E][a] += sum_B mu_B T_a[e(B) - E][m_B] (carried by
// the near part of the adjoint with -mu_B in the deposit's slot of B) and,
// per charge, the derivative of -Q_j / |x_B - x_j| weighted by mu_B.
void fep3m_ctx::reverse_box(double *F, double *dUdQ) {
  stage_mark(FEP3M_PROF_ADJ_SOLVE, true);
  stage_mark(FEP3M_PROF_DEPOSIT, true);
  if (launch_deposit(stream, nb, p, n, N, bas, start, sg, sQ, gE) != 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "deposit variant");
  if (launch_box_assemble(stream, nb, n, p, gE, bxg) != 0) throw Status(FEP3M_ERR_UNSUPPORTED, "assembly variant");
  stage_mark(FEP3M_PROF_DEPOSIT, false);
  if (insulated) {
    // lambda = K^+ G (mean zero, so the projection drops out of the adjoint);
    // the surface load's table term rides in the near part of the moment
    // adjoint (-hF in the boundary elements' deposit), its pair term per charge
    box_solve_neumann(bxg, bxlam, 1);
    stage_mark(FEP3M_PROF_ADJ_SOLVE, false);
    stage_mark(FEP3M_PROF_ADJ_NEAR, true);
    if (launch_box_flux_adj(stream, nb, n, p, bxquad, bxlam, bxLw, bxhF) != 0 ||
        launch_box_h_slots(stream, nb, n, p, bxhF, gE) != 0 ||
        box_adjoint_moments() != 0)
      throw Status(FEP3M_ERR_UNSUPPORTED, "adjoint variant");
    stage_mark(FEP3M_PROF_ADJ_NEAR, false);
    stage_mark(FEP3M_PROF_FORCES, true);
    if (launch_forces<double>(stream, nb, off_d, p, n, nl, N, 1.0 / h, bas, sg, sQ, Wel, Aadj, fpair, phip_s, phim_s,
                              perm, F, dUdQ) != 0 ||
        launch_box_flux_charge(stream, nb, n, nsr, p, N, off_d, 1.0 / h, bxquad, sg, sQ, bxLw, perm, F, dUdQ) != 0)
      throw Status(FEP3M_ERR_UNSUPPORTED, "forces variant");
    stage_mark(FEP3M_PROF_FORCES, false);
    return;
  }
  const size_t nv = size_t(Pb) * Pb * Pb * nb;
  launch_box_fill(stream, nv, 0.0, bxlam);
  box_solve(bxg, bxlam, 1, true);
  box_apply(bxlam, bxy);
  launch_box_axpby(stream, nv, 1.0, bxg, -1.0, bxy);   // mu = G - K lambda (read on the boundary nodes)
  stage_mark(FEP3M_PROF_ADJ_SOLVE, false);
  stage_mark(FEP3M_PROF_ADJ_NEAR, true);
  // the boundary term of the moment adjoint as -mu in the deposit's
  // canonical slots (the deposit is rebuilt by every reverse pass)
  if (launch_box_mu_slots(stream, nb, n, p, bxy, gE) != 0 ||
      box_adjoint_moments() != 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "adjoint variant");
  stage_mark(FEP3M_PROF_ADJ_NEAR, false);
  stage_mark(FEP3M_PROF_FORCES, true);
  if (launch_forces<double>(stream, nb, off_d, p, n, nl, N, 1.0 / h, bas, sg, sQ, Wel, Aadj, fpair, phip_s, phim_s,
                            perm, F, dUdQ) != 0 ||
      launch_box_charge_bnd(stream, nb, n, nsr, p, N, off_d, 1.0 / h, bxnodes, sg, sQ, bxy, perm, F, dUdQ) != 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "forces variant");
  stage_mark(FEP3M_PROF_FORCES, false);
}

// PCG on K out = rhs (rhs compatible), preconditioned by one V-cycle, for
// every configuration of the batch at once: the scalars of each
// configuration live on the device (one thread per configuration updates
// them) and a configuration that has converged keeps alpha = beta = 0, so
// its iterate no longer changes while the others finish.  The host reads
// the nb relative residuals once per iteration.  In mixed precision the
// V-cycle runs in float32 on a float32 copy of the residual, and the
// iteration uses the flexible (Polak-Ribiere) update beta = -alpha
// (z_new . q) / (z_old . r_old), which stays a descent method when the
// preconditioner carries float32 rounding; everything else (K p, the
// updates, every norm and inner product) is float64.
void fep3m_ctx::solve(const double *rhs, double *sol, int which) {
  if (opt.solver == FEP3M_SOLVER_FDM) {
    fdm_solve(rhs, sol, which);
    return;
  }
  MGLevel &L0 = lv[0];
  const size_t per = L0.ndof, nd = per * nbs;
  launch_sum_partials(stream, launch_dot(stream, nbs, per, rhs, rhs, partial), partial, pcs.bn2, nbs);
  // The residual starts as the right side itself (read in place, not
  // copied) and lives in rr from the first update on.  x = 0 is implicit:
  // each iteration's x += alpha p is deferred to the pass that forms the
  // next direction (p is read there anyway), the last one runs after the
  // loop.
  const double *rcur = rhs;
  bool xinit = false;
  // z = M^-1 r; rzn = z . r (and zq = z . q when q is given)
  auto precondition = [&](const double *q) {
    if (!mixed) {   // z . r from the V-cycle's last smoothing step
      launch_sum_partials(stream, vcycle<double>(0, rcur, partial), partial, pcs.rzn, nbs);
    } else {
      if (!q) launch_to_f32(stream, nd, rcur, L0.vf.f);   // later residuals come with their float copy
      vcycle<float>(0, L0.vf.f);
      const int K = launch_dot2_f32(stream, nbs, per, L0.vf.x, rcur, q, dot_scr);
      launch_sum_partials(stream, K, dot_scr, pcs.rzn, nbs);
      launch_sum_partials(stream, K, dot_scr + size_t(nbs) * K, pcs.zq, nbs);
    }
  };
  auto set_p = [&] {   // x += alpha p (deferred); p = z + beta p
    if (!mixed) launch_xp_update<double>(stream, nbs, per, pcs.alpha, pcs.beta, L0.vd.x, pv, sol, xinit);
    else launch_xp_update<float>(stream, nbs, per, pcs.alpha, pcs.beta, L0.vf.x, pv, sol, xinit);
    xinit = true;
  };
  precondition(nullptr);
  launch_pcg_scalars(stream, nbs, kPcgStart, 0.0, pcs);   // act = (b != 0), beta = 0, rz = z . r
  if (!mixed) launch_p_init<double>(stream, nbs, per, L0.vd.x, pv);
  else launch_p_init<float>(stream, nbs, per, L0.vf.x, pv);
  // Eagerly, the host reads the residuals after every iteration and stops
  // once all configurations have converged.  Under graph capture the loop
  // runs the iteration count of the eager call it was captured after; the
  // residuals are checked after each replay (a configuration that converged
  // earlier does not change in the extra iterations).
  const int fixed = capturing ? cap_iters[which] : 0;
  double relmax = 0.0;
  int it = 0;
  for (it = 1; it <= opt.mg_max_iter; ++it) {
    const int Ka = apply0<double>(pv, nullptr, qv, nullptr, nullptr, 0.0, 0.0, kApplyDot, partial);
    launch_sum_partials(stream, Ka, partial, pcs.pq, nbs);
    launch_pcg_scalars(stream, nbs, kPcgAlpha, 0.0, pcs);
    launch_sum_partials(stream, launch_r_update(stream, nbs, per, pcs.alpha, qv, rcur, rr, partial,
                                                mixed ? L0.vf.f : nullptr), partial, pcs.rr, nbs);
    rcur = rr;
    launch_pcg_scalars(stream, nbs, kPcgResid, opt.mg_rtol, pcs);
    if (capturing) {
      if (it >= fixed) break;
    } else {
      hip_check(hipMemcpyAsync(host_cs, pcs.rel, nbs * sizeof(double), hipMemcpyDeviceToHost, stream),
                "copy residuals");
      sync("mesh solve residual");
      relmax = 0.0;
      for (int bb = 0; bb < nbs; ++bb) relmax = std::max(relmax, host_cs[bb]);
      if (relmax <= opt.mg_rtol) break;
    }
    precondition(qv);
    launch_pcg_scalars(stream, nbs, mixed ? kPcgBetaPR : kPcgBeta, 0.0, pcs);
    set_p();
  }
  // the loop left through its break (converged, or the captured count):
  // the last iteration's x update is still pending (at the iteration cap
  // set_p has applied it)
  if (it <= opt.mg_max_iter) launch_x_final(stream, nbs, per, pcs.alpha, pv, sol, xinit);
  store_rel(which);
  check_launch("mesh solve");
  if (capturing) return;
  stats.mg_iterations = std::min(it, opt.mg_max_iter);
  stats.mg_rel_residual = relmax;
  if (!(relmax <= opt.mg_rtol))
    throw Status(FEP3M_ERR_NOT_CONVERGED, "mesh solve reached relative residual " + std::to_string(relmax));
}

// Gauge-fixed periodic solve: out = K^+ rhs with int out = 0.
// nsys = 2: rhs and out hold the forward then the adjoint blocks, solved
// together (which = 0).
void fep3m_ctx::mesh_solve(double *rhs, double *out, int which, int nsys) {
  nbs = nb * nsys;
  struct Reset { int &v; int to; ~Reset() { v = to; } } reset{nbs, nb};
  solve(rhs, out, which);
  const int Km = launch_mass_dot(stream, nbs, n, p, w1, out, partial);
  if (Km < 0) throw Status(FEP3M_ERR_UNSUPPORTED, "mass integral variant");
  launch_sum_partials(stream, Km, partial, gauge, nbs);
  launch_sub_const(stream, nbs, lv[0].ndof, 1.0 / (double(n) * n * n), gauge, out);
}

// Final relative residuals into the per-configuration slots: one system
// (forward or adjoint, by `which`) or both.
void fep3m_ctx::store_rel(int which) {
  if (nbs == nb) {
    launch_copy_f64(stream, nb, pcs.rel, cfgs(which ? kCsAdjRel : kCsFwdRel));
  } else {
    launch_copy_f64(stream, nb, pcs.rel, cfgs(kCsFwdRel));
    launch_copy_f64(stream, nb, pcs.rel + nb, cfgs(kCsAdjRel));
  }
}

// ----------------------------------------------------------------- evaluate

void fep3m_ctx::forward(const double *x, const double *Qc, double *Phi, double *U, bool pair_forces) {
  const int MT = nb * n * n * n;
  stage_mark(FEP3M_PROF_SORT, true);
  launch_fill_int(stream, MT, 0, count);
  launch_fill_int(stream, 4, 0, flags);
  const int gb = launch_bin(stream, nb, off_d, N, x, Qc, L, n, box ? 1 : 0, gtmp, elem, slot, count, flags, partial);
  launch_sum_partials(stream, gb, partial, cfgs(kCsQ), nb);
  launch_sum_partials(stream, gb, partial + size_t(nb) * gb, cfgs(kCsQabs), nb);
  if (!capturing) {   // under capture the same checks run after each replay
    hip_check(hipMemcpyAsync(host_cs, cs, 2 * size_t(nb) * sizeof(double), hipMemcpyDeviceToHost, stream), "copy");
    hip_check(hipMemcpyAsync(host_scal + 4, flags, sizeof(int), hipMemcpyDeviceToHost, stream), "copy");
    sync("binning");
    check_inputs();
  }

  launch_scan(stream, MT, count, start, maxcount, scan_scr);
  launch_scatter(stream, N, elem, slot, start, tmp);
  launch_rank(stream, N, tmp, elem, start, gtmp, Qc, perm, sg, sQ);
  items_titem = -1;   // the pair work list follows this call's element starts
  if (mixed) launch_local_f32(stream, n, N, sg, sQ, su, si, sel);
  stage_mark(FEP3M_PROF_SORT, false);
  if (box) {
    forward_box(Phi, U, pair_forces);
    return;
  }
  // overlap only with the decompositions of short blocks (one wave per
  // element, rows of elements) that interleave with the solve's; persistent
  // waves would hold every CU for the pass
  // and only on meshes of at least 2^16 elements in all: below that the pass
  // is too short to pay for the fork and the join (graph replays of 1000
  // charges on 8^3 elements: 1.25 -> 1.39 ms)
  if (opt.autotune == 2) plan = PairPlan{2, 2, 0};
  const bool overlap = !(opt.autotune == 1 && !tuned && !prof.on) && plan.kind != 1 && !arena && opt.pair_stream &&
                       size_t(nb) * n * n * n >= (size_t(1) << 16);
  if (overlap) {
    side_stream();
    hip_check(hipEventRecord(ev_fork, stream), "event");
    hip_check(hipStreamWaitEvent(pstream, ev_fork, 0), "wait");
    struct Restore { hipStream_t &s; hipStream_t to; ~Restore() { s = to; } } restore{stream, stream};
    stream = pstream;   // the pair pass's launches and stage events go to the second stream
    pair_pass(pair_forces);
    hip_check(hipEventRecord(ev_join, pstream), "event");
  }
  // the main stream waits for the pair pass before the interpolation, and on
  // any early exit, so that no later work overwrites what it reads
  struct Join {
    hipStream_t &s;
    hipEvent_t e;
    bool pending;
    void now() { if (pending) hip_check(hipStreamWaitEvent(s, e, 0), "wait"); pending = false; }
    ~Join() { if (pending) (void)hipStreamWaitEvent(s, e, 0); }
  } join{stream, ev_join, overlap};
  stage_mark(FEP3M_PROF_ASSIGN, true);
  stage_mark(FEP3M_PROF_MOMENTS, true);
  if (generic) {
    if (launch_moments_g(stream, nb, n, nl, N, start, sg, sQ, C) != 0)
      throw Status(FEP3M_ERR_UNSUPPORTED, "moments variant");
  } else {
    launch_moments(stream, nb, n, N, start, sg, sQ, C);
  }
  stage_mark(FEP3M_PROF_MOMENTS, false);
  stage_mark(FEP3M_PROF_LOAD, true);
  const int Kl = generic ? launch_load_g(stream, nb, n, p, span, nl, 0, C, gw, b, partial, lsep)
                         : launch_load(stream, nb, n, p, C, gw, b, partial);
  stage_mark(FEP3M_PROF_LOAD, false);
  if (Kl < 0) throw Status(FEP3M_ERR_UNSUPPORTED, "load variant");
  launch_sum_partials(stream, Kl, partial, cfgs(kCsLoad), nb);
  if (launch_sub_mass_ones(stream, nb, n, p, w1, cfgs(kCsLoad), b) != 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "projection variant");
  check_launch("assignment");
  stage_mark(FEP3M_PROF_ASSIGN, false);
  // With forces the adjoint right side (the charges' deposit, which does not
  // depend on phi) is built now and both systems go through one solve.
  lam_ready = pair_forces;
  if (pair_forces) {
    stage_mark(FEP3M_PROF_ADJ_SOLVE, true);
    adjoint_rhs();
    stage_mark(FEP3M_PROF_ADJ_SOLVE, false);
  }
  stage_mark(FEP3M_PROF_SOLVE, true);
  mesh_solve(b, sol, 0, pair_forces ? 2 : 1);
  stage_mark(FEP3M_PROF_SOLVE, false);
  stage_mark(FEP3M_PROF_NEAR, true);
  int ps;
  adj_near_ready = false;
  if (near_fft) {
    // with forces the deposits (built before the solve) are transformed too
    // and one pass over the spectrum serves both products
    ps = launch_near_fft(stream, nb, n, p, C, pair_forces ? gE : nullptr, spec, twd, zc, zpsi, zg, za);
    if (ps == 0)
      ps = mixed ? launch_psi_fft_finish<float>(stream, nb, n, p, twd, sol, zpsi, Welf)
                 : launch_psi_fft_finish<double>(stream, nb, n, p, twd, sol, zpsi, Wel);
    adj_near_ready = pair_forces;
    prof.near_both = pair_forces;
  } else if (generic) {   // the matrix cores where the family has a kernel there, else the table sums
    ps = launch_psi_mfma_g(stream, nb, n, nsr, p, nl, 0, C, T, sol, Wel);
    if (ps != 0) ps = launch_psi_g(stream, nb, n, nsr, p, nl, 0, C, T, sol, Wel);
  } else
    ps = mixed ? launch_psi<float>(stream, nb, n, nsr, p, 0, C, Tf, sol, Welf)
               : launch_psi<double>(stream, nb, n, nsr, p, 0, C, T, sol, Wel);
  if (ps != 0) throw Status(FEP3M_ERR_UNSUPPORTED, "near field variant");
  stage_mark(FEP3M_PROF_NEAR, false);
  if (overlap) join.now();
  else pair_pass(pair_forces);
  stage_mark(FEP3M_PROF_INTERP, true);
  stage_mark(FEP3M_PROF_INTERP_KERNEL, true);
  const int is = mixed ? launch_interp_f32(stream, nb, off_d, p, n, N, 1.0 / h, bas, su, sel, Welf, phip_s, perm,
                                           phim_s, phi_s, Phi)
                       : launch_interp(stream, nb, off_d, p, n, N, 1.0 / h, bas, sg, Wel, phip_s, perm, phim_s, phi_s,
                                       Phi);
  if (is != 0) throw Status(FEP3M_ERR_UNSUPPORTED, "interpolation variant");
  stage_mark(FEP3M_PROF_INTERP_KERNEL, false);
  if (U) {
    const int Ke = launch_energy(stream, nb, off_d, N, sQ, phi_s, partial);
    launch_sum_partials(stream, Ke, partial, cfgs(kCsEnergy), nb);
    launch_half(stream, nb, cfgs(kCsEnergy), U);
  }
  stage_mark(FEP3M_PROF_INTERP, false);
}

int fep3m_ctx::pair_launch(const PairPlan &pl, bool pair_forces) {
  double *fp = pair_forces ? fpair : nullptr;
  if (pl.kind == 2) {
    if (mixed) return -1;
    return launch_pair_rows(stream, nb, n, nsr, pl.titem, box ? 1 : 0, N, start, rowstart, rnit, ritem_start,
                            riscan_max, ritems, scan_scr, sg, sQ, phip_s, fp);
  }
  if (pl.kind == 0)
    return mixed ? launch_pair_f32(stream, nb, n, nsr, N, start, si, sel, phip_s, fp)
                 : launch_pair(stream, nb, n, nsr, N, start, sg, sQ, phip_s, fp);
  const int MT = nb * n * n * n;
  if (items_titem != pl.titem) {
    launch_items(stream, MT, pl.titem, start, nit, item_start, iscan_max, items, scan_scr);
    items_titem = pl.titem;
  }
  return mixed ? launch_pair_queue_f32(stream, pl.waves, n, nsr, N, start, items, item_start + MT, icounter, pl.titem,
                                       si, sel, phip_s, fp)
               : launch_pair_queue(stream, pl.waves, n, nsr, N, start, items, item_start + MT, icounter, pl.titem, sg,
                                   sQ, phip_s, fp);
}

// Time each candidate decomposition of the pair sum on this call's data and
// keep the fastest.  Kinds 0 and 1 produce identical results; kind 2 sums
// each target's pairs in another order (equal to rounding), so the chosen
// plan runs once more when it is not the last one timed: the call's outputs
// are those of the plan every later call uses.
void fep3m_ctx::tune_pairs(bool pair_forces) {
  std::vector<PairPlan> cand;
  cand.push_back(PairPlan{0, 0, 0});
  for (int titem : {8, 32, 64})
    for (int per_cu : {16, 32}) cand.push_back(PairPlan{1, titem, per_cu * cus});
  if (!mixed)   // rows of elements, 1, 2 or 4 lanes per target
    for (int sl : {1, 2, 4}) cand.push_back(PairPlan{2, sl, 0});
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  double best = 1e300, dflt = 0.0;
  PairPlan pick = cand[0];
  for (const PairPlan &pl : cand) {
    if (pl.kind == 1 && items_titem != pl.titem) {   // list construction is not part of the timing
      launch_items(stream, nb * n * n * n, pl.titem, start, nit, item_start, iscan_max, items, scan_scr);
      items_titem = pl.titem;
    }
    hip_check(hipEventRecord(e0, stream), "event");
    if (pair_launch(pl, pair_forces) != 0) throw Status(FEP3M_ERR_UNSUPPORTED, "pair variant");
    hip_check(hipEventRecord(e1, stream), "event");
    hip_check(hipEventSynchronize(e1), "tuning");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    if (pl.kind == 0) dflt = ms;
    if (ms < best) { best = ms; pick = pl; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const PairPlan &last = cand.back();
  if (pick.kind != last.kind || pick.titem != last.titem || pick.waves != last.waves) {
    if (pick.kind == 1 && items_titem != pick.titem) {
      launch_items(stream, nb * n * n * n, pick.titem, start, nit, item_start, iscan_max, items, scan_scr);
      items_titem = pick.titem;
    }
    if (pair_launch(pick, pair_forces) != 0) throw Status(FEP3M_ERR_UNSUPPORTED, "pair variant");
  }
  plan = pick;
  tuned = true;
  stats.tune_ms_best = best;
  stats.tune_ms_default = dflt;
}

void fep3m_ctx::pair_pass(bool pair_forces) {
  if (opt.autotune == 1 && !tuned && !prof.on) tune_pairs(pair_forces);
  stage_mark(FEP3M_PROF_PAIR, true);
  if (pair_launch(plan, pair_forces) != 0) throw Status(FEP3M_ERR_UNSUPPORTED, "pair variant");
  prof.pair_forces = pair_forces;
  stage_mark(FEP3M_PROF_PAIR, false);
  stats.pair_variant = plan.kind;
  stats.pair_item_targets = plan.titem;
  stats.pair_waves = plan.waves;
}

// Reverse pass over the state the forward pass left in the context: deposit,
// second mesh solve, moment adjoint, per-charge gradients.
// Adjoint right side: deposit g, assembly G, compatibility projection.
void fep3m_ctx::adjoint_rhs() {
  stage_mark(FEP3M_PROF_DEPOSIT, true);
  if (launch_deposit(stream, nb, p, n, N, bas, start, sg, sQ, gE) != 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "deposit variant");
  const int Ka = launch_assemble(stream, nb, p, n, gE, Gv, partial);
  if (Ka < 0) throw Status(FEP3M_ERR_UNSUPPORTED, "assembly variant");
  stage_mark(FEP3M_PROF_DEPOSIT, false);
  launch_sum_partials(stream, Ka, partial, cfgs(kCsAdjLoad), nb);
  if (launch_sub_mass_ones(stream, nb, n, p, w1, cfgs(kCsAdjLoad), Gv) != 0)
    throw Status(FEP3M_ERR_UNSUPPORTED, "projection variant");
}

void fep3m_ctx::reverse(double *F, double *dUdQ) {
  if (box) {
    reverse_box(F, dUdQ);
    return;
  }
  const int fwd_iters = stats.mg_iterations;
  const double fwd_rel = stats.mg_rel_residual;
  if (!lam_ready) {   // lambda not solved with phi: a backward call after an energy-only forward
    stage_mark(FEP3M_PROF_ADJ_SOLVE, true);
    adjoint_rhs();
    mesh_solve(Gv, lam, 1);
    stage_mark(FEP3M_PROF_ADJ_SOLVE, false);
    lam_ready = true;
  }
  stage_mark(FEP3M_PROF_ADJ_NEAR, true);
  int as;
  if (near_fft) {
    prof.adj_full = !adj_near_ready;
    as = adj_near_ready ? 0 : launch_near_fft(stream, nb, n, p, nullptr, gE, spec, twd, zc, zpsi, zg, za);
    if (as == 0) as = launch_adj_fft_finish(stream, nb, n, p, lam, gw, za, Aadj);
    adj_near_ready = false;
  } else if (generic) {
    as = launch_adj_g(stream, nb, n, nsr, p, span, nl, 0, gE, Tt, lam, gw, Aadj, lsep);
  } else {
    as = launch_adj_moments(stream, nb, p, n, nsr, 0, gE, Tt, lam, gw, Aadj);
  }
  if (as != 0) throw Status(FEP3M_ERR_UNSUPPORTED, "adjoint variant");
  stage_mark(FEP3M_PROF_ADJ_NEAR, false);
  stage_mark(FEP3M_PROF_FORCES, true);
  const int fs =
      mixed ? launch_forces<float>(stream, nb, off_d, p, n, nl, N, 1.0 / h, bas, sg, sQ, Welf, Aadj, fpair, phip_s,
                                   phim_s, perm, F, dUdQ)
            : launch_forces<double>(stream, nb, off_d, p, n, nl, N, 1.0 / h, bas, sg, sQ, Wel, Aadj, fpair, phip_s,
                                    phim_s, perm, F, dUdQ);
  if (fs != 0) throw Status(FEP3M_ERR_UNSUPPORTED, "forces variant");
  stage_mark(FEP3M_PROF_FORCES, false);
  if (capturing) return;   // counts are recorded by the eager call before a capture
  stats.adj_iterations = stats.mg_iterations;
  stats.mg_iterations = fwd_iters;
  stats.mg_rel_residual = fwd_rel;
}

void fep3m_ctx::finish(bool count_pairs) {
  if (count_pairs) {
    launch_fill_int(stream, 2, 0, reinterpret_cast<int *>(paircount));
    launch_pair_count(stream, nb, n, nsr, start, paircount);
  }
  if (capturing) return;
  if (count_pairs) {
    hip_check(hipMemcpyAsync(host_scal + 8, paircount, sizeof(unsigned long long), hipMemcpyDeviceToHost, stream),
              "copy");
    hip_check(hipMemcpyAsync(host_scal + 9, maxcount, sizeof(int), hipMemcpyDeviceToHost, stream), "copy");
  }
  check_launch("evaluation");
  sync("evaluation");
  if (count_pairs) finish_host();
  if (prof.on) profile_collect();
}

void fep3m_ctx::finish_host() {   // pair statistics already copied to host_scal[8..9]
  unsigned long long pc;
  std::memcpy(&pc, host_scal + 8, sizeof(pc));
  int mc;
  std::memcpy(&mc, host_scal + 9, sizeof(int));
  stats.near_pairs = int64_t(pc);
  stats.max_per_element = mc;
}

void fep3m_ctx::run_once(const double *x, const double *Qc, double *Phi, double *U, double *F, double *dUdQ) {
  prof.begin_call();
  stage_mark(FEP3M_PROF_TOTAL, true);
  forward(x, Qc, Phi, U, F != nullptr);
  if (F) reverse(F, dUdQ);
  stage_mark(FEP3M_PROF_TOTAL, false);
  finish(true);
}

void fep3m_ctx::evaluate(const double *x, const double *Qc, double *Phi, double *U, double *F, double *dUdQ) {
  fwd_valid = false;
  if (opt.use_graph && !prof.on && opt.solver == FEP3M_SOLVER_MG) evaluate_graph(x, Qc, Phi, U, F, dUdQ);
  else run_once(x, Qc, Phi, U, F, dUdQ);
  ++generation;
  stats.generation = int64_t(generation);
  fwd_valid = true;
}

// Graph mode.  The evaluation runs on an internal stream ordered after the
// caller's stream (and the caller's stream after it), on context copies of
// the inputs and outputs.  A call that asks for the same outputs as the
// captured graph replays it and then checks, on the host, the input flags,
// the per-configuration neutrality and the final residuals of the mesh
// solves; any other call (or a replay whose solves needed more iterations
// than were captured) runs eagerly, which also yields the iteration counts,
// and then captures the evaluation again.
void fep3m_ctx::evaluate_graph(const double *x, const double *Qc, double *Phi, double *U, double *F, double *dUdQ) {
  if (!gstream) {
    hip_check(hipStreamCreateWithFlags(&gstream, hipStreamNonBlocking), "graph stream");
    hip_check(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming), "event");
    hip_check(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming), "event");
    gx = alloc<double>(3 * size_t(N), "graph positions");
    gQ = alloc<double>(size_t(N), "graph charges");
    gPhi = alloc<double>(size_t(N), "graph potentials");
    gU = alloc<double>(size_t(nb), "graph energies");
    gF = alloc<double>(3 * size_t(N), "graph forces");
    gD = alloc<double>(size_t(N), "graph charge derivatives");
  }
  const int mask = (Phi ? 1 : 0) | (U ? 2 : 0) | (F ? 4 : 0) | (dUdQ ? 8 : 0);
  double *oPhi = Phi ? gPhi : nullptr, *oU = U ? gU : nullptr, *oF = F ? gF : nullptr, *oD = dUdQ ? gD : nullptr;
  hipStream_t user = stream;
  hip_check(hipEventRecord(ev_in, user), "event");
  hip_check(hipStreamWaitEvent(gstream, ev_in, 0), "wait");
  stream = gstream;
  try {
    launch_copy_f64(stream, 3 * size_t(N), x, gx);
    launch_copy_f64(stream, size_t(N), Qc, gQ);
    bool done = false;
    if (graph_ready && mask == gmask) {
      hip_check(hipGraphLaunch(gexec, gstream), "graph launch");
      hip_check(hipMemcpyAsync(host_cs, cs, size_t(kCsSlots) * nb * sizeof(double), hipMemcpyDeviceToHost, gstream),
                "copy");
      hip_check(hipMemcpyAsync(host_scal + 4, flags, sizeof(int), hipMemcpyDeviceToHost, gstream), "copy");
      hip_check(hipMemcpyAsync(host_scal + 8, paircount, sizeof(unsigned long long), hipMemcpyDeviceToHost, gstream),
                "copy");
      hip_check(hipMemcpyAsync(host_scal + 9, maxcount, sizeof(int), hipMemcpyDeviceToHost, gstream), "copy");
      sync("graph replay");
      stats.graph_replays = ++replays;
      check_inputs();
      double fr = 0.0, ar = 0.0;
      for (int bb = 0; bb < nb; ++bb) {
        fr = std::max(fr, host_cs[kCsFwdRel * nb + bb]);
        ar = std::max(ar, host_cs[kCsAdjRel * nb + bb]);
      }
      if (fr <= opt.mg_rtol && (!F || ar <= opt.mg_rtol)) {
        done = true;
        lam_ready = F != nullptr;   // the replayed forward solved lambda only with forces
        adj_near_ready = false;     // the replay's reverse pass consumed it
        finish_host();
        stats.mg_iterations = cap_iters[0];
        stats.mg_rel_residual = fr;
        if (F) stats.adj_iterations = cap_iters[1];
      }
    }
    if (!done) {
      run_once(gx, gQ, oPhi, oU, oF, oD);   // eager; synchronises and yields the iteration counts
      cap_iters[0] = stats.mg_iterations;
      cap_iters[1] = F ? stats.adj_iterations : 0;
      if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; }
      if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
      graph_ready = false;
      side_stream();
      hip_check(hipStreamBeginCapture(gstream, hipStreamCaptureModeThreadLocal), "begin capture");
      capturing = true;
      try {
        run_once(gx, gQ, oPhi, oU, oF, oD);
      } catch (...) {
        capturing = false;
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(gstream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      capturing = false;
      hip_check(hipStreamEndCapture(gstream, &graph), "end capture");
      hip_check(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0), "instantiate");
      graph_ready = true;
      gmask = mask;
    }
    if (Phi) launch_copy_f64(stream, size_t(N), gPhi, Phi);
    if (U) launch_copy_f64(stream, size_t(nb), gU, U);
    if (F) launch_copy_f64(stream, 3 * size_t(N), gF, F);
    if (dUdQ) launch_copy_f64(stream, size_t(N), gD, dUdQ);
    check_launch("graph outputs");
  } catch (...) {
    stream = user;
    throw;
  }
  hip_check(hipEventRecord(ev_out, gstream), "event");
  hip_check(hipStreamWaitEvent(user, ev_out, 0), "wait");
  stream = user;
}

void fep3m_ctx::backward(int64_t gen, double *F, double *dUdQ) {
  if (!fwd_valid || gen != int64_t(generation))
    throw Status(FEP3M_ERR_ARG, "backward needs the state of forward call " + std::to_string(gen) +
                                    " but the context holds call " + std::to_string(generation) +
                                    (fwd_valid ? "" : " (failed)"));
  prof.begin_call();
  stage_mark(FEP3M_PROF_TOTAL, true);
  pair_pass(true);       // pair gradients recomputed, not stored by the forward call
  reverse(F, dUdQ);
  stage_mark(FEP3M_PROF_TOTAL, false);
  finish(false);
}

void fep3m_ctx::profile_collect() {
  for (int s = 0; s < FEP3M_PROF_SLOTS; ++s) {
    if (s == FEP3M_PROF_FINE_APPLY || s == FEP3M_PROF_FINE_APPLY_F32 || !(prof.marked & (1u << s))) continue;
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, prof.stage_ev[2 * s], prof.stage_ev[2 * s + 1]), "elapsed");
    prof.acc.ms[s] += ms;
    prof.acc.count[s] += 1;
  }
  const double S = 2 * nsr + 1;
  const double Me = double(n) * n * n * nb, NM = double(p + 1) * (p + 1) * (p + 1);
  double near_flop = 2.0 * double(na) * NM * S * S * S * Me, adj_work = near_flop;
  if (near_fft) {   // bytes in and out of every launch of the FFT pipelines
    const double spec_b = double(spec_freqs(n)) * 8.0 * NM * 16.0;
    const double f4 = Me * 4.0 * 16.0, f108 = Me * NM / 2.0 * 16.0, phi_b = Me * 125.0 * 8.0;
    const double w_b = Me * NM * (mixed ? 4.0 : 8.0);
    // moments: 3 passes; products; Psi: 2 passes and the last with phi and W
    const double psi_part = 3.0 * 2.0 * f4 + (spec_b + f4 + f108) + 2.0 * 2.0 * f108 + (f108 + phi_b + w_b);
    // deposits: 3 passes; their products (f108 in, f4 out); B: 3 passes
    const double adj_part = 3.0 * 2.0 * f108 + (f108 + f4) + 3.0 * 2.0 * f4;
    const double finish = f4 + phi_b + Me * 8.0 * 8.0;   // lambda term and A
    near_flop = psi_part + (prof.near_both ? adj_part : 0.0);
    adj_work = finish + (prof.adj_full ? adj_part + spec_b : 0.0);
  }
  if (prof.marked & (1u << FEP3M_PROF_NEAR)) prof.acc.work[FEP3M_PROF_NEAR] += near_flop;
  if (prof.marked & (1u << FEP3M_PROF_PAIR))
    prof.acc.work[FEP3M_PROF_PAIR] += (prof.pair_forces ? 20.0 : 11.0) * double(stats.near_pairs);
  if (prof.marked & (1u << FEP3M_PROF_ADJ_NEAR)) prof.acc.work[FEP3M_PROF_ADJ_NEAR] += adj_work;
  // bytes of the assignment, deposit and interpolation kernels
  const double P3 = double(lv[0].ndof) * nb, Nd = double(N);
  const double bytes[4] = {32.0 * Nd + (4.0 + 8.0 * na) * Me,                  // moments
                           8.0 * na * Me + 8.0 * P3,                           // load
                           32.0 * Nd + 2.0 * 8.0 * NM * Me + 8.0 * P3,         // deposit and assembly
                           60.0 * Nd + (mixed ? 4.0 : 8.0) * NM * Me};         // interpolation
  const int slots[4] = {FEP3M_PROF_MOMENTS, FEP3M_PROF_LOAD, FEP3M_PROF_DEPOSIT, FEP3M_PROF_INTERP_KERNEL};
  for (int k = 0; k < 4; ++k)
    if (prof.marked & (1u << slots[k])) prof.acc.work[slots[k]] += bytes[k];
  for (int k = 0; k < prof.kused; ++k) {
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, prof.kev[2 * k], prof.kev[2 * k + 1]), "elapsed");
    prof.acc.ms[prof.kslot[k]] += ms;
    prof.acc.count[prof.kslot[k]] += 1;
    prof.acc.work[prof.kslot[k]] += prof.kwork[k];
  }
}

// ----------------------------------------------------------------- C ABI

namespace {

thread_local std::string g_create_error;

template <class F>
int guarded(fep3m_ctx *ctx, F &&f) {
  try {
    if (ctx) ctx->err.clear();
    f();
    return FEP3M_OK;
  } catch (const Status &s) {
    if (ctx) ctx->err = s.what();
    return s.code;
  } catch (const std::bad_alloc &) {
    if (ctx) ctx->err = "host allocation failed";
    return FEP3M_ERR_OOM;
  } catch (const std::exception &e) {
    if (ctx) ctx->err = e.what();
    return FEP3M_ERR_DEVICE;
  }
}

bool valid_options(const fep3m_options &o, std::string &why) {
  if (o.n_sr < 1 || o.n_sr > 3) { why = "n_sr must be 1..3"; return false; }
  if (o.precision != FEP3M_PRECISION_FP64 && o.precision != FEP3M_PRECISION_MIXED) { why = "unknown precision"; return false; }
  if (!(o.mg_rtol > 0.0) || !(o.mg_rtol < 1.0)) { why = "mg_rtol must be in (0, 1)"; return false; }
  if (o.mg_max_iter < 1 || o.mg_max_iter > 1000) { why = "mg_max_iter must be 1..1000"; return false; }
  if (o.cheb_degree < 1 || o.cheb_degree > 10) { why = "cheb_degree must be 1..10"; return false; }
  if (o.autotune < 0 || o.autotune > 2) { why = "autotune must be 0, 1 or 2"; return false; }
  if (o.autotune == 2 && o.precision != FEP3M_PRECISION_FP64) { why = "autotune = 2 needs float64"; return false; }
  if (o.use_graph != 0 && o.use_graph != 1) { why = "use_graph must be 0 or 1"; return false; }
  if (o.solver != FEP3M_SOLVER_MG && o.solver != FEP3M_SOLVER_FDM) { why = "unknown solver"; return false; }
  if (o.near_field < FEP3M_NEAR_AUTO || o.near_field > FEP3M_NEAR_FFT) { why = "unknown near_field"; return false; }
  if (o.support != FEP3M_SUPPORT_ONE && o.support != FEP3M_SUPPORT_27) { why = "unknown support"; return false; }
  if (o.pair_stream != 0 && o.pair_stream != 1) { why = "pair_stream must be 0 or 1"; return false; }
  if (o.boundary != FEP3M_BOUNDARY_PERIODIC && o.boundary != FEP3M_BOUNDARY_GROUNDED &&
      o.boundary != FEP3M_BOUNDARY_INSULATED) {
    why = "unknown boundary";
    return false;
  }
  if (o.table_box % 2 == 0 || o.table_box < 2 * o.n_sr + 3 || o.table_box > 41) {
    why = "table_box must be odd, > 2 n_sr + 1 and <= 41";
    return false;
  }
  return true;
}

}  // namespace

extern "C" {

int fep3m_default_options(fep3m_options *opt) {
  if (!opt) return FEP3M_ERR_ARG;
  opt->n_sr = 3;
  opt->precision = FEP3M_PRECISION_FP64;
  opt->mg_rtol = 1e-7;
  opt->mg_max_iter = 60;
  opt->cheb_degree = 3;
  opt->table_box = 2 * 3 + 9;
  opt->autotune = 1;
  opt->use_graph = 0;
  opt->solver = FEP3M_SOLVER_MG;
  opt->near_field = FEP3M_NEAR_AUTO;
  opt->pair_stream = 1;
  opt->support = FEP3M_SUPPORT_ONE;
  opt->boundary = FEP3M_BOUNDARY_PERIODIC;
  return FEP3M_OK;
}

namespace {

int create_common(double L, const std::vector<int64_t> &Ns, const int32_t dims[3], int32_t q,
                  const fep3m_options *opt, fep3m_ctx **out, bool static_storage = false) {
  if (!out) return FEP3M_ERR_ARG;
  *out = nullptr;
  fep3m_options o;
  if (opt) o = *opt; else fep3m_default_options(&o);
  std::string why;
  if (!dims) return FEP3M_ERR_ARG;
  if (!(L > 0.0) || !std::isfinite(L)) return FEP3M_ERR_ARG;
  if (Ns.empty() || Ns.size() > 1024) return FEP3M_ERR_ARG;
  int64_t total = 0;
  for (int64_t v : Ns) {
    if (v < 2 || v > (int64_t(1) << 30)) return FEP3M_ERR_ARG;
    total += v;
  }
  if (total > (int64_t(1) << 30)) return FEP3M_ERR_ARG;
  if (dims[0] != dims[1] || dims[1] != dims[2]) return FEP3M_ERR_ARG;
  if (int64_t(Ns.size()) * dims[0] * dims[0] * dims[0] > (int64_t(1) << 28)) return FEP3M_ERR_ARG;
  if (!valid_options(o, why)) return FEP3M_ERR_ARG;
  if (dims[0] < 2 * o.n_sr + 1 || dims[0] > 512) return FEP3M_ERR_ARG;
  if (o.support == FEP3M_SUPPORT_ONE ? (q < 2 || q > 6) : (q < 1 || q > 4)) return FEP3M_ERR_ARG;
  if (q + 2 > kMaxP) {
    g_create_error = "element orders above 6 (one-element screens of degree 5 and 6) are not implemented";
    return FEP3M_ERR_UNSUPPORTED;
  }
  if (!(o.support == FEP3M_SUPPORT_ONE && q == 3)) {   // the other screen families: float64, table sums
    if (o.precision != FEP3M_PRECISION_FP64 || o.near_field == FEP3M_NEAR_FFT) {
      g_create_error = "screens other than the one-element q = 3 screen run in float64 with the direct near field";
      return FEP3M_ERR_UNSUPPORTED;
    }
  }
  if (o.near_field == FEP3M_NEAR_FFT && !fft_size_ok(dims[0])) return FEP3M_ERR_UNSUPPORTED;
  if (o.boundary != FEP3M_BOUNDARY_PERIODIC &&
      (o.support != FEP3M_SUPPORT_ONE || o.precision != FEP3M_PRECISION_FP64 || o.solver != FEP3M_SOLVER_FDM ||
       o.near_field == FEP3M_NEAR_FFT || o.use_graph || static_storage)) {
    g_create_error = "the grounded and insulating boxes take one-element screens in float64 with the exact mesh solve "
                     "and the direct near field, eager (no graph, no static storage)";
    return FEP3M_ERR_UNSUPPORTED;
  }
  int dev = -1;
  if (static_storage) {
    // no tuning events, graph staging buffers, side stream or library handles
    if (o.use_graph || o.solver != FEP3M_SOLVER_MG) {
      g_create_error = "static contexts support neither use_graph nor the FDM solver";
      return FEP3M_ERR_UNSUPPORTED;
    }
    o.autotune = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
      g_create_error = "no usable device for static storage";
      return FEP3M_ERR_DEVICE;
    }
  }
  std::unique_ptr<fep3m_ctx> ctx(new (std::nothrow) fep3m_ctx());
  if (!ctx) return FEP3M_ERR_OOM;
  if (static_storage) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_busy[dev]) {
      g_create_error = "the device's static storage is held by another static context (destroy it first)";
      return FEP3M_ERR_ARG;
    }
    if (!g_static_ptr[dev]) {
      void *ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        g_create_error = std::string("static storage address: ") + hipGetErrorString(e);
        return FEP3M_ERR_DEVICE;
      }
      g_static_ptr[dev] = ptr;
    }
    g_static_busy[dev] = true;
    ctx->arena = static_cast<unsigned char *>(g_static_ptr[dev]);
    ctx->arena_dev = dev;   // the destructor releases the claim
  }
  int st = guarded(ctx.get(), [&] {
    if (ctx->arena)   // the array keeps the last static context's contents
      hip_check(hipMemset(ctx->arena, 0, kStaticBytes), "clear static storage");
    ctx->build(L, Ns, dims[0], q, o);
  });
  if (st != FEP3M_OK) {
    g_create_error = ctx->err;
    return st;
  }
  *out = ctx.release();
  return FEP3M_OK;
}

}  // namespace

int fep3m_create_ex(double L, int64_t N, const int32_t dims[3], int32_t q, const fep3m_options *opt, fep3m_ctx **out) {
  return create_common(L, std::vector<int64_t>{N}, dims, q, opt, out);
}

int fep3m_create_batch(double L, int32_t nconf, const int64_t *N_per_conf, const int32_t dims[3], int32_t q,
                       const fep3m_options *opt, fep3m_ctx **out) {
  if (out) *out = nullptr;
  if (!N_per_conf || nconf < 1 || nconf > 1024) return FEP3M_ERR_ARG;
  return create_common(L, std::vector<int64_t>(N_per_conf, N_per_conf + nconf), dims, q, opt, out);
}

int fep3m_create(double L, int64_t N, const int32_t dims[3], int32_t q, fep3m_ctx **out) {
  return fep3m_create_ex(L, N, dims, q, nullptr, out);
}

int fep3m_create_static(double L, int64_t N, const int32_t dims[3], int32_t q, const fep3m_options *opt,
                        fep3m_ctx **out) {
  return create_common(L, std::vector<int64_t>{N}, dims, q, opt, out, true);
}

int fep3m_set_stream(fep3m_ctx *ctx, void *hip_stream) {
  if (!ctx) return FEP3M_ERR_ARG;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return FEP3M_OK;
}

int fep3m_potential(fep3m_ctx *ctx, const double *x, const double *Q, double *Phi) {
  if (!ctx || !x || !Q || !Phi) return FEP3M_ERR_ARG;
  return guarded(ctx, [&] { ctx->evaluate(x, Q, Phi, nullptr); });
}

int fep3m_energy(fep3m_ctx *ctx, const double *x, const double *Q, double *Phi, double *U) {
  if (!ctx || !x || !Q || !Phi || !U) return FEP3M_ERR_ARG;
  return guarded(ctx, [&] { ctx->evaluate(x, Q, Phi, U); });
}

int fep3m_energy_forces_ex(fep3m_ctx *ctx, const double *x, const double *Q, double *Phi, double *U, double *F,
                           double *dUdQ) {
  if (!ctx || !x || !Q || !U || !F) return FEP3M_ERR_ARG;
  return guarded(ctx, [&] { ctx->evaluate(x, Q, Phi ? Phi : ctx->Phi_int, U, F, dUdQ); });
}

int fep3m_energy_forces(fep3m_ctx *ctx, const double *x, const double *Q, double *U, double *F) {
  return fep3m_energy_forces_ex(ctx, x, Q, nullptr, U, F, nullptr);
}

int fep3m_backward(fep3m_ctx *ctx, int64_t generation, double *F, double *dUdQ) {
  if (!ctx || (!F && !dUdQ)) return FEP3M_ERR_ARG;
  return guarded(ctx, [&] { ctx->backward(generation, F, dUdQ); });
}

int64_t fep3m_stage_bytes(const fep3m_ctx *ctx, int32_t stage) {
  if (!ctx) return 0;
  const int64_t M = int64_t(ctx->n) * ctx->n * ctx->n * ctx->nb;
  const int64_t P3 = ctx->box ? int64_t(ctx->Pb) * ctx->Pb * ctx->Pb * ctx->nb
                              : int64_t(ctx->lv.empty() ? 0 : ctx->lv[0].ndof) * ctx->nb;
  switch (stage) {
    case 0: return ctx->N * 4;
    case 1: return (M + 1) * 4;
    case 2: return M * ctx->na * 8;
    case 3: case 4: return P3 * 8;
    case 5: case 6: return ctx->N * 8;
    case 7: return int64_t(ctx->T_host.size()) * 8;
    default: return 0;
  }
}

int fep3m_debug_stage(fep3m_ctx *ctx, int32_t stage, void *out, int64_t out_bytes) {
  if (!ctx || !out) return FEP3M_ERR_ARG;
  const int64_t need = fep3m_stage_bytes(ctx, stage);
  if (need == 0 || out_bytes < need) {
    ctx->err = "unknown stage or buffer too small";
    return FEP3M_ERR_ARG;
  }
  return guarded(ctx, [&] {
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    switch (stage) {
      case 0: hip_check(hipMemcpyAsync(out, ctx->perm, need, k, ctx->stream), "stage"); break;
      case 1: hip_check(hipMemcpyAsync(out, ctx->start, need, k, ctx->stream), "stage"); break;
      case 2: hip_check(hipMemcpyAsync(out, ctx->C, need, k, ctx->stream), "stage"); break;
      case 3: hip_check(hipMemcpyAsync(out, ctx->box ? ctx->bxb : ctx->b, need, k, ctx->stream), "stage"); break;
      case 4: hip_check(hipMemcpyAsync(out, ctx->box ? ctx->bxphi : ctx->sol, need, k, ctx->stream), "stage"); break;
      case 5: launch_unpermute(ctx->stream, ctx->N, 1.0 / ctx->h, ctx->perm, ctx->phip_s, static_cast<double *>(out)); break;
      case 6: launch_unpermute(ctx->stream, ctx->N, 1.0, ctx->perm, ctx->phim_s, static_cast<double *>(out)); break;
      case 7: hip_check(hipMemcpyAsync(out, ctx->T_host.data(), need, hipMemcpyHostToDevice, ctx->stream), "stage"); break;
    }
    ctx->check_launch("stage");
    ctx->sync("stage");
  });
}

int fep3m_set_profiling(fep3m_ctx *ctx, int32_t on) {
  if (!ctx) return FEP3M_ERR_ARG;
  return guarded(ctx, [&] {
    if (on && ctx->prof.kev.empty()) {
      for (hipEvent_t &e : ctx->prof.stage_ev) hip_check(hipEventCreate(&e), "event create");
      ctx->prof.kev.resize(2 * 512);
      ctx->prof.kwork.resize(512);
      ctx->prof.kslot.resize(512);
      for (hipEvent_t &e : ctx->prof.kev) hip_check(hipEventCreate(&e), "event create");
    }
    ctx->prof.on = on != 0;
    ctx->prof.acc = fep3m_profile{};
  });
}

int fep3m_get_profile(const fep3m_ctx *ctx, fep3m_profile *prof) {
  if (!ctx || !prof) return FEP3M_ERR_ARG;
  *prof = ctx->prof.acc;
  return FEP3M_OK;
}

int fep3m_get_stats(const fep3m_ctx *ctx, fep3m_stats *stats) {
  if (!ctx || !stats) return FEP3M_ERR_ARG;
  *stats = ctx->stats;
  return FEP3M_OK;
}

void fep3m_destroy(fep3m_ctx *ctx) { delete ctx; }

const char *fep3m_last_error(const fep3m_ctx *ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->err.c_str();
}

const char *fep3m_status_string(int status) {
  switch (status) {
    case FEP3M_OK: return "ok";
    case FEP3M_ERR_ARG: return "invalid argument";
    case FEP3M_ERR_NOT_NEUTRAL: return "charges are not neutral";
    case FEP3M_ERR_NONFINITE: return "non-finite input";
    case FEP3M_ERR_NOT_CONVERGED: return "mesh solve did not converge";
    case FEP3M_ERR_DEVICE: return "device error";
    case FEP3M_ERR_OOM: return "out of memory";
    case FEP3M_ERR_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

int fep3m_host_tables(int32_t q, int32_t support, int32_t n_sr, int32_t box, double *out, int64_t out_len) {
  if (!out || (support != FEP3M_SUPPORT_ONE && support != FEP3M_SUPPORT_27) || n_sr < 1 || n_sr > 3 ||
      box % 2 == 0 || box < 2 * n_sr + 3 || box > 41)
    return FEP3M_ERR_ARG;
  if (support == FEP3M_SUPPORT_ONE ? (q < 2 || q > 6) : (q < 1 || q > 4)) return FEP3M_ERR_ARG;
  const Screen1D scr = make_screen(q, support);
  const int p = q + 2, S = 2 * n_sr + 1, nl = scr.d + 1;
  const int64_t need = int64_t(nl) * nl * nl * S * S * S * (p + 1) * (p + 1) * (p + 1);
  if (out_len < need) return FEP3M_ERR_ARG;
  try {
    Vec T;
    compute_tables(p, scr, n_sr, box, T);
    std::memcpy(out, T.data(), size_t(need) * sizeof(double));
  } catch (...) {
    return FEP3M_ERR_ARG;
  }
  return FEP3M_OK;
}

}  // extern "C"
