"""MI355X finite-element P3M: Python binding of libfep3m.so.

Argument marshalling only: every step of the evaluation runs in the HIP
kernels of the C library (include/fep3m.h).  PyTorch provides device memory
and the current HIP stream.  If the library has not been built the import
still succeeds but every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfep3m.so")

OK = 0
ERR_ARG = -1
ERR_NOT_NEUTRAL = -2
ERR_NONFINITE = -3
ERR_NOT_CONVERGED = -4
ERR_DEVICE = -5
ERR_OOM = -6
ERR_UNSUPPORTED = -7

PRECISION_FP64 = 0
PRECISION_MIXED = 1

SOLVER_MG = 0
SOLVER_FDM = 1

NEAR_AUTO = 0
NEAR_DIRECT = 1
NEAR_FFT = 2

STAGES = {"perm": 0, "start": 1, "C": 2, "b": 3, "phi": 4, "Phi_p": 5, "Phi_m": 6, "T": 7}


class Options(ctypes.Structure):
    _fields_ = [("n_sr", ctypes.c_int32), ("precision", ctypes.c_int32), ("mg_rtol", ctypes.c_double),
                ("mg_max_iter", ctypes.c_int32), ("cheb_degree", ctypes.c_int32), ("table_box", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("solver", ctypes.c_int32),
                ("near_field", ctypes.c_int32), ("pair_stream", ctypes.c_int32), ("support", ctypes.c_int32),
                ("boundary", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("mg_iterations", ctypes.c_int32), ("mg_rel_residual", ctypes.c_double),
                ("near_pairs", ctypes.c_int64), ("max_per_element", ctypes.c_int32),
                ("adj_iterations", ctypes.c_int32),
                ("mg_levels", ctypes.c_int32), ("create_seconds", ctypes.c_double),
                ("generation", ctypes.c_int64), ("pair_variant", ctypes.c_int32),
                ("pair_item_targets", ctypes.c_int32), ("pair_waves", ctypes.c_int32),
                ("tune_ms_best", ctypes.c_double), ("tune_ms_default", ctypes.c_double),
                ("graph_replays", ctypes.c_int64), ("near_fft", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64)]


PROF_SLOTS = ["sort", "assign", "solve", "near", "pair", "interp", "fine_apply", "total",
              "adj_solve", "adj_near", "forces", "fine_apply_f32", "moments", "load", "deposit", "interp_kernel"]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(PROF_SLOTS)), ("count", ctypes.c_int64 * len(PROF_SLOTS)),
                ("work", ctypes.c_double * len(PROF_SLOTS))]


class FEP3MError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fep3m status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load the library (raises if it is missing: no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1503_08509_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.fep3m_default_options.argtypes = [ctypes.POINTER(Options)]
        L.fep3m_create.argtypes = [dp, i64, ctypes.POINTER(i32), i32, ctypes.POINTER(vp)]
        L.fep3m_create_ex.argtypes = [dp, i64, ctypes.POINTER(i32), i32, ctypes.POINTER(Options), ctypes.POINTER(vp)]
        L.fep3m_create_batch.argtypes = [dp, i32, ctypes.POINTER(i64), ctypes.POINTER(i32), i32,
                                         ctypes.POINTER(Options), ctypes.POINTER(vp)]
        L.fep3m_create_static.argtypes = [dp, i64, ctypes.POINTER(i32), i32, ctypes.POINTER(Options),
                                          ctypes.POINTER(vp)]
        L.fep3m_set_stream.argtypes = [vp, vp]
        L.fep3m_potential.argtypes = [vp, vp, vp, vp]
        L.fep3m_energy.argtypes = [vp, vp, vp, vp, vp]
        L.fep3m_energy_forces.argtypes = [vp, vp, vp, vp, vp]
        L.fep3m_energy_forces_ex.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.fep3m_backward.argtypes = [vp, i64, vp, vp]
        L.fep3m_debug_stage.argtypes = [vp, i32, vp, i64]
        L.fep3m_stage_bytes.argtypes = [vp, i32]
        L.fep3m_stage_bytes.restype = i64
        L.fep3m_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.fep3m_destroy.argtypes = [vp]
        L.fep3m_destroy.restype = None
        L.fep3m_last_error.argtypes = [vp]
        L.fep3m_last_error.restype = ctypes.c_char_p
        L.fep3m_status_string.argtypes = [ctypes.c_int]
        L.fep3m_status_string.restype = ctypes.c_char_p
        L.fep3m_set_profiling.argtypes = [vp, i32]
        L.fep3m_get_profile.argtypes = [vp, ctypes.POINTER(Profile)]
        L.fep3m_host_tables.argtypes = [i32, i32, i32, i32, ctypes.POINTER(dp), i64]
        _lib = L
    return _lib


def default_options():
    o = Options()
    lib().fep3m_default_options(ctypes.byref(o))
    return o


SUPPORT_ONE, SUPPORT_27 = 0, 1
BOUNDARY_PERIODIC, BOUNDARY_GROUNDED, BOUNDARY_INSULATED = 0, 1, 2
_SUPPORTS = {"one": SUPPORT_ONE, "27": SUPPORT_27, SUPPORT_ONE: SUPPORT_ONE, SUPPORT_27: SUPPORT_27}


def host_tables(q=3, n_sr=3, box=None, support="one"):
    """Near-field tables from the library's create-time precompute (host):
    shape (nl^3, (2 n_sr + 1)^3, (q + 3)^3), nl moments per axis."""
    box = 2 * n_sr + 9 if box is None else box
    sup = _SUPPORTS[support]
    p = q + 2
    nl = q + 1 if sup == SUPPORT_27 else q - 1
    S = 2 * n_sr + 1
    out = np.zeros(nl**3 * S**3 * (p + 1) ** 3)
    st = lib().fep3m_host_tables(q, sup, n_sr, box, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size)
    if st != OK:
        raise FEP3MError(st, lib().fep3m_status_string(st).decode())
    return out.reshape(nl**3, S**3, (p + 1) ** 3)


class Context:
    """FE-P3M on n^3 elements of the periodic cube of side L, screen degree q.

    N is the number of charges, or a sequence of counts for a batch of
    independent configurations evaluated together (arrays then concatenate
    the configurations in order, and energies come back one per
    configuration)."""

    def __init__(self, L, N, n, q=3, static=False, **opts):
        """static=True: fep3m_create_static (one configuration; device buffers
        in the library's static storage, nothing allocated)."""
        import torch  # device memory and streams only

        self._torch = torch
        o = default_options()
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        dims = (ctypes.c_int32 * 3)(n, n, n)
        h = ctypes.c_void_p()
        self.batch = not np.isscalar(N)
        counts = [int(v) for v in N] if self.batch else [int(N)]
        if static and self.batch:
            raise ValueError("static contexts hold one configuration")
        if static:
            st = lib().fep3m_create_static(float(L), counts[0], dims, int(q), ctypes.byref(o), ctypes.byref(h))
        elif self.batch:
            arr = (ctypes.c_int64 * len(counts))(*counts)
            st = lib().fep3m_create_batch(float(L), len(counts), arr, dims, int(q), ctypes.byref(o), ctypes.byref(h))
        else:
            st = lib().fep3m_create_ex(float(L), counts[0], dims, int(q), ctypes.byref(o), ctypes.byref(h))
        if st != OK:
            raise FEP3MError(st, lib().fep3m_last_error(None).decode() or lib().fep3m_status_string(st).decode())
        self._h = h
        self.counts = counts
        self.offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        self.nconf = len(counts)
        self.L, self.N, self.n, self.q = float(L), int(sum(counts)), int(n), int(q)
        self.options = o

    def _check(self, st):
        if st != OK:
            msg = lib().fep3m_last_error(self._h).decode() or lib().fep3m_status_string(st).decode()
            raise FEP3MError(st, msg)

    def _prep(self, x, Q):
        t = self._torch
        if not (isinstance(x, t.Tensor) and isinstance(Q, t.Tensor)):
            raise TypeError("x and Q must be torch tensors on the GPU")
        if x.device.type != "cuda" or Q.device.type != "cuda":
            raise ValueError("x and Q must be device tensors")
        if x.dtype != t.float64 or Q.dtype != t.float64:
            raise TypeError("x and Q must be float64")
        if tuple(x.shape) != (self.N, 3) or tuple(Q.shape) != (self.N,):
            raise ValueError(f"expected x [{self.N}, 3] and Q [{self.N}]")
        x = x.contiguous()
        Q = Q.contiguous()
        self._check(lib().fep3m_set_stream(self._h, ctypes.c_void_p(t.cuda.current_stream(x.device).cuda_stream)))
        return x, Q

    def potential(self, x, Q):
        x, Q = self._prep(x, Q)
        Phi = self._torch.empty(self.N, dtype=self._torch.float64, device=x.device)
        self._check(lib().fep3m_potential(self._h, x.data_ptr(), Q.data_ptr(), Phi.data_ptr()))
        return Phi

    def energy(self, x, Q):
        """Phi [N] and U (0-d; [nconf] for a batch)."""
        x, Q = self._prep(x, Q)
        t = self._torch
        Phi = t.empty(self.N, dtype=t.float64, device=x.device)
        U = t.empty(self.nconf, dtype=t.float64, device=x.device)
        self._check(lib().fep3m_energy(self._h, x.data_ptr(), Q.data_ptr(), Phi.data_ptr(), U.data_ptr()))
        return Phi, (U if self.batch else U[0])

    def energy_forces(self, x, Q, dUdQ=False, Phi=False):
        """U (0-d; [nconf] for a batch), F [N,3] = -dU/dx and optionally
        dU/dQ [N] and Phi [N]."""
        x, Q = self._prep(x, Q)
        t = self._torch
        U = t.empty(self.nconf, dtype=t.float64, device=x.device)
        F = t.empty((self.N, 3), dtype=t.float64, device=x.device)
        g = t.empty(self.N, dtype=t.float64, device=x.device) if dUdQ else None
        P = t.empty(self.N, dtype=t.float64, device=x.device) if Phi else None
        self._check(lib().fep3m_energy_forces_ex(self._h, x.data_ptr(), Q.data_ptr(),
                                                 P.data_ptr() if P is not None else None, U.data_ptr(),
                                                 F.data_ptr(), g.data_ptr() if g is not None else None))
        out = {"U": U if self.batch else U[0], "F": F}
        if dUdQ:
            out["dUdQ"] = g
        if Phi:
            out["Phi"] = P
        return out

    def backward(self, generation, F=True, dUdQ=True, device="cuda"):
        """F = -dU/dx and dU/dQ of forward call `generation` (the value of
        stats()["generation"] right after it), from the state that call left
        in the context; the near-pair gradients are recomputed."""
        t = self._torch
        self._check(lib().fep3m_set_stream(self._h, ctypes.c_void_p(t.cuda.current_stream(device).cuda_stream)))
        Fo = t.empty((self.N, 3), dtype=t.float64, device=device) if F else None
        g = t.empty(self.N, dtype=t.float64, device=device) if dUdQ else None
        self._check(lib().fep3m_backward(self._h, int(generation), Fo.data_ptr() if Fo is not None else None,
                                         g.data_ptr() if g is not None else None))
        return Fo, g

    def stage(self, name, device="cuda"):
        t = self._torch
        sid = STAGES[name]
        nbytes = lib().fep3m_stage_bytes(self._h, sid)
        dtype = t.int32 if name in ("perm", "start") else t.float64
        out = t.empty(nbytes // (4 if dtype == t.int32 else 8), dtype=dtype, device=device)
        self._check(lib().fep3m_debug_stage(self._h, sid, out.data_ptr(), nbytes))
        return out

    def stats(self):
        s = Stats()
        self._check(lib().fep3m_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def set_profiling(self, on=True):
        self._check(lib().fep3m_set_profiling(self._h, 1 if on else 0))

    def profile(self):
        p = Profile()
        self._check(lib().fep3m_get_profile(self._h, ctypes.byref(p)))
        return {name: {"ms": p.ms[i], "count": p.count[i], "work": p.work[i]} for i, name in enumerate(PROF_SLOTS)}

    def close(self):
        if getattr(self, "_h", None):
            lib().fep3m_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _energy_function():
    import torch

    class FEP3MEnergy(torch.autograd.Function):
        """U = FEP3MEnergy.apply(x, Q, ctx): the method's energy as a 0-d
        float64 tensor (one entry per configuration of a batch context),
        differentiable in x [N, 3] and Q [N].  The backward
        pass is the library's hand-written adjoint (fep3m_backward): it
        reuses the forward call's bins and mesh potential, recomputes the
        near-pair terms, and returns grad_x = -F * dL/dU, grad_Q = dU/dQ *
        dL/dU.  The context must not evaluate another configuration between
        the forward call and its backward (an error is raised if it did)."""

        @staticmethod
        def forward(fctx, x, Q, ctx):
            _, U = ctx.energy(x.detach(), Q.detach())
            fctx.ctx = ctx
            fctx.generation = ctx.stats()["generation"]
            fctx.device = x.device
            return U

        @staticmethod
        def backward(fctx, gU):
            need_x, need_Q = fctx.needs_input_grad[0], fctx.needs_input_grad[1]
            if not (need_x or need_Q):
                return None, None, None
            ctx = fctx.ctx
            F, g = ctx.backward(fctx.generation, F=need_x, dUdQ=need_Q, device=fctx.device)
            if ctx.batch:   # dL/dU_b applies to the charges of configuration b
                gU = gU.repeat_interleave(torch.tensor(ctx.counts, device=gU.device))
            gx = -F * (gU[:, None] if ctx.batch else gU) if need_x else None
            gQ = g * gU if need_Q else None
            return gx, gQ, None

    return FEP3MEnergy


def __getattr__(name):
    if name == "FEP3MEnergy":
        fn = _energy_function()
        globals()["FEP3MEnergy"] = fn
        return fn
    raise AttributeError(name)
