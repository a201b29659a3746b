"""Python binding of libmlsgd: MLMC entropic-risk gradients on AMD MI355X.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libmlsgd.so``.  Device memory comes from PyTorch (ROCm) tensors
whose data pointers are handed to the C ABI declared in ``include/mlsgd.h``.
There is no CPU fallback: if the library is missing this module raises.
"""
import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlsgd.so")

MLSGD_OK, MLSGD_EINVAL, MLSGD_ENOCONV, MLSGD_ENONFINITE, MLSGD_EHIP, MLSGD_EOOM = 0, -1, -2, -3, -4, -5
MAX_LEVELS = 8
MAX_K = 5
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
SOLVER_CG, SOLVER_MGPCG = 0, 1

EXPORTS = [
    "mlsgd_create", "mlsgd_destroy", "mlsgd_last_error", "mlsgd_sample_fields",
    "mlsgd_philox_words", "mlsgd_solve_state_adjoint", "mlsgd_solve_sizes", "mlsgd_mlmc_gradient",
    "mlsgd_mlmc_objective", "mlsgd_set_batch", "mlsgd_step", "mlsgd_kernel_timing",
    "mlsgd_get_tuning", "mlsgd_set_tuning", "mlsgd_set_graph", "mlsgd_solve_state_adjoint_noalloc",
    "mlsgd_dense_coarse_inverse",
]
SMOOTHER_RBGS, SMOOTHER_RBGS_FUSED, SMOOTHER_CHEBYSHEV = 0, 1, 2
ADAPT_BATCH, ADAPT_STEP = 1, 2
LAW_ALGEBRAIC, LAW_EXPONENTIAL = 0, 1
TUNING_FILE = os.path.join(HERE, "tuning.json")


class MlsgdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mlsgd error {code}: {msg}")
        self.code = code


class NotConverged(MlsgdError):
    pass


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_levels", ctypes.c_int32),
        ("grid_n", ctypes.c_int32 * MAX_LEVELS),
        ("seed", ctypes.c_uint64),
        ("kl_K", ctypes.c_int32),
        ("kl_sigma2", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("solver", ctypes.c_int32),
        ("rtol", ctypes.c_double),
        ("max_iters", ctypes.c_int32),
        ("u_lo", ctypes.c_double),
        ("u_hi", ctypes.c_double),
        ("f", ctypes.c_void_p),
        ("y_d", ctypes.c_void_p),
        ("kl_law", ctypes.c_int32),
        ("kl_rho", ctypes.c_double),
    ]


class _SolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("nonconverged", ctypes.c_int32),
                ("max_relres", ctypes.c_double)]


_D8 = ctypes.c_double * MAX_LEVELS


class _GradStats(ctypes.Structure):
    _fields_ = [
        ("s", ctypes.c_double), ("EY_shifted", ctypes.c_double), ("J", ctypes.c_double),
        ("truncated", ctypes.c_int32), ("iters_state", ctypes.c_int32),
        ("iters_adjoint", ctypes.c_int32), ("nonconverged", ctypes.c_int32),
        ("max_relres", ctypes.c_double),
        ("mean_dY", _D8), ("norm2_mean_dX", _D8), ("m2_dX", _D8), ("m2_dY", _D8),
        ("mean_phi_f", _D8),
        ("grad_norm", ctypes.c_double), ("norm2_EX", ctypes.c_double),
        ("ms_solve", ctypes.c_double), ("ms_total", ctypes.c_double),
        ("work_per_sample", _D8),
    ]

    def as_dict(self, L):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v)[:L] if isinstance(v, ctypes.Array) else v
        return d


class _Tuning(ctypes.Structure):
    _fields_ = [("smoother", ctypes.c_int32), ("sweeps", ctypes.c_int32), ("omega", ctypes.c_double),
                ("cheb_lo", ctypes.c_double), ("tile_y", ctypes.c_int32), ("xchunk", ctypes.c_int32),
                ("cache", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class _StepStats(ctypes.Structure):
    _fields_ = [("grad", _GradStats), ("M_next", ctypes.c_int64 * MAX_LEVELS),
                ("offset", ctypes.c_int64 * MAX_LEVELS), ("err_sam", ctypes.c_double),
                ("err_num", ctypes.c_double), ("eps", ctypes.c_double),
                ("tau", ctypes.c_double)]


_lib = None


def lib():
    """Load libmlsgd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2606_09291_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    P, vp = ctypes.POINTER, ctypes.c_void_p
    i64, i32 = ctypes.c_int64, ctypes.c_int
    L.mlsgd_create.argtypes = [P(vp), P(_Problem), vp]
    L.mlsgd_destroy.argtypes = [vp]
    L.mlsgd_last_error.argtypes = [vp]
    L.mlsgd_last_error.restype = ctypes.c_char_p
    L.mlsgd_sample_fields.argtypes = [vp, i32, i64, i64, vp]
    L.mlsgd_philox_words.argtypes = [ctypes.c_uint64, i32, i64, i32, i32, vp, vp]
    L.mlsgd_solve_state_adjoint.argtypes = [vp, i32, i32, i64, i64, vp, vp, vp, vp,
                                            P(_SolveStats)]
    L.mlsgd_solve_state_adjoint_noalloc.argtypes = [vp, i32, i32, i64, i64, vp, vp, vp, vp,
                                                    P(_SolveStats), P(i64)]
    L.mlsgd_dense_coarse_inverse.argtypes = [vp, i32, i32, i64, i32, vp]
    L.mlsgd_solve_sizes.argtypes = [vp, i32, P(i32), i32, i64, ctypes.c_double, vp,
                                    P(_SolveStats)]
    L.mlsgd_mlmc_gradient.argtypes = [vp, vp, i32, P(i64), P(i64), vp, P(_GradStats)]
    L.mlsgd_mlmc_objective.argtypes = [vp, vp, i32, P(i64), P(i64), P(ctypes.c_double),
                                       P(_GradStats)]
    L.mlsgd_set_batch.argtypes = [vp, i32, P(i64), P(i64)]
    L.mlsgd_step.argtypes = [vp, vp, ctypes.c_double, i32, P(_StepStats)]
    L.mlsgd_kernel_timing.argtypes = [vp, i32, i32, P(ctypes.c_double), P(i64),
                                      P(ctypes.c_double)]
    L.mlsgd_get_tuning.argtypes = [vp, P(_Tuning)]
    L.mlsgd_set_graph.argtypes = [vp, i32]
    L.mlsgd_set_tuning.argtypes = [vp, P(_Tuning)]
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


def _torch():
    import torch
    return torch


def _dev_f64(x, device):
    torch = _torch()
    t = torch.as_tensor(x, dtype=torch.float64, device=device)
    return t.contiguous()


def _i64_array(vals, n):
    arr = (ctypes.c_int64 * max(n, 1))()
    for i, v in enumerate(vals):
        arr[i] = int(v)
    return arr


@dataclass
class Problem:
    """Problem data of the entropic-risk control problem (see include/mlsgd.h)."""
    grid_n: Sequence[int]
    y_d: object                      # finest-grid target (array-like, n^3)
    f: Optional[object] = None       # finest-grid source (array-like), None = 0
    seed: int = 0
    K: int = 4
    sigma2: float = 1.0
    theta: float = 1.0
    alpha: float = 1e-3
    precision: int = FP64
    solver: int = SOLVER_MGPCG
    rtol: float = 1e-12
    max_iters: int = 500
    u_lo: float = 1.0
    u_hi: float = -1.0               # u_lo > u_hi: no box constraint
    law: int = 0                     # LAW_ALGEBRAIC or LAW_EXPONENTIAL (Sec. 5)
    rho: float = 0.15                # correlation length of LAW_EXPONENTIAL
    extra: dict = field(default_factory=dict)


class Context:
    """One libmlsgd context bound to a CUDA (HIP) device and stream."""

    def __init__(self, problem: Problem, device="cuda:0", stream=None, use_tuned=True):
        torch = _torch()
        self.lib = lib()
        self.device = torch.device(device)
        self.problem = problem
        self.L = len(problem.grid_n)
        self.nfin = problem.grid_n[-1]
        self.K = problem.K
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._yd = _dev_f64(problem.y_d, self.device).reshape(-1)
        self._f = _dev_f64(problem.f, self.device).reshape(-1) if problem.f is not None else None
        pb = _Problem()
        pb.n_levels = self.L
        for i, n in enumerate(problem.grid_n):
            pb.grid_n[i] = int(n)
        pb.seed = int(problem.seed)
        pb.kl_K = int(problem.K)
        pb.kl_sigma2 = float(problem.sigma2)
        pb.theta = float(problem.theta)
        pb.alpha = float(problem.alpha)
        pb.precision = int(problem.precision)
        pb.solver = int(problem.solver)
        pb.rtol = float(problem.rtol)
        pb.max_iters = int(problem.max_iters)
        pb.u_lo = float(problem.u_lo)
        pb.u_hi = float(problem.u_hi)
        pb.kl_law = int(problem.law)
        pb.kl_rho = float(problem.rho)
        pb.f = self._f.data_ptr() if self._f is not None else None
        pb.y_d = self._yd.data_ptr()
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.mlsgd_create(ctypes.byref(h), ctypes.byref(pb),
                                       ctypes.c_void_p(self.stream.cuda_stream))
        if rc != MLSGD_OK:
            raise MlsgdError(rc, "mlsgd_create failed (invalid problem or HIP error)")
        self._h = h
        if use_tuned:
            t = tuned_for(self.problem)
            if t is not None:
                self.set_tuning(**t)

    def close(self):
        if getattr(self, "_h", None):
            self.lib.mlsgd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_noconv=False):
        if rc == MLSGD_OK:
            return
        msg = self.lib.mlsgd_last_error(self._h).decode()
        if rc == MLSGD_ENOCONV:
            if allow_noconv:
                return
            raise NotConverged(rc, msg)
        raise MlsgdError(rc, msg)

    def _u(self, u):
        t = _dev_f64(u, self.device).reshape(-1)
        if t.numel() != self.nfin ** 3:
            raise ValueError(f"u must have {self.nfin}^3 entries")
        return t

    def sample_fields(self, level, first, count):
        torch = _torch()
        out = torch.empty((max(count, 0), self.K ** 3), dtype=torch.float64, device=self.device)
        rc = self.lib.mlsgd_sample_fields(self._h, level, first, count,
                                          ctypes.c_void_p(out.data_ptr() if count > 0 else 0))
        self._check(rc)
        return out

    def solve_state_adjoint(self, level, coarse, first, count, u, want_y=True, want_p=True,
                            allow_noconv=False):
        torch = _torch()
        n = self.problem.grid_n[level - coarse]
        uu = self._u(u)
        y = torch.empty((count, n, n, n), dtype=torch.float64, device=self.device) if want_y else None
        p = torch.empty((count, n, n, n), dtype=torch.float64, device=self.device) if want_p else None
        phi = torch.empty((count,), dtype=torch.float64, device=self.device)
        st = _SolveStats()
        rc = self.lib.mlsgd_solve_state_adjoint(
            self._h, level, coarse, first, count, ctypes.c_void_p(uu.data_ptr()),
            ctypes.c_void_p(y.data_ptr() if y is not None else 0),
            ctypes.c_void_p(p.data_ptr() if p is not None else 0),
            ctypes.c_void_p(phi.data_ptr()), ctypes.byref(st))
        self._check(rc, allow_noconv)
        stats = {"iterations": st.iterations, "nonconverged": st.nonconverged,
                 "max_relres": st.max_relres}
        return y, p, phi, stats

    def solve_state_adjoint_noalloc(self, level, coarse, first, count, u, y, p, phi,
                                    allow_noconv=False):
        """mlsgd_solve_state_adjoint_noalloc on caller-allocated outputs (device
        float64 tensors: y and p of count*n^3 or None, phi of count or None).
        Returns (stats, scratch bytes the batch needs)."""
        uu = self._u(u)
        st = _SolveStats()
        need = ctypes.c_int64(0)
        rc = self.lib.mlsgd_solve_state_adjoint_noalloc(
            self._h, level, coarse, first, count, ctypes.c_void_p(uu.data_ptr()),
            ctypes.c_void_p(y.data_ptr() if y is not None else 0),
            ctypes.c_void_p(p.data_ptr() if p is not None else 0),
            ctypes.c_void_p(phi.data_ptr() if phi is not None else 0), ctypes.byref(st),
            ctypes.byref(need))
        self._check(rc, allow_noconv)
        return ({"iterations": st.iterations, "nonconverged": st.nonconverged,
                 "max_relres": st.max_relres}, need.value)

    def solve_sizes(self, n_list, level=6, first=0, f_value=1.0, want_y=True,
                    allow_noconv=False):
        """Independent state solves on grids of the given sizes (mlsgd_solve_sizes).
        Returns (list of n^3 solution tensors or None, stats)."""
        torch = _torch()
        ns = [int(n) for n in n_list]
        arr = (ctypes.c_int32 * len(ns))(*ns)
        tot = sum(n ** 3 for n in ns)
        y = torch.empty((tot,), dtype=torch.float64, device=self.device) if want_y else None
        st = _SolveStats()
        rc = self.lib.mlsgd_solve_sizes(self._h, len(ns), arr, level, first, float(f_value),
                                        ctypes.c_void_p(y.data_ptr() if y is not None else 0),
                                        ctypes.byref(st))
        self._check(rc, allow_noconv)
        stats = {"iterations": st.iterations, "nonconverged": st.nonconverged,
                 "max_relres": st.max_relres}
        if y is None:
            return None, stats
        out, o = [], 0
        for n in ns:
            out.append(y[o:o + n ** 3].view(n, n, n))
            o += n ** 3
        return out, stats

    def dense_coarse_inverse(self, n, level, first, count):
        """Inverses of the rediscretised n^3 operators of the given draws
        (mlsgd_dense_coarse_inverse), as a (count, N, N) float64 tensor."""
        torch = _torch()
        N = (n - 2) ** 3
        out = torch.empty((count, N, N), dtype=torch.float64, device=self.device)
        self._check(self.lib.mlsgd_dense_coarse_inverse(self._h, int(n), int(level), int(first),
                                                        int(count),
                                                        ctypes.c_void_p(out.data_ptr())))
        return out

    def set_graph(self, enable=True):
        """Run estimates as replayed HIP graphs (mlsgd_set_graph)."""
        self._check(self.lib.mlsgd_set_graph(self._h, 1 if enable else 0))

    def mlmc_gradient(self, u, M, first=None, out=None, allow_noconv=False):
        torch = _torch()
        L = len(M)
        uu = self._u(u)
        g = out if out is not None else torch.empty((self.nfin,) * 3, dtype=torch.float64,
                                                     device=self.device)
        st = _GradStats()
        Ma = _i64_array(M, L)
        Fa = _i64_array(first, L) if first is not None else None
        rc = self.lib.mlsgd_mlmc_gradient(self._h, ctypes.c_void_p(uu.data_ptr()), L, Ma, Fa,
                                          ctypes.c_void_p(g.data_ptr()), ctypes.byref(st))
        self._check(rc, allow_noconv)
        return g, st.as_dict(L)

    def mlmc_objective(self, u, M, first=None, allow_noconv=False):
        L = len(M)
        uu = self._u(u)
        st = _GradStats()
        J = ctypes.c_double(0.0)
        Ma = _i64_array(M, L)
        Fa = _i64_array(first, L) if first is not None else None
        rc = self.lib.mlsgd_mlmc_objective(self._h, ctypes.c_void_p(uu.data_ptr()), L, Ma, Fa,
                                           ctypes.byref(J), ctypes.byref(st))
        self._check(rc, allow_noconv)
        return J.value, st.as_dict(L)

    def set_batch(self, M, offsets=None):
        L = len(M)
        rc = self.lib.mlsgd_set_batch(self._h, L, _i64_array(M, L),
                                      _i64_array(offsets, L) if offsets is not None else None)
        self._check(rc)

    def step(self, u, tau, adapt=False, adapt_step=False, allow_noconv=False):
        """In-place projected SGD step on the device tensor u (float64, n^3).
        adapt: adaptive batch controller; adapt_step: adaptive step size (tau is
        then the first step and the fallback)."""
        if not (u.is_cuda and u.dtype == _torch().float64 and u.is_contiguous()):
            raise ValueError("u must be a contiguous float64 device tensor")
        st = _StepStats()
        flags = (ADAPT_BATCH if adapt else 0) | (ADAPT_STEP if adapt_step else 0)
        rc = self.lib.mlsgd_step(self._h, ctypes.c_void_p(u.data_ptr()), float(tau), flags,
                                 ctypes.byref(st))
        self._check(rc, allow_noconv)
        L = self.L
        return {"grad": st.grad.as_dict(L), "M_next": list(st.M_next)[:L],
                "offset": list(st.offset)[:L], "err_sam": st.err_sam, "err_num": st.err_num,
                "eps": st.eps, "tau": st.tau}


    def get_tuning(self):
        t = _Tuning()
        self._check(self.lib.mlsgd_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        """Change solver/tile parameters (see mlsgd_tuning in include/mlsgd.h)."""
        cur = self.get_tuning()
        cur.update({k: v for k, v in kw.items() if k in cur})
        t = _Tuning(**cur)
        self._check(self.lib.mlsgd_set_tuning(self._h, ctypes.byref(t)))

    def kernel_timing(self, enable, n=0):
        """Read the smoothing-pass event totals, then (enable >= 0) reset and
        switch timing on for grid n (1) or off (0)."""
        ms = ctypes.c_double(0.0)
        cnt = ctypes.c_int64(0)
        by = ctypes.c_double(0.0)
        rc = self.lib.mlsgd_kernel_timing(self._h, int(enable), int(n), ctypes.byref(ms),
                                          ctypes.byref(cnt), ctypes.byref(by))
        self._check(rc)
        return {"ms": ms.value, "launches": cnt.value, "bytes": by.value}


def tuning_key(problem):
    """Key of the autotuner's cache: precision, solver and grid list."""
    return f"gfx950:p{int(problem.precision)}:s{int(problem.solver)}:" + "x".join(
        str(int(n)) for n in problem.grid_n)


def tuned_for(problem):
    """Tuning chosen by the autotuner for this kind of problem, if any."""
    import json
    try:
        with open(TUNING_FILE) as fh:
            table = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = table.get(tuning_key(problem))
    return entry.get("tuning") if entry else None


def philox_words(seed, level, sample, tag, nblocks, device="cuda:0"):
    """Raw Philox4x64-10 words (as int64 bit patterns) computed on the GPU."""
    torch = _torch()
    out = torch.empty((4 * nblocks,), dtype=torch.int64, device=device)
    stream = torch.cuda.current_stream(torch.device(device))
    rc = lib().mlsgd_philox_words(ctypes.c_uint64(seed), level, sample, tag, nblocks,
                                  ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(stream.cuda_stream))
    if rc != MLSGD_OK:
        raise MlsgdError(rc, "mlsgd_philox_words failed")
    return out
