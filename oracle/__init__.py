"""ctypes wrapper of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  The product path never imports it.
The oracle shares no code with the HIP path; arrays are numpy float64 in the
``[n][n][n]`` vertex layout (z fastest) with the Dirichlet boundary at 0.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlsgd_oracle.so")

OR_MAX_LEVELS = 8
SOLVE_AUTO, SOLVE_CG, SOLVE_MGPCG, SOLVE_DENSE = 0, 1, 2, 3


class OrProblem(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int),
        ("n", ctypes.c_int * OR_MAX_LEVELS),
        ("seed", ctypes.c_uint64),
        ("K", ctypes.c_int),
        ("sigma2", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("method", ctypes.c_int),
        ("rtol", ctypes.c_double),
        ("maxit", ctypes.c_int),
        ("nthreads", ctypes.c_int),
        ("common_xi", ctypes.c_int),
        ("law", ctypes.c_int),
        ("rho", ctypes.c_double),
    ]


class OrStats(ctypes.Structure):
    _fields_ = [
        ("s", ctypes.c_double),
        ("EY_shifted", ctypes.c_double),
        ("J", ctypes.c_double),
        ("truncated", ctypes.c_int),
        ("max_relres", ctypes.c_double),
        ("max_iters", ctypes.c_int),
        ("mean_dY", ctypes.c_double * OR_MAX_LEVELS),
        ("norm2_mean_dX", ctypes.c_double * OR_MAX_LEVELS),
        ("m2_dX", ctypes.c_double * OR_MAX_LEVELS),
        ("m2_dY", ctypes.c_double * OR_MAX_LEVELS),
        ("mean_phi_f", ctypes.c_double * OR_MAX_LEVELS),
        ("norm2_EX", ctypes.c_double),
    ]

    def as_dict(self, L):
        return {
            "s": self.s, "EY_shifted": self.EY_shifted, "J": self.J,
            "truncated": self.truncated, "max_relres": self.max_relres,
            "max_iters": self.max_iters,
            "mean_dY": list(self.mean_dY)[:L],
            "norm2_mean_dX": list(self.norm2_mean_dX)[:L],
            "m2_dX": list(self.m2_dX)[:L], "m2_dY": list(self.m2_dY)[:L],
            "mean_phi_f": list(self.mean_phi_f)[:L],
            "norm2_EX": self.norm2_EX,
        }


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        d, i64, u64 = ctypes.c_double, ctypes.c_int64, ctypes.c_uint64
        L.or_philox4x64_10.argtypes = [P(u64), P(u64), P(u64)]
        L.or_philox_words.argtypes = [u64, ctypes.c_int, i64, ctypes.c_int, ctypes.c_int, P(u64)]
        L.or_normals.argtypes = [u64, ctypes.c_int, i64, ctypes.c_int, ctypes.c_int, P(d)]
        L.or_kl_coeffs.argtypes = [u64, ctypes.c_int, i64, ctypes.c_int, d, P(d)]
        L.or_draws.argtypes = [u64, ctypes.c_int, i64, ctypes.c_int, ctypes.c_int, P(d)]
        L.or_kl_coeffs_law.argtypes = [u64, ctypes.c_int, i64, ctypes.c_int, d, ctypes.c_int, d,
                                       P(d)]
        L.or_log_coeff.argtypes = [ctypes.c_int, ctypes.c_int, P(d), P(d)]
        L.or_apply.argtypes = [ctypes.c_int, ctypes.c_int, P(d), P(d), P(d)]
        L.or_assemble_dense.argtypes = [ctypes.c_int, ctypes.c_int, P(d), P(d)]
        L.or_solve.argtypes = [ctypes.c_int, ctypes.c_int, P(d), P(d), P(d), ctypes.c_int,
                               d, ctypes.c_int, P(d)]
        L.or_solve.restype = ctypes.c_int
        L.or_restrict.argtypes = [ctypes.c_int, P(d), P(d)]
        L.or_prolong.argtypes = [ctypes.c_int, P(d), P(d)]
        L.or_misfit.argtypes = [ctypes.c_int, P(d), P(d)]
        L.or_misfit.restype = d
        L.or_mlmc_gradient.argtypes = [P(OrProblem), P(d), P(d), P(d), P(i64), P(i64), P(d),
                                       P(OrStats)]
        L.or_mlmc_gradient.restype = ctypes.c_int
        L.or_mlmc_objective.argtypes = [P(OrProblem), P(d), P(d), P(d), P(i64), P(i64), P(d),
                                        P(OrStats)]
        L.or_mlmc_objective.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def philox4x64_10(ctr, key):
    c = (ctypes.c_uint64 * 4)(*[int(x) for x in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(x) for x in key])
    o = (ctypes.c_uint64 * 4)()
    lib().or_philox4x64_10(c, k, o)
    return np.array(list(o), dtype=np.uint64)


def philox_words(seed, level, sample, tag, nblocks):
    out = np.zeros(4 * nblocks, dtype=np.uint64)
    lib().or_philox_words(seed, level, sample, tag, nblocks,
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


def normals(seed, level, sample, tag, count):
    out = np.zeros(count)
    lib().or_normals(seed, level, sample, tag, count, _dp(out))
    return out


LAW_ALGEBRAIC, LAW_EXPONENTIAL = 0, 1


def kl_coeffs(seed, level, sample, K, sigma2=1.0, law=LAW_ALGEBRAIC, rho=0.15):
    out = np.zeros(K ** 3)
    lib().or_kl_coeffs_law(seed, level, sample, K, sigma2, law, rho, _dp(out))
    return out


def draws(seed, level, sample, K, law=LAW_ALGEBRAIC):
    """The K^3 draws xi of one sample in draw order under the given law."""
    out = np.zeros(K ** 3)
    lib().or_draws(seed, level, sample, K, law, _dp(out))
    return out


def log_coeff(n, c):
    c = _f64(c)
    K = round(len(c) ** (1.0 / 3.0))
    out = np.zeros((n, n, n))
    lib().or_log_coeff(n, K, _dp(c), _dp(out))
    return out


def apply(n, c, y):
    c, y = _f64(c), _f64(y)
    K = round(len(c) ** (1.0 / 3.0))
    out = np.zeros((n, n, n))
    lib().or_apply(n, K, _dp(c), _dp(y), _dp(out))
    return out


def assemble_dense(n, c):
    c = _f64(c)
    K = round(len(c) ** (1.0 / 3.0))
    m = (n - 2) ** 3
    out = np.zeros((m, m))
    lib().or_assemble_dense(n, K, _dp(c), _dp(out))
    return out


def solve(n, c, b, method=SOLVE_AUTO, rtol=1e-13, maxit=2000):
    c, b = _f64(c), _f64(b)
    K = round(len(c) ** (1.0 / 3.0))
    x = np.zeros((n, n, n))
    rr = ctypes.c_double(0.0)
    it = lib().or_solve(n, K, _dp(c), _dp(b), _dp(x), method, rtol, maxit, ctypes.byref(rr))
    return x, it, rr.value


def restrict(nf, fine):
    fine = _f64(fine)
    nc = (nf - 1) // 2 + 1
    out = np.zeros((nc, nc, nc))
    lib().or_restrict(nf, _dp(fine), _dp(out))
    return out


def prolong(nc, coarse):
    coarse = _f64(coarse)
    nf = 2 * (nc - 1) + 1
    out = np.zeros((nf, nf, nf))
    lib().or_prolong(nc, _dp(coarse), _dp(out))
    return out


def misfit(n, y, yd):
    return lib().or_misfit(n, _dp(_f64(y)), _dp(_f64(yd)))


def make_problem(grid_n, seed=0, K=4, sigma2=1.0, theta=1.0, alpha=1e-3,
                 method=SOLVE_AUTO, rtol=1e-13, maxit=2000, nthreads=None,
                 common_xi=False, law=LAW_ALGEBRAIC, rho=0.15):
    pb = OrProblem()
    pb.L = len(grid_n)
    for i, n in enumerate(grid_n):
        pb.n[i] = n
    pb.seed = seed
    pb.K = K
    pb.sigma2 = sigma2
    pb.theta = theta
    pb.alpha = alpha
    pb.method = method
    pb.rtol = rtol
    pb.maxit = maxit
    pb.nthreads = nthreads if nthreads else min(16, os.cpu_count() or 1)
    pb.common_xi = 1 if common_xi else 0
    pb.law = law
    pb.rho = rho
    return pb


def mlmc_gradient(pb, f, u, yd, M, first=None):
    L = pb.L
    nL = pb.n[L - 1]
    u, yd = _f64(u), _f64(yd)
    f = _f64(f) if f is not None else np.zeros_like(u)
    Ma = np.ascontiguousarray(M, dtype=np.int64)
    Fa = np.ascontiguousarray(first if first is not None else np.zeros(L), dtype=np.int64)
    g = np.zeros((nL, nL, nL))
    st = OrStats()
    rc = lib().or_mlmc_gradient(ctypes.byref(pb), _dp(f), _dp(u), _dp(yd),
                                Ma.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                Fa.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                _dp(g), ctypes.byref(st))
    if rc != 0:
        raise ValueError("oracle rejected the problem (rc=%d)" % rc)
    return g, st.as_dict(L)


def mlmc_objective(pb, f, u, yd, M, first=None):
    L = pb.L
    u, yd = _f64(u), _f64(yd)
    f = _f64(f) if f is not None else np.zeros_like(u)
    Ma = np.ascontiguousarray(M, dtype=np.int64)
    Fa = np.ascontiguousarray(first if first is not None else np.zeros(L), dtype=np.int64)
    J = ctypes.c_double(0.0)
    st = OrStats()
    rc = lib().or_mlmc_objective(ctypes.byref(pb), _dp(f), _dp(u), _dp(yd),
                                 Ma.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 Fa.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 ctypes.byref(J), ctypes.byref(st))
    if rc != 0:
        raise ValueError("oracle rejected the problem (rc=%d)" % rc)
    return J.value, st.as_dict(L)


def sgd(pb, f, u0, yd, M, steps, tau, first=None):
    """Projected SGD u_{k+1} = u_k - tau_k g_k with fresh samples each step
    (Sec. 2.2, projection = identity).  ``tau`` is a float or a callable of k.
    Per-level running offsets advance by M after each step."""
    L = pb.L
    off = np.zeros(L, dtype=np.int64) if first is None else np.array(first, dtype=np.int64)
    u = np.array(u0, dtype=np.float64, copy=True)
    hist = []
    for k in range(steps):
        g, st = mlmc_gradient(pb, f, u, yd, M, off)
        t = tau(k) if callable(tau) else tau
        u = u - t * g
        off = off + np.asarray(M, dtype=np.int64)
        hist.append({"J": st["J"], "gnorm2": float(np.sum(g * g)) / (pb.n[L - 1] - 1) ** 3})
    return u, hist
