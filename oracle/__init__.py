"""FP64 CPU oracle of the cross-matrix Krylov projection path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg are the
only callers.  The product path (the HIP library and its binding) never imports this package, and
this package imports nothing from the product.

The arithmetic lives in plain C (``xkp_oracle.c``, built with gcc, no contraction of multiply-add);
this module only marshals numpy arrays.  Each function names the part of the paper it follows.

Parity status: every function here is pinned by the non-GPU tests (closed-form eigenpairs, row
sums, the Cole-Hopf exact solution, brute-force least squares, dense LU, Galerkin orthogonality,
the Arnoldi relation; the verification residual by the eigenpairs, the explicit matrix and a
planted residual of known norm; the image-cycle chain by its one-block, repeated-block and
two-seed reductions), except the end-to-end agreement with the paper's own timings, which the
paper does not print at this tolerance (parity unpinned there).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xkp_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

OK, EINVAL, ENOMEM, ENOCONV, ESINGULAR = 0, 1, 2, 4, 5
TARGET_GALERKIN, SEED_GALERKIN, SEED_LSQ = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_LIB), exist_ok=True)
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Op(ct.Structure):
    _fields_ = [("H", ct.c_int), ("W", ct.c_int), ("dt", ct.c_double), ("g", ct.c_double),
                ("mt", ct.c_void_p), ("fx", ct.c_void_p), ("fy", ct.c_void_p)]


class _Info(ct.Structure):
    _fields_ = [("status", ct.c_int), ("iters", ct.c_int), ("restarts", ct.c_int),
                ("basis_dim", ct.c_int), ("res_est", ct.c_double), ("res_true", ct.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ct.CDLL(build())
        P = ct.c_void_p
        _lib.xo_coeffs.argtypes = [ct.POINTER(_Op), P, P, P, P, P]
        _lib.xo_rhs.argtypes = [ct.POINTER(_Op), P, P]
        _lib.xo_apply.argtypes = [ct.POINTER(_Op), P, P]
        _lib.xo_dense.argtypes = [ct.POINTER(_Op), P]
        _lib.xo_lu_solve.argtypes = [ct.c_int, P, P]
        _lib.xo_banded_solve.argtypes = [ct.POINTER(_Op), P, P]
        _lib.xo_residual.argtypes = [ct.POINTER(_Op), P, P]
        _lib.xo_residual.restype = ct.c_double
        gm = [ct.c_int, ct.c_int, ct.c_double, ct.c_int, ct.c_int, P, P, ct.POINTER(_Info), P,
              ct.c_int]
        _lib.xo_gmres.argtypes = [ct.POINTER(_Op), P, P] + gm
        _lib.xo_gmres_dense.argtypes = [ct.c_int, P, P, P] + gm
        _lib.xo_project.argtypes = [ct.POINTER(_Op), P, P, ct.c_int, P, P, ct.c_int, ct.c_int, P, P]
        _lib.xo_accumulate.argtypes = [ct.c_int, ct.c_int, P, P, ct.c_int, ct.c_int, P]
    return _lib


def set_mutation(code: int) -> None:
    """Plant a known mistake in the oracle (0 restores it); used only to show the pins bite."""
    ct.c_int.in_dll(lib(), "xo_mutation").value = int(code)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data


@dataclass
class Operator:
    """One linear system's operator at one timestep (Section 2.3): square grid H x H,
    dt = 1/T, diffusion g, lagged log-density m~ and optional drift components (f = 0 if None)."""
    H: int
    dt: float
    g: float
    mt: np.ndarray
    fx: np.ndarray | None = None
    fy: np.ndarray | None = None

    def __post_init__(self):
        self.mt = _f64(self.mt).reshape(-1)
        self.fx = None if self.fx is None else _f64(self.fx).reshape(-1)
        self.fy = None if self.fy is None else _f64(self.fy).reshape(-1)
        if self.mt.size != self.H * self.H:
            raise ValueError("m~ must have H*H values")
        self._s = _Op(self.H, self.H, float(self.dt), float(self.g), _p(self.mt), _p(self.fx),
                      _p(self.fy))

    @property
    def n(self) -> int:
        return self.H * self.H

    @property
    def ref(self):
        return ct.byref(self._s)


@dataclass
class GmresResult:
    x: np.ndarray
    status: int
    iters: int
    restarts: int
    basis_dim: int
    res_est: float
    res_true: float
    V: np.ndarray | None = None      # n x (k+1) first-cycle basis (columns), when requested
    Hbar: np.ndarray | None = None   # (k+1) x k first-cycle Hessenberg matrix, when requested
    hist: np.ndarray | None = None


def coeffs(A: Operator):
    """Per-row C_diag, C_east, C_west, C_north, C_south (Section 2.3)."""
    out = [np.empty(A.n) for _ in range(5)]
    lib().xo_coeffs(A.ref, *[_p(o) for o in out])
    return tuple(out)


def rhs(A: Operator, mprev) -> np.ndarray:
    """b = m^{n-1}/dt - Div f (Section 2.3)."""
    mprev = _f64(mprev).reshape(-1)
    b = np.empty(A.n)
    lib().xo_rhs(A.ref, _p(mprev), _p(b))
    return b


def apply(A: Operator, u) -> np.ndarray:
    u = _f64(u).reshape(-1)
    y = np.empty(A.n)
    lib().xo_apply(A.ref, _p(u), _p(y))
    return y


def dense(A: Operator) -> np.ndarray:
    D = np.empty((A.n, A.n))
    lib().xo_dense(A.ref, _p(D))
    return D


def lu_solve(D, b):
    """Dense LU with partial pivoting. Returns (x, status)."""
    D = _f64(D).copy()
    x = _f64(b).copy()
    st = lib().xo_lu_solve(D.shape[0], _p(D), _p(x))
    return x, st


def banded_solve(A: Operator, b):
    """Direct banded LU solve (the paper's direct-solver baseline). Returns (x, status)."""
    b = _f64(b).reshape(-1)
    x = np.zeros(A.n)
    st = lib().xo_banded_solve(A.ref, _p(b), _p(x))
    return x, st


def residual(A: Operator, b, x) -> float:
    """||b - A x||_2 / ||b||_2 (||r||_2 when b = 0)."""
    b = _f64(b).reshape(-1)
    x = _f64(x).reshape(-1)
    return lib().xo_residual(A.ref, _p(b), _p(x))


def _gmres_common(call, n, b, x0, m, max_restarts, tol, max_iters, keep_basis, hist_cap):
    b = _f64(b).reshape(-1)
    x = np.zeros(n) if x0 is None else _f64(x0).reshape(-1).copy()
    V = np.zeros((m + 1, n)) if keep_basis else None     # row c = column c of V
    Hb = np.zeros((m, m + 1)) if keep_basis else None    # row c = column c of Hbar
    hist = np.zeros(hist_cap) if hist_cap else None
    info = _Info()
    call(b, x, V, Hb, info, hist)
    k = info.basis_dim
    res = GmresResult(x, info.status, info.iters, info.restarts, k, info.res_est, info.res_true)
    if keep_basis:
        res.V = V[:k + 1].T.copy()
        res.Hbar = Hb[:k].T[:k + 1].copy()
        res._ldh = m + 1
    if hist_cap:
        res.hist = hist[:min(info.iters, hist_cap)].copy()
    return res


def gmres(A: Operator, b, x0=None, m=30, max_restarts=1000, tol=1e-8, max_iters=0,
          keep_basis=False, hist_cap=0, passes=2) -> GmresResult:
    """Restarted GMRES(m) on the stencil operator (Section 3 Krylov solve; Saad Alg. 6.9/6.11),
    with `passes` (1 or 2) modified Gram-Schmidt passes per Arnoldi step."""
    if passes not in (1, 2):
        raise ValueError("passes must be 1 or 2")

    def call(b, x, V, Hb, info, hist):
        lib().xo_gmres(A.ref, _p(b), _p(x), m, max_restarts, tol, max_iters, passes, _p(V),
                       _p(Hb), ct.byref(info), _p(hist), 0 if hist is None else hist.size)
    return _gmres_common(call, A.n, b, x0, m, max_restarts, tol, max_iters, keep_basis, hist_cap)


def gmres_dense(D, b, x0=None, m=30, max_restarts=1000, tol=1e-8, max_iters=0,
                keep_basis=False, hist_cap=0, passes=2) -> GmresResult:
    """The same GMRES(m) on an explicit dense matrix (for the brute-force pins)."""
    if passes not in (1, 2):
        raise ValueError("passes must be 1 or 2")
    D = _f64(D)
    n = D.shape[0]

    def call(b, x, V, Hb, info, hist):
        lib().xo_gmres_dense(n, _p(D), _p(b), _p(x), m, max_restarts, tol, max_iters, passes,
                             _p(V), _p(Hb), ct.byref(info), _p(hist),
                             0 if hist is None else hist.size)
    return _gmres_common(call, n, b, x0, m, max_restarts, tol, max_iters, keep_basis, hist_cap)


def project(At: Operator, b, V, Hbar, mode=TARGET_GALERKIN, x_base=None):
    """Section 3, Phase 2: x0 = x_base + V_k alpha from the seed basis.

    V is n x (k+1) (the seed's first-cycle basis), Hbar is (k+1) x k.  Returns (x0, alpha, status).
    """
    b = _f64(b).reshape(-1)
    V = np.asarray(V, dtype=np.float64)
    k = V.shape[1] - 1
    Vc = np.ascontiguousarray(V.T)                 # column c contiguous
    Hc = np.ascontiguousarray(np.asarray(Hbar, dtype=np.float64).T)  # column c contiguous, ld k+1
    xb = None if x_base is None else _f64(x_base).reshape(-1)
    x0 = np.empty(At.n)
    alpha = np.zeros(max(k, 1))
    st = lib().xo_project(At.ref, _p(b), _p(xb), k, _p(Vc), _p(Hc), k + 1, mode, _p(x0),
                          _p(alpha))
    return x0, alpha[:k], st


def accumulate(sources, per_source, cap):
    """Krylov subspace expansion over an image cycle: `sources` is a list of (n, k_s) arrays of
    orthonormal columns (the seeds' first-cycle bases V_k, in cycle order); returns the (n, kd)
    orthonormal basis gathered from them (two modified Gram-Schmidt passes per column, norm left
    > 1e-8 to append, at most per_source columns per source and cap in total)."""
    srcs = [np.asfortranarray(_f64(V)) for V in sources]
    n = srcs[0].shape[0]
    if any(V.shape[0] != n for V in srcs):
        raise ValueError("every source needs the same number of rows")
    ptrs = (ct.c_void_p * len(srcs))(*[V.ctypes.data for V in srcs])
    ks = (ct.c_int * len(srcs))(*[V.shape[1] for V in srcs])
    out = np.zeros((cap, n))                      # row c = column c
    kd = lib().xo_accumulate(n, len(srcs), ptrs, ks, int(per_source), int(cap), _p(out))
    return out[:kd].T.copy()
