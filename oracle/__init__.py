"""CPU FP64 oracle for chordal-decomposed primal ADMM -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product library: the two share only the
seeded instance generator ``sdpgen``.

The arithmetic lives in ``sdp_oracle.c`` (plain C, FP64); this module only
marshals arrays through ctypes.  See that file's header for the passages of
the paper each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OK = 0
MAX_ITER = 1
ERR_ARG = -1
ERR_PATTERN_UNCOVERED = -2
ERR_OFF_PATTERN = -3
ERR_CLIQUE_ORDER = -4
ERR_RANK_DEFICIENT = -5
ERR_NONFINITE = -6
ERR_UNSUPPORTED = -7

_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_lp = C.POINTER(C.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    lib.orc_create.argtypes = [C.c_int, C.c_int, C.c_int64, _ip, _ip, C.c_int, _ip, _ip,
                               C.c_int, _lp, _ip, _dp, _dp, _dp, C.POINTER(C.c_void_p)]
    lib.orc_create.restype = C.c_int
    lib.orc_create_ex.argtypes = lib.orc_create.argtypes[:-1] + [C.c_int, C.POINTER(C.c_void_p)]
    lib.orc_create_ex.restype = C.c_int
    lib.orc_free.argtypes = [C.c_void_p]
    lib.orc_reset.argtypes = [C.c_void_p, C.c_double]
    lib.orc_set_jacobi.argtypes = [C.c_void_p, C.c_int, C.c_double]
    lib.orc_run.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_double,
                            C.c_double, C.c_int, _ip, _dp, _dp, _dp]
    lib.orc_run.restype = C.c_int
    lib.orc_run_dual.argtypes = lib.orc_run.argtypes
    lib.orc_run_dual.restype = C.c_int
    lib.orc_set_affine_cg.argtypes = [C.c_void_p, C.c_int, C.c_double]
    lib.orc_set_affine_cg.restype = C.c_int
    lib.orc_pcg.argtypes = [C.c_void_p, _dp, _dp, C.c_int, C.c_double, _dp]
    lib.orc_pcg.restype = C.c_int
    lib.orc_cg_steps.argtypes = [C.c_void_p]
    lib.orc_cg_steps.restype = C.c_int64
    lib.orc_dual_objective.argtypes = [C.c_void_p]
    lib.orc_dual_objective.restype = C.c_double
    lib.orc_get_vd.argtypes = [C.c_void_p, _dp]
    lib.orc_set_vd.argtypes = [C.c_void_p, _dp]
    lib.orc_hsde_setup.argtypes = [C.c_void_p]
    lib.orc_hsde_setup.restype = C.c_int
    lib.orc_run_hsde.argtypes = [C.c_void_p, C.c_int, C.c_double, _ip, _dp, _dp]
    lib.orc_run_hsde.restype = C.c_int
    lib.orc_hsde_get.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_hsde_inner.argtypes = [C.c_void_p] + [_dp] * 8
    lib.orc_hsde_set.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, C.c_double, C.c_double]
    lib.orc_hsde_raw.argtypes = [C.c_void_p, _dp, _dp]
    lib.orc_jacobi_eig.argtypes = [C.c_int, _dp, _dp, _dp, C.c_int, C.c_double]
    lib.orc_jacobi_eig.restype = C.c_int
    lib.orc_psd_project.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_int, C.c_double]
    lib.orc_psd_project.restype = C.c_int
    lib.orc_cholesky.argtypes = [C.c_int, _dp, _dp]
    lib.orc_cholesky.restype = C.c_int
    lib.orc_chol_solve.argtypes = [C.c_int, _dp, _dp, _dp]
    lib.orc_form_bhat.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _dp]
    lib.orc_affine.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    for name in ("orc_get_u", "orc_get_y", "orc_get_D", "orc_get_L", "orc_next_w",
                 "orc_diagnostics"):
        getattr(lib, name).argtypes = [C.c_void_p, _dp]
    lib.orc_get_blocks.argtypes = [C.c_void_p, _dp, _dp]
    lib.orc_gather_blocks.argtypes = [C.c_void_p, _dp, _dp]
    lib.orc_set_blocks.argtypes = [C.c_void_p, _dp, _dp]
    lib.orc_set_rho.argtypes = [C.c_void_p, C.c_double]
    lib.orc_psd_project_derivative.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
    lib.orc_unrolled_vjp.argtypes = [C.c_void_p, C.c_int, C.c_double, _dp, _dp, _dp, _dp]
    lib.orc_unrolled_vjp.restype = C.c_int
    lib.orc_set_cb.argtypes = [C.c_void_p, _dp, _dp]
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_get_max_threads.restype = C.c_int
    for name, rt in (("orc_nblk", C.c_int64), ("orc_rho", C.c_double), ("orc_iters", C.c_int),
                     ("orc_eps_c", C.c_double), ("orc_eps_l", C.c_double),
                     ("orc_total_sweeps", C.c_int64), ("orc_max_sweeps_seen", C.c_int),
                     ("orc_objective", C.c_double)):
        getattr(lib, name).argtypes = [C.c_void_p]
        getattr(lib, name).restype = rt
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _l(a):
    return a.ctypes.data_as(_lp)


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


def max_threads() -> int:
    return int(_load().orc_get_max_threads())


# --------------------------------------------------------------------------
# Dense building blocks
# --------------------------------------------------------------------------

def jacobi_eig(A, max_sweeps=50, tol=1e-14):
    """Cyclic Jacobi: returns (theta, V, sweeps) with A = V diag(theta) V^T."""
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    s = A.shape[0]
    V = np.zeros((s, s))
    th = np.zeros(max(s, 1))
    sw = _load().orc_jacobi_eig(s, _d(A), _d(V), _d(th), max_sweeps, tol)
    return th[:s], V, sw


def psd_project(W, max_sweeps=50, tol=1e-14, return_eig=False):
    """Projection of a symmetric matrix onto the PSD cone (XkUpdate)."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    s = W.shape[0]
    X = np.zeros((s, s))
    th = np.zeros(max(s, 1))
    V = np.zeros((s, s))
    sw = _load().orc_psd_project(s, _d(W), _d(X), _d(th), _d(V), max_sweeps, tol)
    if return_eig:
        return X, th[:s], V, sw
    return X


def psd_project_derivative(V, theta, G):
    """Daleckii-Krein derivative of the PSD projection at V diag(theta) V^T,
    applied to the symmetric direction G (also its vector-Jacobian product)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    out = np.zeros_like(G)
    _load().orc_psd_project_derivative(V.shape[0], _d(V), _d(th), _d(G), _d(out))
    return out


def cholesky(M):
    M = np.ascontiguousarray(M, dtype=np.float64)
    m = M.shape[0]
    L = np.zeros((m, m))
    rc = _load().orc_cholesky(m, _d(M), _d(L))
    return rc, L


def chol_solve(L, r):
    L = np.ascontiguousarray(L, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    y = np.zeros_like(r)
    _load().orc_chol_solve(L.shape[0], _d(L), _d(r), _d(y))
    return y


# --------------------------------------------------------------------------
# Whole-problem oracle
# --------------------------------------------------------------------------

class HsdeResult:
    def __init__(self, status, iters, hist_e, hist_c):
        self.status, self.iters, self.hist_e, self.hist_c = status, iters, hist_e, hist_c


@dataclass
class RunResult:
    status: int
    iters: int
    eps_c: float
    eps_l: float
    rho: float
    hist_eps_c: np.ndarray
    hist_eps_l: np.ndarray
    hist_rho: np.ndarray


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


class Problem:
    """Algorithm 1 on one SDP instance (an ``sdpgen.Instance``)."""

    def __init__(self, inst, rho0: float = 1.0, factor: bool = True):
        """factor=False skips the Cholesky factor of A W D^-1 A^T (for large m):
        the problem then runs Algorithm 1 only after set_affine_cg."""
        lib = _load()
        self.inst = inst
        self._keep = []
        pr = np.ascontiguousarray(inst.pat_row, dtype=np.int32)
        pc = np.ascontiguousarray(inst.pat_col, dtype=np.int32)
        cp = np.ascontiguousarray(inst.clique_ptr, dtype=np.int32)
        cv = np.ascontiguousarray(inst.clique_vert, dtype=np.int32)
        av = np.ascontiguousarray(inst.a_val, dtype=np.float64)
        b = np.ascontiguousarray(inst.b, dtype=np.float64)
        c = np.ascontiguousarray(inst.c, dtype=np.float64)
        if inst.a_format == 1:
            ar = np.ascontiguousarray(inst.a_rowptr, dtype=np.int64)
            ac = np.ascontiguousarray(inst.a_col, dtype=np.int32)
            arp, acp = _l(ar), _i(ac)
        else:
            arp, acp = None, None
        h = C.c_void_p()
        rc = lib.orc_create_ex(int(inst.n), int(inst.m), int(pr.shape[0]), _i(pr), _i(pc),
                               int(cp.shape[0] - 1), _i(cp), _i(cv), int(inst.a_format),
                               arp, acp, _d(av), _d(b), _d(c), int(bool(factor)), C.byref(h))
        if rc != OK:
            raise OracleError(rc)
        self._h = h
        self.n, self.m, self.nnz = inst.n, inst.m, int(pr.shape[0])
        self.sizes = np.diff(cp)
        self.blk_off = np.concatenate([[0], np.cumsum(self.sizes.astype(np.int64) ** 2)])
        lib.orc_reset(h, rho0)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    # state ------------------------------------------------------------------
    def reset(self, rho0: float = 1.0):
        _load().orc_reset(self._h, rho0)

    def set_jacobi(self, max_sweeps=50, tol=1e-14):
        _load().orc_set_jacobi(self._h, max_sweeps, tol)

    def run(self, max_iter, tol=1e-4, adaptive=False, mu=2.0, nu=10.0, rho_period=1):
        """Algorithm 1 (domain-space primal ADMM)."""
        return self._run(_load().orc_run, max_iter, tol, adaptive, mu, nu, rho_period)

    def run_dual(self, max_iter, tol=1e-4, adaptive=False, mu=2.0, nu=10.0, rho_period=1):
        """Algorithm 2 (range-space dual ADMM): z_k in blocks()[0], lambda_k in
        blocks()[1], x in u(), y in y()."""
        return self._run(_load().orc_run_dual, max_iter, tol, adaptive, mu, nu, rho_period)

    def dual_objective(self):
        """b^T y of the current Algorithm 2 iterate."""
        return float(_load().orc_dual_objective(self._h))

    def v_blocks(self):
        """The slack blocks v_k of Algorithm 2 (full s_k x s_k matrices)."""
        n = int(_load().orc_nblk(self._h))
        V = np.zeros(n)
        _load().orc_get_vd(self._h, _d(V))
        return self._split(V)

    # ---- Algorithm 3 (HSDE) ----
    def hsde_setup(self):
        """Factor I + A W P^-1 A^T, form M^-1 zeta; u = v = (0, ..., 0, 1)."""
        return int(_load().orc_hsde_setup(self._h))

    def run_hsde(self, max_iter, tol=1e-4):
        """Algorithm 3; status 0 solved, 1 iteration limit, 2 primal
        infeasible, 3 dual infeasible; hist_e = max(eps_p, eps_d, eps_g),
        hist_c = eps_c per iteration."""
        lib = _load()
        he = np.zeros(max(max_iter, 1))
        hc = np.zeros(max(max_iter, 1))
        it = C.c_int(0)
        st = lib.orc_run_hsde(self._h, int(max_iter), float(tol), C.byref(it), _d(he), _d(hc))
        k = it.value
        return HsdeResult(st, k, he[:k], hc[:k])

    def hsde_solution(self):
        n = int(_load().orc_nblk(self._h))
        x, y = np.zeros(self.nnz), np.zeros(max(self.m, 1))
        S, Z, T, out = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(6)
        _load().orc_hsde_get(self._h, _d(x), _d(y), _d(S), _d(Z), _d(T), _d(out))
        return dict(x=x, y=y[:self.m], s=self._split(S), z=self._split(Z), t=self._split(T),
                    tau=out[0], kappa=out[1], eps_p=out[2], eps_d=out[3], eps_g=out[4],
                    eps_c=out[5])

    def hsde_raw(self):
        """u_x and u_y (not divided by tau)."""
        x, y = np.zeros(self.nnz), np.zeros(max(self.m, 1))
        _load().orc_hsde_raw(self._h, _d(x), _d(y))
        return x, y[:self.m]

    def hsde_set(self, ux, us, uy, ut, vz, tau, kappa):
        cat = lambda bl: np.ascontiguousarray(np.concatenate([np.asarray(b, float).ravel()
                                                              for b in bl]))
        a = [np.ascontiguousarray(ux, float), cat(us), np.ascontiguousarray(uy, float),
             cat(ut), cat(vz)]
        _load().orc_hsde_set(self._h, *[_d(v) for v in a], float(tau), float(kappa))

    def hsde_inner(self, nx, ns, ny, nt):
        """sigma = M^-1 nu for the inner system of Section 5.2.2."""
        n = int(_load().orc_nblk(self._h))
        cat = lambda bl: np.ascontiguousarray(np.concatenate([np.asarray(b, float).ravel()
                                                              for b in bl]))
        nx, ny = np.ascontiguousarray(nx, float), np.ascontiguousarray(ny, float)
        ns, nt = cat(ns), cat(nt)
        sx, sy = np.zeros(self.nnz), np.zeros(max(self.m, 1))
        ss, st = np.zeros(n), np.zeros(n)
        _load().orc_hsde_inner(self._h, _d(nx), _d(ns), _d(ny), _d(nt), _d(sx), _d(ss), _d(sy),
                               _d(st))
        return sx, self._split(ss), sy[:self.m], self._split(st)

    def set_v_blocks(self, Vs):
        V = np.concatenate([np.asarray(v, dtype=np.float64).ravel() for v in Vs])
        _load().orc_set_vd(self._h, _d(V))

    def _run(self, fn, max_iter, tol, adaptive, mu, nu, rho_period):
        lib = _load()
        hc = np.zeros(max(max_iter, 1))
        hl = np.zeros(max(max_iter, 1))
        hr = np.zeros(max(max_iter, 1))
        it = C.c_int(0)
        st = fn(self._h, int(max_iter), float(tol), int(bool(adaptive)), float(mu),
                float(nu), int(rho_period), C.byref(it), _d(hc), _d(hl), _d(hr))
        k = it.value
        return RunResult(st, k, lib.orc_eps_c(self._h), lib.orc_eps_l(self._h),
                         lib.orc_rho(self._h), hc[:k], hl[:k], hr[:k])

    @property
    def rho(self):
        return _load().orc_rho(self._h)

    @rho.setter
    def rho(self, v):
        _load().orc_set_rho(self._h, float(v))

    @property
    def iters(self):
        return _load().orc_iters(self._h)

    def total_sweeps(self):
        return int(_load().orc_total_sweeps(self._h))

    def max_sweeps_seen(self):
        return int(_load().orc_max_sweeps_seen(self._h))

    def u(self):
        out = np.zeros(self.nnz)
        _load().orc_get_u(self._h, _d(out))
        return out

    def y(self):
        out = np.zeros(max(self.m, 1))
        _load().orc_get_y(self._h, _d(out))
        return out[:self.m]

    def y_dual(self):
        return -self.rho * self.y()

    # conjugate-gradient affine step ----------------------------------------
    def set_affine_cg(self, max_iter: int, tol: float = 0.0):
        """Algorithm 1's affine step by preconditioned CG (max_iter > 0) or by
        the cached factor (max_iter = 0)."""
        rc = _load().orc_set_affine_cg(self._h, int(max_iter), float(tol))
        if rc != OK:
            raise OracleError(rc)

    def pcg(self, rhs, y0, max_iter: int, tol_abs: float = 0.0):
        """Standalone PCG on (A W D^-1 A^T) y = rhs from y0 (after
        set_affine_cg): (y, residual norms ||r_j||_2 for j = 0..steps)."""
        y = np.array(y0, dtype=np.float64)
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        hist = np.zeros(max_iter + 1)
        k = _load().orc_pcg(self._h, _d(rhs), _d(y), int(max_iter), float(tol_abs), _d(hist))
        return y, hist[:k + 1]

    def cg_steps(self) -> int:
        return int(_load().orc_cg_steps(self._h))

    def D(self):
        out = np.zeros(self.nnz)
        _load().orc_get_D(self._h, _d(out))
        return out

    def L(self):
        out = np.zeros((self.m, self.m))
        _load().orc_get_L(self._h, _d(out))
        return out

    def blocks(self):
        """(X_k, Lambda_k) lists of full s_k x s_k matrices."""
        n = int(_load().orc_nblk(self._h))
        X = np.zeros(n)
        Lm = np.zeros(n)
        _load().orc_get_blocks(self._h, _d(X), _d(Lm))
        return self._split(X), self._split(Lm)

    def set_blocks(self, Xs, Ls):
        X = np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in Xs])
        Lm = np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in Ls])
        _load().orc_set_blocks(self._h, _d(X), _d(Lm))

    def next_w(self):
        """Projection inputs W_k of the next iteration from the current state."""
        n = int(_load().orc_nblk(self._h))
        W = np.zeros(n)
        _load().orc_next_w(self._h, _d(W))
        return self._split(W)

    def gather(self, u):
        """E_k U E_k^T for every clique, as full matrices."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        n = int(_load().orc_nblk(self._h))
        out = np.zeros(n)
        _load().orc_gather_blocks(self._h, _d(u), _d(out))
        return self._split(out)

    def _split(self, flat):
        return [flat[self.blk_off[k]:self.blk_off[k + 1]].reshape(s, s)
                for k, s in enumerate(self.sizes)]

    def form_bhat(self, Xs, Ls, rho):
        X = np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in Xs])
        Lm = np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in Ls])
        out = np.zeros(self.nnz)
        _load().orc_form_bhat(self._h, _d(X), _d(Lm), float(rho), _d(out))
        return out

    def affine(self, bhat, b=None):
        bhat = np.ascontiguousarray(bhat, dtype=np.float64)
        bb = np.ascontiguousarray(self.inst.b if b is None else b, dtype=np.float64)
        u = np.zeros(self.nnz)
        y = np.zeros(max(self.m, 1))
        _load().orc_affine(self._h, _d(bhat), _d(bb), _d(u), _d(y))
        return u, y[:self.m]

    def objective(self):
        return float(_load().orc_objective(self._h))

    def set_cb(self, c=None, b=None):
        """Replace C (lower values) and/or b; A and the factor are unchanged."""
        cc = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
        bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
        _load().orc_set_cb(self._h, None if cc is None else _d(cc), None if bb is None else _d(bb))
        if cc is not None:
            self._c_keep = cc
        if bb is not None:
            self._b_keep = bb

    def unrolled_vjp(self, T, rho, ubar):
        """u_T of T unrolled iterations (fixed rho, from X = Lambda = 0) and the
        VJP (cbar, bbar) for the cotangent ubar of u_T (Frobenius products)."""
        ub = np.ascontiguousarray(ubar, dtype=np.float64)
        uT = np.zeros(self.nnz)
        cb = np.zeros(self.nnz)
        bb = np.zeros(max(self.m, 1))
        _load().orc_unrolled_vjp(self._h, int(T), float(rho), _d(ub), _d(uT), _d(cb), _d(bb))
        return uT, cb, bb[:self.m]

    def unrolled_forward(self, T, rho):
        self.reset(rho)
        self.run(T, tol=0.0)
        return self.u()

    def diagnostics(self):
        out = np.zeros(6)
        _load().orc_diagnostics(self._h, _d(out))
        return dict(eps_p=out[0], eps_d=out[1], eps_g=out[2], eps_alpha=out[3],
                    objective=out[4], dual_objective=out[5])


def create_status(inst) -> int:
    """Status code the oracle's validation returns for ``inst`` (0 if valid)."""
    try:
        Problem(inst)
    except OracleError as e:
        return e.code
    return OK
