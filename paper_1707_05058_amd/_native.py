"""ctypes binding of libsdp (include/sdp.h): argument marshalling only.

Every step of the solver runs in the HIP kernels behind the C ABI.  If the
in-tree library is missing this module raises ImportError -- there is no CPU
fallback.  torch is imported before the library is loaded so that libsdp and
torch share one HIP runtime (device pointers and streams from torch are then
valid inside the library).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

try:  # share torch's HIP runtime when torch is present
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdp.so")

# status codes (include/sdp.h)
OK = 0
MAX_ITER = 1
ERR_ARG = -1
ERR_PATTERN_UNCOVERED = -2
ERR_OFF_PATTERN = -3
ERR_CLIQUE_ORDER = -4
ERR_RANK_DEFICIENT = -5
ERR_NONFINITE = -6
ERR_UNSUPPORTED = -7
ERR_HIP = -8
ERR_OOM = -9

A_DENSE, A_CSR = 0, 1
FP64, FP32_EIG = 0, 1
DTYPE_FP64, DTYPE_FP32 = 0, 1
ALG_PRIMAL, ALG_DUAL, ALG_HSDE = 0, 1, 2
PRIMAL_INFEASIBLE, DUAL_INFEASIBLE = 2, 3

_p = C.c_void_p


class sdp_instance(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("nnz_pattern", C.c_int64),
                ("pat_row", _p), ("pat_col", _p), ("p", C.c_int32),
                ("clique_ptr", _p), ("clique_vert", _p), ("a_format", C.c_int32),
                ("a_rowptr", _p), ("a_col", _p), ("a_val", _p), ("b", _p), ("c", _p)]


class sdp_options(C.Structure):
    _fields_ = [("rho", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("adaptive_rho", C.c_int32), ("mu", C.c_double),
                ("nu", C.c_double), ("rho_period", C.c_int32), ("graph_chunk", C.c_int32),
                ("stream", _p), ("jacobi_max_sweeps", C.c_int32), ("jacobi_tol", C.c_double),
                ("autotune", C.c_int32), ("warm_start", C.c_int32), ("algorithm", C.c_int32),
                ("cg_max_iter", C.c_int32), ("cg_tol", C.c_double),
                ("projection_method", C.c_int32), ("decouple", C.c_int32)]


class sdp_result(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("eps_c", C.c_double),
                ("eps_lambda", C.c_double), ("objective", C.c_double), ("rho", C.c_double),
                ("eps_p", C.c_double), ("eps_d", C.c_double), ("eps_g", C.c_double),
                ("eps_alpha", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["sdp_default_options", "sdp_setup", "sdp_reset", "sdp_admm_step", "sdp_solve",
           "sdp_psd_project_batched", "sdp_projection_variants", "sdp_psd_project_variant",
           "sdp_get_solution", "sdp_set_state", "sdp_get_history",
           "sdp_diagnostics", "sdp_diagnostics_noalloc", "sdp_get_stats",
           "sdp_get_projection_stats", "sdp_projection_plan", "sdp_time_stages",
           "sdp_update_data", "sdp_unrolled_forward", "sdp_vjp", "sdp_cg_steps", "sdp_destroy",
           "sdp_projection_variant_kind", "sdp_projection_plan_variants",
           "sdp_projection_default_variant", "sdp_sign_schedule",
           "sdp_last_error",
           "sdp_pattern_create", "sdp_pattern_sizes", "sdp_pattern_get", "sdp_pattern_destroy",
           "sdp_scale_compute", "sdp_scale_apply", "sdp_scale_recover"]

STAGES = ["scatter", "A_v", "Linv_r", "LinvT_y", "AT_y", "projection", "residual"]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsdp.so not built at {LIB_PATH}; run "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    lib.sdp_default_options.argtypes = [C.POINTER(sdp_options)]
    lib.sdp_default_options.restype = None
    lib.sdp_setup.argtypes = [C.c_int32, C.POINTER(sdp_instance), C.POINTER(sdp_options),
                              C.POINTER(_p)]
    lib.sdp_reset.argtypes = [_p]
    lib.sdp_admm_step.argtypes = [_p, C.c_int32, C.POINTER(sdp_result)]
    lib.sdp_solve.argtypes = [_p, C.POINTER(sdp_result)]
    lib.sdp_psd_project_batched.argtypes = [C.c_int32, C.c_int32, _p, _p, _p, _p, C.c_int32, _p]
    lib.sdp_psd_project_variant.argtypes = [C.c_int32, C.c_int32, C.c_int32, _p, _p, _p, _p,
                                            C.c_int32, _p]
    lib.sdp_projection_variants.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                            C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.sdp_get_solution.argtypes = [_p, C.c_int32, dp, dp, dp, dp]
    lib.sdp_set_state.argtypes = [_p, C.c_int32, dp, dp, C.c_double]
    lib.sdp_get_history.argtypes = [_p, C.c_int32, C.c_int32, dp, dp, dp, C.POINTER(C.c_int32)]
    lib.sdp_diagnostics.argtypes = [_p, C.POINTER(sdp_result)]
    lib.sdp_diagnostics_noalloc.argtypes = [_p, C.POINTER(sdp_result)]
    lib.sdp_get_stats.argtypes = [_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.sdp_get_projection_stats.argtypes = [_p] + [C.POINTER(C.c_int64)] * 3
    ip = C.POINTER(C.c_int32)
    lib.sdp_projection_plan.argtypes = [_p, C.c_int32, ip, ip, ip, ip]
    lib.sdp_time_stages.argtypes = [_p, C.c_int32, dp]
    lib.sdp_update_data.argtypes = [_p, _p, _p]
    lib.sdp_unrolled_forward.argtypes = [_p, C.c_int32, C.c_int32, _p]
    lib.sdp_vjp.argtypes = [_p, _p, _p, _p, C.c_int32]
    lib.sdp_cg_steps.argtypes = [_p, C.POINTER(C.c_int64)]
    lib.sdp_projection_variant_kind.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    lib.sdp_projection_default_variant.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    lib.sdp_sign_schedule.argtypes = [C.c_double, C.c_int32, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]
    lib.sdp_projection_plan_variants.argtypes = [_p, C.c_int32, ip, C.POINTER(C.c_int32)]
    lib.sdp_destroy.argtypes = [_p]
    lib.sdp_destroy.restype = None
    lib.sdp_last_error.argtypes = []
    lib.sdp_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name.startswith(("sdp_pattern_", "sdp_scale_")):
            continue                      # typed in preprocess.py
        if name not in ("sdp_default_options", "sdp_destroy", "sdp_last_error"):
            getattr(lib, name).restype = C.c_int
    return lib


lib = _load()


class SdpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsdp status {code}: {msg}")
        self.code = code


def _check(rc: int, ok=(OK,)) -> int:
    if rc not in ok:
        raise SdpError(rc, lib.sdp_last_error().decode())
    return rc


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_p)


def _dptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def default_options() -> sdp_options:
    o = sdp_options()
    lib.sdp_default_options(C.byref(o))
    return o


def make_options(**kw) -> sdp_options:
    o = default_options()
    for k, v in kw.items():
        if k == "stream":
            v = None if v is None else C.c_void_p(int(v))
        elif k == "precision" and isinstance(v, str):
            v = {"fp64": FP64, "fp32": FP32_EIG, "fp32_eig": FP32_EIG}[v.lower()]
        elif k == "algorithm" and isinstance(v, str):
            v = {"primal": ALG_PRIMAL, "dual": ALG_DUAL, "hsde": ALG_HSDE}[v.lower()]
        elif k == "projection_method" and isinstance(v, str):
            v = {"auto": 0, "scalar": 1, "two_level": 2, "sign": 3}[v.lower()]
        setattr(o, k, v)
    return o


class _Marshalled:
    """Holds the contiguous arrays of one instance while sdp_setup copies them."""

    def __init__(self, inst):
        self.pr = np.ascontiguousarray(inst.pat_row, dtype=np.int32)
        self.pc = np.ascontiguousarray(inst.pat_col, dtype=np.int32)
        self.cp = np.ascontiguousarray(inst.clique_ptr, dtype=np.int32)
        self.cv = np.ascontiguousarray(inst.clique_vert, dtype=np.int32)
        self.av = np.ascontiguousarray(inst.a_val, dtype=np.float64)
        self.b = np.ascontiguousarray(inst.b, dtype=np.float64)
        self.c = np.ascontiguousarray(inst.c, dtype=np.float64)
        csr = int(inst.a_format) == A_CSR
        self.ar = np.ascontiguousarray(inst.a_rowptr, dtype=np.int64) if csr else None
        self.ac = np.ascontiguousarray(inst.a_col, dtype=np.int32) if csr else None
        s = sdp_instance()
        s.n, s.m = int(inst.n), int(inst.m)
        s.nnz_pattern = int(self.pr.shape[0])
        s.pat_row, s.pat_col = _ptr(self.pr), _ptr(self.pc)
        s.p = int(self.cp.shape[0] - 1)
        s.clique_ptr, s.clique_vert = _ptr(self.cp), _ptr(self.cv)
        s.a_format = int(inst.a_format)
        s.a_rowptr, s.a_col = _ptr(self.ar), _ptr(self.ac)
        s.a_val, s.b, s.c = _ptr(self.av), _ptr(self.b), _ptr(self.c)
        self.s = s


def setup_status(instances, **options) -> int:
    """Status sdp_setup returns for these instances (handle destroyed)."""
    ms = [_Marshalled(i) for i in instances]
    arr = (sdp_instance * len(ms))(*[m.s for m in ms])
    opt = make_options(**options)
    h = _p()
    rc = lib.sdp_setup(len(ms), arr, C.byref(opt), C.byref(h))
    if rc == OK:
        lib.sdp_destroy(h)
    return rc


class Solver:
    """Decomposed primal ADMM (Algorithm 1) on a batch of SDP instances."""

    def __init__(self, instances, **options):
        if not isinstance(instances, (list, tuple)):
            instances = [instances]
        self.instances = list(instances)
        ms = [_Marshalled(i) for i in self.instances]
        arr = (sdp_instance * len(ms))(*[m.s for m in ms])
        self.options = make_options(**options)
        h = _p()
        _check(lib.sdp_setup(len(ms), arr, C.byref(self.options), C.byref(h)))
        self._h = h
        self.batch = len(ms)
        self.sizes = [np.diff(np.asarray(i.clique_ptr)).astype(np.int64) for i in self.instances]
        self.npk = [int(np.sum(s * (s + 1) // 2)) for s in self.sizes]

    def close(self):
        if getattr(self, "_h", None):
            lib.sdp_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def reset(self):
        _check(lib.sdp_reset(self._h))

    def step(self, n_steps: int, results: bool = True):
        res = (sdp_result * self.batch)() if results else None
        _check(lib.sdp_admm_step(self._h, int(n_steps), res))
        return [r.as_dict() for r in res] if results else None

    def solve(self):
        res = (sdp_result * self.batch)()
        _check(lib.sdp_solve(self._h, res), ok=(OK, MAX_ITER, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE))
        return [r.as_dict() for r in res]

    def diagnostics(self, noalloc: bool = False):
        """eps_p, eps_d, eps_g, eps_alpha of the current iterate; noalloc selects
        sdp_diagnostics_noalloc (scratch in the library's static device array)."""
        res = (sdp_result * self.batch)()
        fn = lib.sdp_diagnostics_noalloc if noalloc else lib.sdp_diagnostics
        _check(fn(self._h, res))
        return [r.as_dict() for r in res]

    def solution(self, i: int = 0):
        inst = self.instances[i]
        u = np.zeros(inst.pat_row.shape[0])
        y = np.zeros(inst.m)
        X = np.zeros(self.npk[i])
        L = np.zeros(self.npk[i])
        _check(lib.sdp_get_solution(self._h, i, _dptr(u), _dptr(y), _dptr(X), _dptr(L)))
        return dict(u=u, y_dual=y, X_packed=X, L_packed=L)

    def blocks(self, i: int = 0):
        """(X_k, Lambda_k) of instance i as lists of full symmetric matrices."""
        sol = self.solution(i)
        return unpack_blocks(sol["X_packed"], self.sizes[i]), unpack_blocks(sol["L_packed"], self.sizes[i])

    def set_state(self, i: int, X_packed, L_packed, rho: float):
        Xp = np.ascontiguousarray(X_packed, dtype=np.float64)
        Lp = np.ascontiguousarray(L_packed, dtype=np.float64)
        _check(lib.sdp_set_state(self._h, i, _dptr(Xp), _dptr(Lp), float(rho)))

    def history(self, i: int = 0, cap: int = 100000):
        ec, el, rh = np.zeros(cap), np.zeros(cap), np.zeros(cap)
        n = C.c_int32(0)
        _check(lib.sdp_get_history(self._h, i, cap, _dptr(ec), _dptr(el), _dptr(rh), C.byref(n)))
        k = n.value
        return ec[:k], el[:k], rh[:k]

    def time_stages(self, n_iter: int):
        """Mean ms per iteration of each stage (HIP events on the solver's stream)."""
        ms = np.zeros(len(STAGES))
        _check(lib.sdp_time_stages(self._h, int(n_iter), _dptr(ms)))
        return dict(zip(STAGES, ms.tolist()))

    # --- differentiation of the unrolled iteration (device tensors) ---------
    @property
    def total_nnz(self):
        return int(sum(int(i.pat_row.shape[0]) for i in self.instances))

    @property
    def total_m(self):
        return int(sum(int(i.m) for i in self.instances))

    def update_data(self, c=None, b=None):
        """Replace C and/or b (float64 device tensors, concatenated layout)."""
        for t, n in ((c, self.total_nnz), (b, self.total_m)):
            if t is not None:
                _check_tensor(t, n)
        _check(lib.sdp_update_data(self._h, None if c is None else C.c_void_p(c.data_ptr()),
                                   None if b is None else C.c_void_p(b.data_ptr())))

    def unrolled_forward(self, T: int, ckpt_every: int, u_out=None):
        if u_out is not None:
            _check_tensor(u_out, self.total_nnz)
        _check(lib.sdp_unrolled_forward(self._h, int(T), int(ckpt_every),
                                        None if u_out is None else C.c_void_p(u_out.data_ptr())))

    def vjp(self, u_bar, c_bar, b_bar, euclidean: bool = False):
        _check_tensor(u_bar, self.total_nnz)
        _check_tensor(c_bar, self.total_nnz)
        _check_tensor(b_bar, self.total_m)
        _check(lib.sdp_vjp(self._h, C.c_void_p(u_bar.data_ptr()), C.c_void_p(c_bar.data_ptr()),
                           C.c_void_p(b_bar.data_ptr()), int(bool(euclidean))))

    def stats(self):
        sw, pr, sg = C.c_int64(0), C.c_int64(0), C.c_int64(0)
        _check(lib.sdp_get_projection_stats(self._h, C.byref(sw), C.byref(pr), C.byref(sg)))
        return dict(jacobi_sweeps=sw.value, projections=pr.value, sign_fallbacks=sg.value)

    def cg_steps(self) -> int:
        """Conjugate-gradient steps over all instances since the last reset."""
        n = C.c_int64(0)
        _check(lib.sdp_cg_steps(self._h, C.byref(n)))
        return n.value

    def projection_plan(self):
        """[(N, threads, cliques)] of the projection launch lists."""
        n = C.c_int32(0)
        _check(lib.sdp_projection_plan(self._h, 0, None, None, None, C.byref(n)))
        k = n.value
        N, NT, cnt = (C.c_int32 * k)(), (C.c_int32 * k)(), (C.c_int32 * k)()
        _check(lib.sdp_projection_plan(self._h, k, N, NT, cnt, C.byref(n)))
        return [(N[i], NT[i], cnt[i]) for i in range(k)]

    def projection_plan_variants(self):
        """Kernel variant index of each projection launch list."""
        n = C.c_int32(0)
        _check(lib.sdp_projection_plan_variants(self._h, 0, None, C.byref(n)))
        k = n.value
        v = (C.c_int32 * k)()
        _check(lib.sdp_projection_plan_variants(self._h, k, v, C.byref(n)))
        return list(v)


def _check_tensor(t, n):
    import torch as _t
    if t.dtype != _t.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"expected a contiguous float64 device tensor of {n} elements")


def pack_blocks(blocks: Sequence[np.ndarray]) -> np.ndarray:
    """Full symmetric blocks -> packed lower rows (entry (i,j), i>=j, at i(i+1)/2+j)."""
    out = []
    for B in blocks:
        s = B.shape[0]
        r, c = np.tril_indices(s)
        out.append(np.asarray(B)[r, c])
    return np.concatenate(out) if out else np.zeros(0)


def unpack_blocks(flat: np.ndarray, sizes) -> List[np.ndarray]:
    out, o = [], 0
    for s in sizes:
        s = int(s)
        n = s * (s + 1) // 2
        B = np.zeros((s, s))
        r, c = np.tril_indices(s)
        B[r, c] = flat[o:o + n]
        B[c, r] = flat[o:o + n]
        out.append(B)
        o += n
    return out


def psd_project_batched(sizes, offsets, inp, out, max_size: int, stream=None,
                        variant: Optional[int] = None) -> None:
    """Standalone PSD projection of full row-major blocks (torch CUDA tensors).

    sizes: int32 tensor [count]; offsets: int64 tensor [count] (element
    offsets); inp/out: float32 or float64 tensors of the same dtype.  variant:
    an index into projection_variants(dtype) (None: the smallest block size
    that fits max_size).
    """
    import torch as _t
    if inp.dtype == _t.float64:
        dt = DTYPE_FP64
    elif inp.dtype == _t.float32:
        dt = DTYPE_FP32
    else:
        raise TypeError("inp must be float32 or float64")
    if out.dtype != inp.dtype or sizes.dtype != _t.int32 or offsets.dtype != _t.int64:
        raise TypeError("dtype mismatch")
    for t in (sizes, offsets, inp, out):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("all tensors must be contiguous device tensors")
    count = int(sizes.shape[0])
    if count and int(offsets.shape[0]) != count:
        raise ValueError("sizes/offsets length mismatch")
    st = _t.cuda.current_stream().cuda_stream if stream is None else int(stream)
    args = (count, int(max_size), C.c_void_p(sizes.data_ptr()), C.c_void_p(offsets.data_ptr()),
            C.c_void_p(inp.data_ptr()), C.c_void_p(out.data_ptr()), dt, C.c_void_p(st))
    if variant is None:
        _check(lib.sdp_psd_project_batched(*args))
    else:
        _check(lib.sdp_psd_project_variant(int(variant), *args))


def projection_variant_kind(dtype: int, variant: int) -> int:
    """0 scalar Jacobi, 1 two-level Jacobi, 2 sign function (no eigenvectors)."""
    t = C.c_int32(0)
    _check(lib.sdp_projection_variant_kind(int(dtype), int(variant), C.byref(t)))
    return t.value


def sign_schedule(tol: float, n: int):
    """(k1, k2): fast and Newton-Schulz steps of the sign iteration for blocks
    of n vertices at tolerance tol (relative to ||W||_F)."""
    k1, k2 = C.c_int32(0), C.c_int32(0)
    _check(lib.sdp_sign_schedule(float(tol), int(n), C.byref(k1), C.byref(k2)))
    return k1.value, k2.value


def projection_default_variant(dtype: int, max_size: int) -> int:
    """The variant psd_project_batched runs (no explicit variant) for blocks of
    up to max_size."""
    t = C.c_int32(0)
    _check(lib.sdp_projection_default_variant(int(dtype), int(max_size), C.byref(t)))
    return t.value


def projection_variant_two_level(dtype: int, variant: int) -> bool:
    """Whether the variant runs the two-level (block) Jacobi method."""
    return projection_variant_kind(dtype, variant) == 1


def projection_variants(dtype: int):
    """[(N, threads)] of the projection kernel variants for DTYPE_FP64/DTYPE_FP32."""
    n = C.c_int32(0)
    _check(lib.sdp_projection_variants(int(dtype), 0, None, None, C.byref(n)))
    k = n.value
    N, NT = (C.c_int32 * k)(), (C.c_int32 * k)()
    _check(lib.sdp_projection_variants(int(dtype), k, N, NT, C.byref(n)))
    return [(N[i], NT[i]) for i in range(k)]