"""Bindings of the host preprocessing entry points of libsdp: argument
marshalling only.

* ``chordal_extension`` -- the chordal extension of a (possibly nonchordal)
  pattern and its maximal cliques (Theorem 1; the preprocessing of Section
  7.1.1), computed by ``sdp_pattern_create``.
* ``extend_instance`` -- an instance given on any pattern, re-expressed on
  that extension (its A and C entries moved to their coordinates in the
  extended pattern, zeros on the added ones) so that the solver accepts it.
* ``scale_instance`` / ``Scaling.recover`` -- the data scaling of Section
  7.1.3 (``sdp_scale_compute``, ``sdp_scale_apply``, ``sdp_scale_recover``).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

from ._native import A_CSR, A_DENSE, _Marshalled, _check, _p, lib

_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_dp = C.POINTER(C.c_double)

lib.sdp_pattern_create.argtypes = [C.c_int32, C.c_int64, _p, _p, C.POINTER(_p)]
lib.sdp_pattern_sizes.argtypes = [_p, _lp, _ip, _lp]
lib.sdp_pattern_get.argtypes = [_p, _p, _p, _p, _p, C.c_int64, _p, _p, _p]
lib.sdp_pattern_destroy.argtypes = [_p]
lib.sdp_pattern_destroy.restype = None
lib.sdp_scale_compute.argtypes = [C.c_void_p, C.c_int32, _p, _p, _dp, _dp]
lib.sdp_scale_apply.argtypes = [C.c_void_p, _p, _p, C.c_double, C.c_double, _p, _p, _p]
lib.sdp_scale_recover.argtypes = [C.c_void_p, _p, _p, C.c_double, C.c_double, _p, _p, _p]
for _name in ("sdp_pattern_create", "sdp_pattern_sizes", "sdp_pattern_get", "sdp_scale_compute",
              "sdp_scale_apply", "sdp_scale_recover"):
    getattr(lib, _name).restype = C.c_int


@dataclass
class InstanceData:
    """An SDP instance in the layout ``sdp_instance`` expects (see sdp.h)."""
    n: int
    m: int
    pat_row: np.ndarray
    pat_col: np.ndarray
    clique_ptr: np.ndarray
    clique_vert: np.ndarray
    a_format: int
    a_val: np.ndarray
    b: np.ndarray
    c: np.ndarray
    a_rowptr: Optional[np.ndarray] = None
    a_col: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.pat_row.shape[0])

    @property
    def p(self) -> int:
        return int(self.clique_ptr.shape[0] - 1)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class ChordalPattern:
    """Result of ``sdp_pattern_create`` on one pattern."""

    def __init__(self, n: int, row, col):
        self.n = int(n)
        self._row, self._col = _i32(row), _i32(col)
        if self._row.shape != self._col.shape:
            raise ValueError("row and col differ in length")
        h = _p()
        _check(lib.sdp_pattern_create(self.n, int(self._row.shape[0]), _ptr(self._row),
                                      _ptr(self._col), C.byref(h)))
        self._h = h
        nnz, p, tot = C.c_int64(), C.c_int32(), C.c_int64()
        _check(lib.sdp_pattern_sizes(h, C.byref(nnz), C.byref(p), C.byref(tot)))
        self.pat_row = np.zeros(nnz.value, np.int32)
        self.pat_col = np.zeros(nnz.value, np.int32)
        self.clique_ptr = np.zeros(p.value + 1, np.int32)
        self.clique_vert = np.zeros(tot.value, np.int32)
        _check(lib.sdp_pattern_get(h, _ptr(self.pat_row), _ptr(self.pat_col), _ptr(self.clique_ptr),
                                   _ptr(self.clique_vert), 0, None, None, None))

    def index_of(self, row, col) -> np.ndarray:
        """Positions of the coordinates (either triangle) in the extended
        pattern (-1 where absent)."""
        r, c = _i32(row), _i32(col)
        out = np.zeros(r.shape[0], np.int64)
        _check(lib.sdp_pattern_get(self._h, None, None, None, None, int(r.shape[0]), _ptr(r),
                                   _ptr(c), _ptr(out)))
        return out

    @property
    def p(self) -> int:
        return int(self.clique_ptr.shape[0] - 1)

    def cliques(self):
        return [self.clique_vert[self.clique_ptr[k]:self.clique_ptr[k + 1]] for k in range(self.p)]

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h is not None and h.value:
            lib.sdp_pattern_destroy(h)

    def __del__(self):
        self.close()


def chordal_extension(n: int, row, col) -> ChordalPattern:
    return ChordalPattern(n, row, col)


def extend_instance(inst, pattern: Optional[ChordalPattern] = None) -> InstanceData:
    """The instance (any object with sdp_instance's fields; its cliques are
    ignored) on the chordal extension of its own pattern."""
    if pattern is None:
        pattern = ChordalPattern(inst.n, inst.pat_row, inst.pat_col)
    idx = pattern.index_of(inst.pat_row, inst.pat_col)
    if (idx < 0).any():
        raise ValueError("pattern coordinate missing from the extension")
    nnz = pattern.pat_row.shape[0]
    c = np.zeros(nnz)
    c[idx] = inst.c
    if int(inst.a_format) == A_DENSE:
        a = np.zeros((inst.m, nnz))
        a[:, idx] = np.asarray(inst.a_val).reshape(inst.m, -1)
        rp = ac = None
    else:
        a = np.array(inst.a_val, dtype=np.float64)
        rp = np.array(inst.a_rowptr, dtype=np.int64)
        ac = idx[np.asarray(inst.a_col)].astype(np.int32)
    return InstanceData(n=int(inst.n), m=int(inst.m), pat_row=pattern.pat_row.copy(),
                        pat_col=pattern.pat_col.copy(), clique_ptr=pattern.clique_ptr.copy(),
                        clique_vert=pattern.clique_vert.copy(), a_format=int(inst.a_format),
                        a_val=a, b=np.array(inst.b, dtype=np.float64), c=c, a_rowptr=rp,
                        a_col=ac, name=(getattr(inst, "name", "") or "instance") + "_ext")


@dataclass
class Scaling:
    """Scaling factors of one instance: e (row_scale), s (vertex_scale),
    rho_b, sigma_c; ``scaled`` is the scaled instance."""
    row_scale: np.ndarray
    vertex_scale: np.ndarray
    rho_b: float
    sigma_c: float
    scaled: InstanceData

    def recover(self, x=None, y=None, z=None):
        """(x, y, z) of the original problem from those of the scaled one
        (copies; None stays None)."""
        xs = None if x is None else np.array(x, dtype=np.float64)
        ys = None if y is None else np.array(y, dtype=np.float64)
        zs = None if z is None else np.array(z, dtype=np.float64)
        mi = _Marshalled(self.scaled)
        _check(lib.sdp_scale_recover(C.byref(mi.s), _ptr(self.row_scale), _ptr(self.vertex_scale),
                                     self.rho_b, self.sigma_c, _ptr(xs), _ptr(ys), _ptr(zs)))
        return xs, ys, zs


def _as_data(inst) -> InstanceData:
    return InstanceData(n=int(inst.n), m=int(inst.m), pat_row=_i32(inst.pat_row),
                        pat_col=_i32(inst.pat_col), clique_ptr=_i32(inst.clique_ptr),
                        clique_vert=_i32(inst.clique_vert), a_format=int(inst.a_format),
                        a_val=np.ascontiguousarray(inst.a_val, dtype=np.float64),
                        b=np.ascontiguousarray(inst.b, dtype=np.float64),
                        c=np.ascontiguousarray(inst.c, dtype=np.float64),
                        a_rowptr=None if inst.a_rowptr is None else np.ascontiguousarray(inst.a_rowptr, np.int64),
                        a_col=None if inst.a_col is None else _i32(inst.a_col),
                        name=getattr(inst, "name", ""))


def scale_instance(inst, iters: int = 10) -> Scaling:
    src = _as_data(inst)
    mi = _Marshalled(src)
    e, s = np.zeros(src.m), np.zeros(src.n)
    rb, sc = C.c_double(), C.c_double()
    _check(lib.sdp_scale_compute(C.byref(mi.s), int(iters), _ptr(e), _ptr(s), C.byref(rb),
                                 C.byref(sc)))
    a, b, c = np.zeros_like(src.a_val), np.zeros(src.m), np.zeros(src.nnz)
    _check(lib.sdp_scale_apply(C.byref(mi.s), _ptr(e), _ptr(s), rb.value, sc.value, _ptr(a),
                               _ptr(b), _ptr(c)))
    scaled = replace(src, a_val=a, b=b, c=c, name=(src.name or "instance") + "_scaled")
    return Scaling(row_scale=e, vertex_scale=s, rho_b=rb.value, sigma_c=sc.value, scaled=scaled)
