"""Seeded synthetic SDP instances with chordal aggregate sparsity.

This module only *builds problem data*; it contains none of the solver's
arithmetic.  Both the CPU oracle and the GPU library consume what it
produces, so it is the one piece of code they share.

Storage convention (used by every consumer):

* The aggregate sparsity pattern E (the paper's G(V, E) with self-loops E*,
  Section "Sparse matrix cones and chordal decomposition") is given by its
  lower-triangle coordinates ``(pat_row[j], pat_col[j])`` with
  ``pat_row >= pat_col``, sorted by column and then by row (the order in which
  ``vec`` stacks columns).  Every diagonal entry is present.
* The maximal cliques C_1..C_p (Theorem 1) are a CSR list
  ``clique_ptr[p+1]``, ``clique_vert[...]`` with 0-based vertices in strictly
  increasing ("natural") order.  The pattern is exactly the union of all
  clique pairs (a chordal graph, or a chordal extension of one).
* A_i and C are symmetric; only their lower-triangle values on the pattern
  are stored.  ``a_val`` is either dense ``m x nnz`` (row i holds A_i) or CSR
  over pattern coordinates.  ``c`` holds C's lower values, ``b`` the m
  right-hand sides.

Random data (block-arrow experiments, Section "Random SDPs with block-arrow
patterns"): each A_i gets N(0,1) values on the pattern, b_i = trace(A_i) so
that X = I is strictly feasible, and C = I + sum_i y0_i A_i with y0 ~ N(0,1)
so that Z = I is strictly dual feasible.  The paper draws U(0,1) data and
builds X_f = W + alpha I; the normal draw with X_f = Z_f = I used here keeps
the same pattern and strict feasibility on both sides.

Draw order per instance with ``numpy.random.default_rng(seed)`` (PCG64):
  1. (batched workload only) l, d, h as inclusive integer uniforms;
  2. the A_i values, row by row over the sorted pattern coordinates
     (sparse workloads: per row a Bernoulli mask first, then normals for the
     kept entries; a row that comes out empty is drawn again);
  3. y0 ~ N(0,1)^m.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

A_DENSE = 0
A_CSR = 1


@dataclass
class Instance:
    n: int
    m: int
    pat_row: np.ndarray          # int32 [nnz]
    pat_col: np.ndarray          # int32 [nnz]
    clique_ptr: np.ndarray       # int32 [p+1]
    clique_vert: np.ndarray      # int32 [clique_ptr[-1]]
    a_format: int                # A_DENSE or A_CSR
    a_val: np.ndarray            # float64: [m, nnz] (dense) or [nnz_A] (csr)
    b: np.ndarray                # float64 [m]
    c: np.ndarray                # float64 [nnz]
    a_rowptr: Optional[np.ndarray] = None   # int64 [m+1] (csr only)
    a_col: Optional[np.ndarray] = None      # int32 [nnz_A] (csr only)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.pat_row.shape[0])

    @property
    def p(self) -> int:
        return int(self.clique_ptr.shape[0] - 1)

    def clique(self, k: int) -> np.ndarray:
        return self.clique_vert[self.clique_ptr[k]:self.clique_ptr[k + 1]]

    def clique_sizes(self) -> np.ndarray:
        return np.diff(self.clique_ptr).astype(np.int32)

    def a_dense(self) -> np.ndarray:
        """A as a dense m x nnz array (copies for CSR)."""
        if self.a_format == A_DENSE:
            return self.a_val
        out = np.zeros((self.m, self.nnz))
        for i in range(self.m):
            lo, hi = self.a_rowptr[i], self.a_rowptr[i + 1]
            out[i, self.a_col[lo:hi]] = self.a_val[lo:hi]
        return out


# ----------------------------------------------------------------------------
# Patterns (vertex sets of the maximal cliques)
# ----------------------------------------------------------------------------

def block_arrow_cliques(l: int, d: int, h: int) -> List[np.ndarray]:
    """Block-arrow pattern: l diagonal blocks of size d, arrow head of width h.

    Vertices of block k are k*d .. k*d+d-1, the head is l*d .. l*d+h-1; the
    maximal cliques are {block k} U head, all of size d + h.
    """
    head = np.arange(l * d, l * d + h, dtype=np.int32)
    return [np.concatenate([np.arange(k * d, (k + 1) * d, dtype=np.int32), head])
            for k in range(l)]


def banded_cliques(n: int, w: int) -> List[np.ndarray]:
    """Banded pattern of half-bandwidth w: maximal cliques {i, ..., i+w}."""
    return [np.arange(i, i + w + 1, dtype=np.int32) for i in range(n - w)]


def pattern_from_cliques(n: int, cliques: Sequence[np.ndarray]):
    """Lower coordinates of the union of all clique pairs, sorted (col, row)."""
    keys = []
    for v in cliques:
        v = np.asarray(v, dtype=np.int64)
        r, c = np.meshgrid(v, v, indexing="ij")
        sel = r >= c
        keys.append(c[sel] * n + r[sel])
    # every vertex carries its diagonal even if it sits in no clique
    keys.append(np.arange(n, dtype=np.int64) * (n + 1))
    k = np.unique(np.concatenate(keys))
    return (k % n).astype(np.int32), (k // n).astype(np.int32)


def cliques_to_csr(cliques: Sequence[np.ndarray]):
    ptr = np.zeros(len(cliques) + 1, dtype=np.int32)
    ptr[1:] = np.cumsum([len(v) for v in cliques])
    vert = (np.concatenate([np.asarray(v, dtype=np.int32) for v in cliques])
            if cliques else np.zeros(0, dtype=np.int32))
    return ptr, vert


# ----------------------------------------------------------------------------
# Random data
# ----------------------------------------------------------------------------

def _finish(n, m, pat_row, pat_col, cliques, a_format, a_val, a_rowptr, a_col,
            y0, name, meta) -> Instance:
    nnz = pat_row.shape[0]
    diag = pat_row == pat_col
    ptr, vert = cliques_to_csr(cliques)
    if a_format == A_DENSE:
        b = a_val[:, diag].sum(axis=1)
        c = diag.astype(np.float64) + y0 @ a_val
    else:
        b = np.zeros(m)
        c = diag.astype(np.float64).copy()
        for i in range(m):
            lo, hi = a_rowptr[i], a_rowptr[i + 1]
            cols, vals = a_col[lo:hi], a_val[lo:hi]
            b[i] = vals[diag[cols]].sum()
            c[cols] += y0[i] * vals
    return Instance(n=n, m=m, pat_row=pat_row, pat_col=pat_col,
                    clique_ptr=ptr, clique_vert=vert, a_format=a_format,
                    a_val=a_val, b=b, c=c, a_rowptr=a_rowptr, a_col=a_col,
                    name=name, meta=meta)


def random_instance(n: int, cliques: Sequence[np.ndarray], m: int, seed=None,
                    density: Optional[float] = None, rng=None, name: str = "",
                    meta: Optional[dict] = None) -> Instance:
    """Random primal SDP on the pattern of ``cliques`` (draw order above)."""
    if rng is None:
        rng = np.random.default_rng(seed)
    pat_row, pat_col = pattern_from_cliques(n, cliques)
    return _instance_on(n, pat_row, pat_col, list(cliques), m, rng, seed, density, name, meta)


def _instance_on(n, pat_row, pat_col, cliques, m, rng, seed, density, name, meta) -> Instance:
    nnz = pat_row.shape[0]
    if density is None:
        a_val = rng.standard_normal((m, nnz))
        a_rowptr = a_col = None
        fmt = A_DENSE
    else:
        rows_c, rows_v = [], []
        for _ in range(m):
            while True:
                mask = rng.random(nnz) < density
                k = int(mask.sum())
                if k > 0:
                    break
            rows_c.append(np.nonzero(mask)[0].astype(np.int32))
            rows_v.append(rng.standard_normal(k))
        a_rowptr = np.zeros(m + 1, dtype=np.int64)
        a_rowptr[1:] = np.cumsum([len(r) for r in rows_c])
        a_col = np.concatenate(rows_c)
        a_val = np.concatenate(rows_v)
        fmt = A_CSR
    y0 = rng.standard_normal(m)
    return _finish(n, m, pat_row, pat_col, cliques, fmt, a_val, a_rowptr,
                   a_col, y0, name, dict(meta or {}, seed=seed))


def block_arrow_instance(l, d, h, m, seed, density=None, name="") -> Instance:
    n = l * d + h
    return random_instance(n, block_arrow_cliques(l, d, h), m, seed=seed,
                           density=density, name=name or f"blockarrow_l{l}_d{d}_h{h}_m{m}_s{seed}",
                           meta=dict(l=l, d=d, h=h))


def banded_instance(n, w, m, seed, name="") -> Instance:
    return random_instance(n, banded_cliques(n, w), m, seed=seed,
                           name=name or f"banded_n{n}_w{w}_m{m}_s{seed}",
                           meta=dict(w=w))


def uneven_block_arrow_instance(seed: int, l_range=(5, 50), d_range=(8, 40),
                                h_range=(2, 10)) -> Instance:
    """One instance of the batched workload: l, d, h drawn first, m = n // 2."""
    rng = np.random.default_rng(seed)
    l = int(rng.integers(l_range[0], l_range[1] + 1))
    d = int(rng.integers(d_range[0], d_range[1] + 1))
    h = int(rng.integers(h_range[0], h_range[1] + 1))
    n = l * d + h
    m = n // 2
    return random_instance(n, block_arrow_cliques(l, d, h), m, rng=rng, seed=seed,
                           name=f"uneven_s{seed}_l{l}_d{d}_h{h}_m{m}",
                           meta=dict(l=l, d=d, h=h))


def primal_infeasible_instance(l, d, h, m, seed) -> Instance:
    """A block-arrow instance with one more constraint <I, X> = -1, which no
    PSD X satisfies (the other m rows are the usual random ones)."""
    base = block_arrow_instance(l, d, h, m, seed)
    diag = (base.pat_row == base.pat_col).astype(np.float64)
    a = np.vstack([base.a_val, diag[None, :]])
    b = np.concatenate([base.b, [-1.0]])
    return Instance(n=base.n, m=m + 1, pat_row=base.pat_row, pat_col=base.pat_col,
                    clique_ptr=base.clique_ptr, clique_vert=base.clique_vert, a_format=A_DENSE,
                    a_val=a, b=b, c=base.c, name=f"primal_infeasible_l{l}_d{d}_h{h}_m{m}_s{seed}")


def dual_infeasible_instance(l, d, h, m, seed) -> Instance:
    """A block-arrow instance in which no constraint touches vertex 0 and
    C_00 = -1: X = I stays feasible while X_00 can grow without bound, so the
    primal is unbounded and no y makes C - sum y_i A_i PSD."""
    base = block_arrow_instance(l, d, h, m, seed)
    touch = (base.pat_row == 0) | (base.pat_col == 0)
    a = base.a_val.copy()
    a[:, touch] = 0.0
    tr = (base.pat_row == base.pat_col).astype(np.float64)
    b = a @ tr                                  # b_i = tr A_i: X = I is feasible
    c = base.c.copy()
    c[touch] = 0.0
    c[(base.pat_row == 0) & (base.pat_col == 0)] = -1.0
    return Instance(n=base.n, m=m, pat_row=base.pat_row, pat_col=base.pat_col,
                    clique_ptr=base.clique_ptr, clique_vert=base.clique_vert, a_format=A_DENSE,
                    a_val=a, b=b, c=c, name=f"dual_infeasible_l{l}_d{d}_h{h}_m{m}_s{seed}")


# ----------------------------------------------------------------------------
# Nonchordal patterns (Section "Nonchordal SDPs": the cone's pattern is first
# given a chordal extension).  These instances carry no cliques: the solver
# takes them only after the extension step.
# ----------------------------------------------------------------------------

def _lower_sorted(n: int, edges) -> tuple:
    """Lower coordinates of the edges plus every diagonal, sorted (col, row)."""
    keys = [np.arange(n, dtype=np.int64) * (n + 1)]
    if len(edges):
        e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
        hi, lo = np.maximum(e[:, 0], e[:, 1]), np.minimum(e[:, 0], e[:, 1])
        keys.append(lo * n + hi)
    k = np.unique(np.concatenate(keys))
    return (k % n).astype(np.int32), (k // n).astype(np.int32)


def grid_pattern(rows: int, cols: int):
    """4-neighbour grid graph on rows x cols vertices (vertex r*cols + c);
    nonchordal for rows, cols >= 2 (every unit square is a chordless 4-cycle)."""
    edges = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            if c + 1 < cols:
                edges.append((v, v + 1))
            if r + 1 < rows:
                edges.append((v, v + cols))
    return _lower_sorted(rows * cols, edges)


def cycle_pattern(n: int):
    """The chordless cycle 0-1-...-(n-1)-0."""
    return _lower_sorted(n, [(i, (i + 1) % n) for i in range(n)])


def random_sparse_pattern(n: int, avg_degree: float, seed: int):
    """A path through all vertices (so the graph is connected) plus uniformly
    drawn extra edges up to the average degree."""
    rng = np.random.default_rng(seed)
    edges = [(i, i + 1) for i in range(n - 1)]
    extra = max(0, int(round(avg_degree * n / 2)) - (n - 1))
    a = rng.integers(0, n, size=extra)
    b = rng.integers(0, n, size=extra)
    edges += [(int(x), int(y)) for x, y in zip(a, b) if x != y]
    return _lower_sorted(n, edges)


def instance_on_pattern(n: int, pat_row, pat_col, m: int, seed: int, density=None,
                        name: str = "") -> Instance:
    """Random data (draw order as for every instance here) on an arbitrary
    pattern; no cliques."""
    rng = np.random.default_rng(seed)
    return _instance_on(n, np.asarray(pat_row, np.int32), np.asarray(pat_col, np.int32), [], m,
                        rng, seed, density, name or f"pattern_n{n}_m{m}_s{seed}", {})


def sparse_rows_instance(n: int, cliques: Sequence[np.ndarray], m: int, nnz_per_row: int,
                         seed: int, name: str = "") -> Instance:
    """Random primal SDP whose constraints each touch nnz_per_row pattern
    coordinates (CSR A).  Draw order: for each row, 2 * nnz_per_row uniform
    coordinate indices (distinct ones kept, first nnz_per_row in draw order,
    then sorted), then nnz_per_row normals; finally y0 ~ N(0,1)^m."""
    rng = np.random.default_rng(seed)
    pat_row, pat_col = pattern_from_cliques(n, cliques)
    nnz = pat_row.shape[0]
    k = min(nnz_per_row, nnz)
    rows_c, rows_v = [], []
    for _ in range(m):
        while True:
            cand = rng.integers(0, nnz, size=2 * k)
            _, first = np.unique(cand, return_index=True)
            if first.shape[0] >= k:
                break
        cols = np.sort(cand[np.sort(first)[:k]]).astype(np.int32)
        rows_c.append(cols)
        rows_v.append(rng.standard_normal(k))
    a_rowptr = np.arange(m + 1, dtype=np.int64) * k
    a_col = np.concatenate(rows_c)
    a_val = np.concatenate(rows_v)
    y0 = rng.standard_normal(m)
    return _finish(n, m, pat_row, pat_col, list(cliques), A_CSR, a_val, a_rowptr, a_col, y0,
                   name or f"sparse_rows_n{n}_m{m}_k{k}_s{seed}", dict(seed=seed))


def workload_large_m(seed: int = 0, n: int = 20000, w: int = 15, m: int = 40000,
                     nnz_per_row: int = 64) -> Instance:
    """Banded n = 20000, half-bandwidth 15 (19985 cliques of 16) with m = 40000
    sparse constraints of 64 coordinates each: the m x m factor would take
    12.8 GB per triangle, the case the conjugate-gradient affine step is for."""
    return sparse_rows_instance(n, banded_cliques(n, w), m, nnz_per_row, seed,
                                name=f"banded_n{n}_w{w}_m{m}_k{nnz_per_row}_s{seed}")


def workload_nonchordal(seed: int = 0, rows: int = 45, cols: int = 45, m: int = 200,
                        density: float = 0.05) -> Instance:
    """Stand-in for the nonchordal experiments (cone sizes about 2000-7500,
    m = 200, sparse constraints): a 45 x 45 grid (n = 2025) with m = 200 sparse
    random constraints on its pattern."""
    pr, pc = grid_pattern(rows, cols)
    return instance_on_pattern(rows * cols, pr, pc, m, seed, density=density,
                               name=f"grid{rows}x{cols}_m{m}_s{seed}")


def rescaled_instance(inst: Instance, seed: int, row_decades: float = 3.0,
                      vertex_decades: float = 1.0, obj_factor: float = 100.0) -> Instance:
    """An equivalent, badly scaled copy: A_i -> f_i T A_i T, b_i -> f_i b_i,
    C -> g T C T with T = diag(t), log10 f ~ U(-row_decades, row_decades),
    log10 t ~ U(-vertex_decades, vertex_decades), g = obj_factor.  X solves the
    copy iff T X T solves the original; the optimal value is multiplied by g."""
    rng = np.random.default_rng(seed)
    f = 10.0 ** rng.uniform(-row_decades, row_decades, inst.m)
    t = 10.0 ** rng.uniform(-vertex_decades, vertex_decades, inst.n)
    tt = t[inst.pat_row] * t[inst.pat_col]
    if inst.a_format == A_DENSE:
        a = f[:, None] * inst.a_val * tt[None, :]
    else:
        rows = np.repeat(np.arange(inst.m), np.diff(inst.a_rowptr))
        a = f[rows] * inst.a_val * tt[inst.a_col]
    return Instance(n=inst.n, m=inst.m, pat_row=inst.pat_row, pat_col=inst.pat_col,
                    clique_ptr=inst.clique_ptr, clique_vert=inst.clique_vert,
                    a_format=inst.a_format, a_val=a, b=f * inst.b, c=obj_factor * tt * inst.c,
                    a_rowptr=inst.a_rowptr, a_col=inst.a_col, name=inst.name + "_rescaled",
                    meta=dict(inst.meta, f=f, t=t, g=obj_factor))


# ----------------------------------------------------------------------------
# The five named workloads
# ----------------------------------------------------------------------------

def workload_small_blockarrow(seed: int = 0) -> Instance:
    """Block-arrow l=10, d=10, h=5 (n=105, 10 cliques of 15), m=100."""
    return block_arrow_instance(10, 10, 5, 100, seed)


def workload_banded(seed: int = 0, n: int = 2000, w: int = 15, m: int = 1000) -> Instance:
    """Banded n=2000, half-bandwidth 15 (1985 cliques of 16), m=1000."""
    return banded_instance(n, w, m, seed)


def workload_large_cliques(seed: int = 0, l: int = 40, d: int = 120, h: int = 8,
                           m: int = 4000, density: float = 0.005) -> Instance:
    """Block-arrow l=40, d=120, h=8 (40 cliques of 128), m=4000, 0.5% dense A."""
    return block_arrow_instance(l, d, h, m, seed, density=density)


def workload_batched(seeds=range(512)) -> List[Instance]:
    """512 uneven block-arrow instances, l~U[5,50], d~U[8,40], h~U[2,10]."""
    return [uneven_block_arrow_instance(s) for s in seeds]


def workload_adjoint(seeds=range(64), l=50, d=16, h=8, m=400) -> List[Instance]:
    """64 block-arrow instances l=50, d=16, h=8 (50 cliques of 24), m=400."""
    return [block_arrow_instance(l, d, h, m, s) for s in seeds]


# ----------------------------------------------------------------------------
# Small structured instances with known optima (used as pins)
# ----------------------------------------------------------------------------

def lovasz_theta_odd_cycle(n: int) -> Instance:
    """Lovasz theta SDP of the cycle C_n as a primal minimisation.

    min <-J, X>  s.t.  trace X = 1,  X_ij = 0 for every cycle edge,  X PSD.
    C = -J is dense, so the pattern is complete and there is one clique.
    """
    cliques = [np.arange(n, dtype=np.int32)]
    pat_row, pat_col = pattern_from_cliques(n, cliques)
    nnz = pat_row.shape[0]
    index = {(int(r), int(c)): j for j, (r, c) in enumerate(zip(pat_row, pat_col))}
    m = 1 + n
    a = np.zeros((m, nnz))
    for i in range(n):
        a[0, index[(i, i)]] = 1.0
    for e in range(n):
        i, j = e, (e + 1) % n
        a[1 + e, index[(max(i, j), min(i, j))]] = 1.0   # A_e = E_ij + E_ji
    b = np.zeros(m)
    b[0] = 1.0
    c = -np.ones(nnz)
    ptr, vert = cliques_to_csr(cliques)
    return Instance(n=n, m=m, pat_row=pat_row, pat_col=pat_col, clique_ptr=ptr,
                    clique_vert=vert, a_format=A_DENSE, a_val=a, b=b, c=c,
                    name=f"lovasz_C{n}")


def random_tree_edges(n: int, seed: int):
    rng = np.random.default_rng(seed)
    parent = [int(rng.integers(0, i)) for i in range(1, n)]
    w = rng.standard_normal(n - 1)
    return [(i + 1, parent[i]) for i in range(n - 1)], w


def maxcut_tree(n: int, seed: int) -> Instance:
    """MaxCut SDP relaxation on a random weighted tree.

    min sum_{edges} w_ij X_ij  s.t.  X_ii = 1,  X PSD.  The pattern is the
    tree (chordal), its maximal cliques are the edges.
    """
    edges, w = random_tree_edges(n, seed)
    cliques = [np.array(sorted(e), dtype=np.int32) for e in edges]
    pat_row, pat_col = pattern_from_cliques(n, cliques)
    nnz = pat_row.shape[0]
    index = {(int(r), int(c)): j for j, (r, c) in enumerate(zip(pat_row, pat_col))}
    a = np.zeros((n, nnz))
    for i in range(n):
        a[i, index[(i, i)]] = 1.0
    c = np.zeros(nnz)
    for (i, j), wij in zip(edges, w):
        c[index[(max(i, j), min(i, j))]] = 0.5 * wij   # <C,X> = sum w_ij X_ij
    ptr, vert = cliques_to_csr(cliques)
    return Instance(n=n, m=n, pat_row=pat_row, pat_col=pat_col, clique_ptr=ptr,
                    clique_vert=vert, a_format=A_DENSE, a_val=a, b=np.ones(n),
                    c=c, name=f"maxcut_tree_n{n}_s{seed}",
                    meta=dict(weights=w, edges=edges))


def as_single_clique(inst: Instance) -> Instance:
    """The same SDP with its pattern completed to one clique V (no decomposition).

    A and C are embedded into the complete pattern with zeros elsewhere, so the
    optimum is unchanged (Theorem 1 with the trivial chordal extension).
    """
    n = inst.n
    cliques = [np.arange(n, dtype=np.int32)]
    pr, pc = pattern_from_cliques(n, cliques)
    index = {(int(r), int(c)): j for j, (r, c) in enumerate(zip(pr, pc))}
    pos = np.array([index[(int(r), int(c))] for r, c in zip(inst.pat_row, inst.pat_col)])
    a_old = inst.a_dense()
    a = np.zeros((inst.m, pr.shape[0]))
    a[:, pos] = a_old
    c = np.zeros(pr.shape[0])
    c[pos] = inst.c
    ptr, vert = cliques_to_csr(cliques)
    return Instance(n=n, m=inst.m, pat_row=pr, pat_col=pc, clique_ptr=ptr,
                    clique_vert=vert, a_format=A_DENSE, a_val=a, b=inst.b.copy(),
                    c=c, name=inst.name + "_onecl")


def goe_blocks(sizes: Sequence[int], seed: int, dtype=np.float64) -> List[np.ndarray]:
    """Symmetric N(0,1) test blocks (Gaussian orthogonal ensemble shape)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in sizes:
        g = rng.standard_normal((s, s))
        out.append(((g + g.T) * 0.5).astype(dtype))
    return out
