"""CPU oracle of the preprocessing steps -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use this module; the product library never does and this
module never imports it.  Plain Python and numpy in FP64, written for
reading, not speed.

Chordal extension and maximal cliques (Theorem 1, and the preprocessing of
Section 7.1.1: a symbolic Cholesky factorisation under a minimum-degree
ordering gives a chordal extension whose maximal cliques define the
decomposition).  The extension is the elimination game: repeatedly take the
remaining vertex of least current degree (ties: smallest label), record its
remaining neighbours, join them pairwise, delete it.  The union of the
original and the added edges is the filled graph.  Its maximal cliques are
the candidate sets {v} U (neighbours of v eliminated later) that no other
candidate strictly contains (every maximal clique of a graph with a perfect
elimination order is such a candidate).

Data scaling (Section 7.1.3, the problem rescaled by diagonal D, E and by
positive scalars multiplying b and C, following the cited SCS scheme).  The
paper fixes the goal -- rows of the scaled A and b near unit norm, columns of
A and c of similar norms, D preserving the cone -- but not the iteration.
The reading used here (one per-vertex positive diagonal S acting by
congruence, which keeps every clique block PSD and the pattern unchanged, and
one factor e_i per constraint):

  scaled data       A'_i = e_i S A_i S,   b'_i = rho_b e_i b_i,   C' = sigma_c S C S
  Ruiz iterations   from e = 1, s = 1, repeat ``iters`` times, with both norms
                    taken on the current scaled A before either update:
                      r_i = ||A'_i||_F,  q_v = sqrt(sum_i sum_u A'_i[v, u]^2)
                      e_i /= sqrt(r_i),  s_v /= sqrt(q_v)   (skipped where 0)
                    then clamp e and s to [1e-4, 1e4]
  scalars           rho_b   = mean_i r_i / max(||E b||_2, 1e-4)
                    sigma_c = mean_v q_v / max(||S C S||_F, 1e-4)
                    (norms of the final scaled A; both clamped to [1e-4, 1e4])
  recovery          X = S X' S / rho_b,  y = E y' / sigma_c,
                    Z = S^-1 Z' S^-1 / sigma_c
"""
from __future__ import annotations

import numpy as np

SCALE_MIN = 1e-4
SCALE_MAX = 1e4


# ---------------------------------------------------------------------------
# chordal extension (Theorem 1; Section 7.1.1)
# ---------------------------------------------------------------------------

def elimination_game(n, row, col):
    """Minimum-degree elimination.  Returns (order, later, edges): the
    elimination order, for every vertex the set of its neighbours eliminated
    after it (at the time it is eliminated), and the filled graph's edges as
    a set of (high, low) pairs."""
    adj = [set() for _ in range(n)]
    for r, c in zip(row, col):
        r, c = int(r), int(c)
        if r != c:
            adj[r].add(c)
            adj[c].add(r)
    remaining = set(range(n))
    order, later = [], [None] * n
    edges = set()
    for v in range(n):
        for u in adj[v]:
            edges.add((max(u, v), min(u, v)))
    while remaining:
        v = min(remaining, key=lambda x: (len(adj[x]), x))
        nb = set(adj[v])
        later[v] = nb
        order.append(v)
        for a in nb:
            for b in nb:
                if a > b:
                    adj[a].add(b)
                    adj[b].add(a)
                    edges.add((a, b))
            adj[a].discard(v)
        adj[v] = set()
        remaining.discard(v)
    return order, later, edges


def maximal_cliques(n, later):
    """Candidate sets {v} U later[v] not strictly inside another candidate;
    each as a sorted list, all in lexicographic order."""
    cand = [frozenset(later[v]) | {v} for v in range(n)]
    keep = []
    for i, a in enumerate(cand):
        if any(a < b for j, b in enumerate(cand) if j != i):
            continue
        keep.append(a)
    uniq = sorted({tuple(sorted(c)) for c in keep})
    return [list(c) for c in uniq]


def extended_pattern(n, edges):
    """Lower coordinates of the filled graph plus every diagonal, sorted by
    column then row."""
    coords = sorted(set(edges) | {(v, v) for v in range(n)}, key=lambda rc: (rc[1], rc[0]))
    return (np.array([r for r, _ in coords], dtype=np.int32),
            np.array([c for _, c in coords], dtype=np.int32))


def chordal_extension(n, row, col):
    """(pat_row, pat_col, cliques) of the extension of the given pattern."""
    order, later, edges = elimination_game(n, row, col)
    pr, pc = extended_pattern(n, edges)
    return pr, pc, maximal_cliques(n, later)


# ---------------------------------------------------------------------------
# data scaling (Section 7.1.3)
# ---------------------------------------------------------------------------

def _full(n, pat_row, pat_col, vals):
    M = np.zeros((n, n))
    M[pat_row, pat_col] = vals
    M[pat_col, pat_row] = vals
    return M


def dense_data(inst):
    """A_i, C as full symmetric n x n arrays (dense stacks; small cases)."""
    A = inst.a_dense()
    As = np.stack([_full(inst.n, inst.pat_row, inst.pat_col, A[i]) for i in range(inst.m)])
    return As, _full(inst.n, inst.pat_row, inst.pat_col, inst.c)


def equilibrate(inst, iters):
    """(e, s, rho_b, sigma_c) of the scaling reading in the header."""
    As, Cf = dense_data(inst)
    m, n = inst.m, inst.n
    e, s = np.ones(m), np.ones(n)

    def norms():
        Ab = e[:, None, None] * s[None, :, None] * As * s[None, None, :]
        r = np.sqrt((Ab ** 2).sum(axis=(1, 2)))
        q = np.sqrt((Ab ** 2).sum(axis=(0, 2)))
        return r, q

    for _ in range(iters):
        r, q = norms()
        e = np.where(r > 0, e / np.sqrt(np.where(r > 0, r, 1.0)), e)
        s = np.where(q > 0, s / np.sqrt(np.where(q > 0, q, 1.0)), s)
        e = np.clip(e, SCALE_MIN, SCALE_MAX)
        s = np.clip(s, SCALE_MIN, SCALE_MAX)
    r, q = norms()
    nb = np.linalg.norm(e * inst.b)
    nc = np.linalg.norm(s[:, None] * Cf * s[None, :])
    rho_b = float(np.clip(r.mean() / max(nb, SCALE_MIN), SCALE_MIN, SCALE_MAX))
    sigma_c = float(np.clip(q.mean() / max(nc, SCALE_MIN), SCALE_MIN, SCALE_MAX))
    return e, s, rho_b, sigma_c


def scale_data(inst, e, s, rho_b, sigma_c):
    """(a_dense', b', c') on the same pattern coordinates."""
    ss = s[inst.pat_row] * s[inst.pat_col]
    A = inst.a_dense()
    return (e[:, None] * A * ss[None, :], rho_b * e * inst.b, sigma_c * ss * inst.c)


def recover(inst, e, s, rho_b, sigma_c, x, y, z=None):
    """(x, y, z) of the original problem from those of the scaled one."""
    ss = s[inst.pat_row] * s[inst.pat_col]
    xo = ss * np.asarray(x) / rho_b
    yo = e * np.asarray(y) / sigma_c
    zo = None if z is None else np.asarray(z) / (ss * sigma_c)
    return xo, yo, zo
