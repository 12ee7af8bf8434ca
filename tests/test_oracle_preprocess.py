"""Pins of the oracle's preprocessing (chordal extension and maximal cliques,
Theorem 1 and Section 7.1.1; data scaling, Section 7.1.3) against what
graph theory and the problem's structure fix:

* the filled graph is chordal, checked by a maximum cardinality search
  (Tarjan and Yannakakis) -- an ordering independent of the elimination game;
* it contains the original edges, and the elimination order is a perfect
  elimination order of it;
* its maximal cliques equal those found by brute force over all vertex
  subsets (small graphs);
* closed forms: a chordless n-cycle gets n - 3 fill edges and n - 2 triangles;
  chordal inputs (block-arrow, banded, trees) get no fill and their own
  cliques back;
* Theorem 1 through the extension: the decomposed problem on the extension
  has the undecomposed optimum;
* scaling: the generator's certificates X = I (A(X) = b) and
  Z = C - sum y0_i A_i = I map to a feasible X' and a PSD Z' of the scaled
  problem under the stated recovery maps; the scaled optimum maps back to the
  original one; Ruiz iterations shrink the spread of row and vertex norms.
"""
import itertools

import numpy as np
import pytest

import sdpgen
from cases import oracle_extended
from oracle import preprocess as pp
from test_oracle_pins import full_sym_from_lower


def adjacency(n, edges):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    return adj


def mcs_is_chordal(n, adj):
    """Maximum cardinality search; the reverse visiting order is a perfect
    elimination order iff the graph is chordal."""
    weight = [0] * n
    visited = [False] * n
    visit = []
    for _ in range(n):
        v = max((u for u in range(n) if not visited[u]), key=lambda u: (weight[u], -u))
        visited[v] = True
        visit.append(v)
        for u in adj[v]:
            if not visited[u]:
                weight[u] += 1
    return is_perfect_elimination(list(reversed(visit)), adj)


def is_perfect_elimination(order, adj):
    pos = {v: i for i, v in enumerate(order)}
    for v in order:
        later = [u for u in adj[v] if pos[u] > pos[v]]
        for a, b in itertools.combinations(later, 2):
            if b not in adj[a]:
                return False
    return True


def brute_force_maximal_cliques(n, adj):
    cliques = []
    for mask in range(1, 1 << n):
        vs = [v for v in range(n) if mask >> v & 1]
        if all(b in adj[a] for a, b in itertools.combinations(vs, 2)):
            cliques.append(frozenset(vs))
    cs = set(cliques)
    maximal = [c for c in cliques if not any(c < d for d in cs)]
    return sorted(sorted(c) for c in maximal)


def edge_list(pr, pc):
    return [(int(r), int(c)) for r, c in zip(pr, pc) if r != c]


def patterns_small():
    out = [("cycle7", 7, *sdpgen.cycle_pattern(7)), ("grid3x4", 12, *sdpgen.grid_pattern(3, 4))]
    for seed in range(6):
        out.append((f"rand{seed}", 11, *sdpgen.random_sparse_pattern(11, 3.5, seed)))
    return out


@pytest.mark.parametrize("name,n,pr,pc", patterns_small() + [
    ("grid12", 144, *sdpgen.grid_pattern(12, 12)),
    ("rand200", 200, *sdpgen.random_sparse_pattern(200, 3.0, 9))])
def test_filled_graph_is_chordal_and_contains_the_pattern(name, n, pr, pc):
    order, later, edges = pp.elimination_game(n, pr, pc)
    orig = {(max(a, b), min(a, b)) for a, b in edge_list(pr, pc)}
    assert orig <= edges
    adj = adjacency(n, edges)
    assert mcs_is_chordal(n, adj)
    assert is_perfect_elimination(order, adj)
    assert sorted(order) == list(range(n))


@pytest.mark.parametrize("name,n,pr,pc", patterns_small())
def test_maximal_cliques_match_brute_force(name, n, pr, pc):
    er, ec, cliques = pp.chordal_extension(n, pr, pc)
    adj = adjacency(n, edge_list(er, ec))
    assert cliques == brute_force_maximal_cliques(n, adj)


def test_extended_pattern_layout():
    er, ec, cliques = pp.chordal_extension(12, *sdpgen.grid_pattern(3, 4))
    assert (er >= ec).all()
    keys = ec.astype(np.int64) * 12 + er
    assert (np.diff(keys) > 0).all()
    assert ((er == ec).sum()) == 12
    # the pattern is exactly the union of the clique pairs
    pr, pc = sdpgen.pattern_from_cliques(12, [np.array(c) for c in cliques])
    assert np.array_equal(pr, er) and np.array_equal(pc, ec)


@pytest.mark.parametrize("n", [4, 5, 9, 16])
def test_cycle_closed_form(n):
    pr, pc = sdpgen.cycle_pattern(n)
    er, ec, cliques = pp.chordal_extension(n, pr, pc)
    assert len(edge_list(er, ec)) - n == n - 3
    assert len(cliques) == n - 2 and all(len(c) == 3 for c in cliques)


@pytest.mark.parametrize("kind", ["blockarrow", "banded", "tree"])
def test_chordal_input_gets_no_fill(kind):
    if kind == "blockarrow":
        n, cl = 4 * 5 + 3, sdpgen.block_arrow_cliques(4, 5, 3)
    elif kind == "banded":
        n, cl = 30, sdpgen.banded_cliques(30, 4)
    else:
        n = 25
        edges, _ = sdpgen.random_tree_edges(n, 4)
        cl = [np.array(sorted(e), dtype=np.int32) for e in edges]
    pr, pc = sdpgen.pattern_from_cliques(n, cl)
    er, ec, cliques = pp.chordal_extension(n, pr, pc)
    assert np.array_equal(er, pr) and np.array_equal(ec, pc)
    assert cliques == sorted(sorted(int(v) for v in c) for c in cl)


@pytest.mark.parametrize("kind", ["grid", "cycle"])
def test_extension_keeps_the_optimum(oracle_mod, kind):
    """Theorem 1 through the chordal extension: Algorithm 1 on the extended,
    decomposed problem reaches the optimum of the undecomposed SDP."""
    if kind == "grid":
        pr, pc = sdpgen.grid_pattern(3, 4)
        inst = sdpgen.instance_on_pattern(12, pr, pc, 6, seed=5)
    else:
        pr, pc = sdpgen.cycle_pattern(9)
        inst = sdpgen.instance_on_pattern(9, pr, pc, 5, seed=6)
    ext = oracle_extended(inst)
    assert ext.p > 1
    one = sdpgen.as_single_clique(inst)
    Pe, Pu = oracle_mod.Problem(ext), oracle_mod.Problem(one)
    assert Pe.run(400000, tol=1e-10, adaptive=True).status == 0
    assert Pu.run(400000, tol=1e-10, adaptive=True).status == 0
    assert abs(Pe.objective() - Pu.objective()) <= 1e-6 * (1 + abs(Pu.objective()))


def block_arrow_cases():
    base = sdpgen.block_arrow_instance(3, 4, 2, 8, seed=1)
    return [base, sdpgen.rescaled_instance(base, seed=3)]


def test_scaling_maps_the_certificates():
    """For the generator's instance, X = I is feasible and C - sum y0_i A_i = I.
    Under A'_i = e_i S A_i S, b' = rho_b E b, C' = sigma_c S C S the matrix
    X' = rho_b S^-1 S^-1 is feasible and y'_i = sigma_c y0_i / e_i leaves
    C' - sum y'_i A'_i = sigma_c S^2, i.e. the recovery maps X = S X' S / rho_b
    and y = E y' / sigma_c invert these."""
    inst = sdpgen.block_arrow_instance(3, 4, 2, 8, seed=1)
    rng = np.random.default_rng(0)
    y0 = np.linalg.lstsq(inst.a_dense().T,
                         inst.c - (inst.pat_row == inst.pat_col).astype(float), rcond=None)[0]
    e, s, rb, sc = pp.equilibrate(inst, 10)
    e = e * rng.uniform(0.5, 2.0, e.shape)          # any positive scalings must work
    a, b, c = pp.scale_data(inst, e, s, rb, sc)
    diag = inst.pat_row == inst.pat_col
    Xs = np.where(diag, rb / s[inst.pat_row] ** 2, 0.0)
    w = np.where(diag, 1.0, 2.0)
    assert np.allclose(a @ (w * Xs), b, rtol=1e-12, atol=1e-12 * np.abs(b).max())
    ys = sc * y0 / e
    Z = full_sym_from_lower(inst, c - ys @ a)
    assert np.allclose(Z, np.diag(sc * s ** 2), atol=1e-10 * sc * s.max() ** 2)
    x_back, y_back, _ = pp.recover(inst, e, s, rb, sc, Xs, ys)
    assert np.allclose(x_back, diag.astype(float), atol=1e-12)
    assert np.allclose(y_back, y0, rtol=1e-12, atol=1e-12)


def test_scaled_optimum_maps_back(oracle_mod):
    inst = sdpgen.block_arrow_instance(3, 4, 2, 8, seed=1)
    P = oracle_mod.Problem(inst)
    assert P.run(400000, tol=1e-10, adaptive=True).status == 0
    e, s, rb, sc = pp.equilibrate(inst, 10)
    a, b, c = pp.scale_data(inst, e, s, rb, sc)
    scaled = sdpgen.Instance(n=inst.n, m=inst.m, pat_row=inst.pat_row, pat_col=inst.pat_col,
                             clique_ptr=inst.clique_ptr, clique_vert=inst.clique_vert,
                             a_format=0, a_val=a, b=b, c=c)
    Ps = oracle_mod.Problem(scaled)
    assert Ps.run(400000, tol=1e-10, adaptive=True).status == 0
    x, y, _ = pp.recover(inst, e, s, rb, sc, Ps.u(), Ps.y())
    w = np.where(inst.pat_row == inst.pat_col, 1.0, 2.0)
    assert abs(np.sum(w * inst.c * x) - P.objective()) <= 1e-6 * (1 + abs(P.objective()))
    assert np.allclose(inst.a_dense() @ (w * x), inst.b, atol=1e-6)


def test_ruiz_iterations_balance_the_norms():
    bad = block_arrow_cases()[1]
    As, _ = pp.dense_data(bad)

    def spread(e, s):
        Ab = e[:, None, None] * s[None, :, None] * As * s[None, None, :]
        r = np.sqrt((Ab ** 2).sum(axis=(1, 2)))
        q = np.sqrt((Ab ** 2).sum(axis=(0, 2)))
        return r.max() / r.min(), q.max() / q.min()

    r0, q0 = spread(np.ones(bad.m), np.ones(bad.n))
    e, s, _, _ = pp.equilibrate(bad, 30)
    r1, q1 = spread(e, s)
    assert r0 > 1e4 and q0 > 10
    assert r1 < 1.1 and q1 < 1.1
    assert pp.equilibrate(bad, 0)[0].tolist() == [1.0] * bad.m


def test_scaling_speeds_up_a_badly_scaled_instance(oracle_mod):
    """With the adaptive penalty (Section 7.1.2), the scaled copy of a badly
    scaled instance needs far fewer iterations than the copy itself."""
    bad = block_arrow_cases()[1]
    e, s, rb, sc = pp.equilibrate(bad, 10)
    a, b, c = pp.scale_data(bad, e, s, rb, sc)
    scaled = sdpgen.Instance(n=bad.n, m=bad.m, pat_row=bad.pat_row, pat_col=bad.pat_col,
                             clique_ptr=bad.clique_ptr, clique_vert=bad.clique_vert,
                             a_format=0, a_val=a, b=b, c=c)
    r_bad = oracle_mod.Problem(bad).run(50000, tol=1e-5, adaptive=True)
    r_sc = oracle_mod.Problem(scaled).run(50000, tol=1e-5, adaptive=True)
    assert r_sc.status == 0
    assert r_sc.iters * 5 <= r_bad.iters
