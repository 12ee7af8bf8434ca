"""Pins of the oracle's Algorithm 3 (ADMM for the homogeneous self-dual
embedding, Section 5) against what the paper and the mathematics fix:

* the inner system M sigma = nu (SecondBlockElimination) and one whole
  iteration (HsdeStep1-3 with the outer system LinearSystem) against dense
  numpy solves of the explicitly built Q (HSDEnotations) on the full pattern
  vector (both triangles, so no compact-coordinate weights enter the
  reference);
* closed-form optima (Lovasz theta, MaxCut on trees) and agreement with
  Algorithm 1;
* infeasibility certificates checked with dense eigh: a primal-infeasible
  instance gives y with b^T y = 1 and -sum y_i A_i PSD up to the tolerance; a
  dual-infeasible one gives X with A(X) ~ 0, <C, X> = -1 and PSD clique
  blocks.
"""
import numpy as np
import pytest

import sdpgen
from test_oracle_pins import full_sym_from_lower, numpy_psd, rand_sym


def weights(inst):
    return np.where(inst.pat_row == inst.pat_col, 1.0, 2.0)


class FullSpace:
    """The pattern E* with both triangles as explicit vector entries, the
    selectors H_k of full s_k x s_k blocks and A, c on that space."""

    def __init__(self, inst):
        self.inst = inst
        ent = []
        for r, c in zip(inst.pat_row, inst.pat_col):
            ent.append((int(r), int(c)))
            if r != c:
                ent.append((int(c), int(r)))
        self.ent = ent
        self.idx = {e: i for i, e in enumerate(ent)}
        self.nf = len(ent)
        lower = {(int(r), int(c)): j for j, (r, c) in enumerate(zip(inst.pat_row, inst.pat_col))}
        self.comp = np.array([lower[(max(r, c), min(r, c))] for r, c in ent])
        A = inst.a_dense()
        self.A = A[:, self.comp]
        self.c = inst.c[self.comp]
        rows = []
        for k in range(inst.p):
            v = inst.clique(k)
            for a in range(len(v)):          # row-major over the block: entry (a, b)
                for b in range(len(v)):
                    rows.append(self.idx[(int(v[a]), int(v[b]))])
        self.H = np.zeros((len(rows), self.nf))
        self.H[np.arange(len(rows)), rows] = 1.0
        self.nd = len(rows)

    def from_compact(self, u):
        return np.asarray(u)[self.comp]

    def to_compact(self, x):
        out = np.zeros(self.inst.nnz)
        out[self.comp] = x                    # symmetric: both positions agree
        return out


def cat(blocks):
    return np.concatenate([np.asarray(b).ravel() for b in blocks])


def random_state(inst, rng, sym_x=True):
    p = inst.p
    sz = [len(inst.clique(k)) for k in range(p)]
    return (rng.standard_normal(inst.nnz), [rand_sym(rng, s) for s in sz],
            rng.standard_normal(inst.m), [rand_sym(rng, s) for s in sz],
            [rand_sym(rng, s) for s in sz])


@pytest.mark.parametrize("shape", [(2, 2, 1, 3), (3, 3, 2, 5)])
def test_inner_system_matches_dense_solve(oracle_mod, shape):
    l, d, h, m = shape
    inst = sdpgen.block_arrow_instance(l, d, h, m, seed=2)
    F = FullSpace(inst)
    rng = np.random.default_rng(7)
    nx, ns, ny, nt, _ = random_state(inst, rng)
    nf, nd = F.nf, F.nd
    Ahat = np.zeros((m + nd, nf + nd))
    Ahat[:m, :nf] = F.A
    Ahat[m:, :nf] = F.H
    Ahat[m:, nf:] = -np.eye(nd)
    Mm = np.block([[np.eye(nf + nd), -Ahat.T], [Ahat, np.eye(m + nd)]])
    rhs = np.concatenate([F.from_compact(nx), cat(ns), ny, cat(nt)])
    sol = np.linalg.solve(Mm, rhs)
    P = oracle_mod.Problem(inst)
    assert P.hsde_setup() == 0
    sx, ss, sy, st = P.hsde_inner(nx, ns, ny, nt)
    assert np.allclose(F.from_compact(sx), sol[:nf], atol=1e-10)
    assert np.allclose(cat(ss), sol[nf:nf + nd], atol=1e-10)
    assert np.allclose(sy, sol[nf + nd:nf + nd + m], atol=1e-10)
    assert np.allclose(cat(st), sol[nf + nd + m:], atol=1e-10)


@pytest.mark.parametrize("shape", [(2, 2, 1, 3), (3, 3, 2, 5)])
def test_one_iteration_matches_dense_embedding(oracle_mod, shape):
    """u_hat = (I + Q)^-1 (u + v), u = P_K(u_hat - v), v = v - u_hat + u with Q
    built explicitly (HSDEnotations)."""
    l, d, h, m = shape
    inst = sdpgen.block_arrow_instance(l, d, h, m, seed=4)
    F = FullSpace(inst)
    rng = np.random.default_rng(8)
    ux, us, uy, ut, vz = random_state(inst, rng)
    tau, kappa = 0.7, 0.4
    nf, nd = F.nf, F.nd
    N = nf + nd + m + nd + 1
    Q = np.zeros((N, N))
    ix, is_, iy, it_, itau = (slice(0, nf), slice(nf, nf + nd), slice(nf + nd, nf + nd + m),
                              slice(nf + nd + m, N - 1), N - 1)
    Q[ix, iy] = -F.A.T
    Q[ix, it_] = -F.H.T
    Q[ix, itau] = F.c
    Q[is_, it_] = np.eye(nd)
    Q[iy, ix] = F.A
    Q[iy, itau] = -inst.b
    Q[it_, ix] = F.H
    Q[it_, is_] = -np.eye(nd)
    Q[itau, ix] = -F.c
    Q[itau, iy] = inst.b
    u = np.concatenate([F.from_compact(ux), cat(us), uy, cat(ut), [tau]])
    v = np.zeros(N)
    v[is_] = cat(vz)
    v[itau] = kappa
    uh = np.linalg.solve(np.eye(N) + Q, u + v)
    w = uh - v
    un = w.copy()
    o = nf
    for k in range(inst.p):
        s = len(inst.clique(k))
        un[o:o + s * s] = numpy_psd(w[o:o + s * s].reshape(s, s)).ravel()
        o += s * s
    un[itau] = max(w[itau], 0.0)
    vn = v - uh + un
    P = oracle_mod.Problem(inst)
    P.hsde_setup()
    P.hsde_set(ux, us, uy, ut, vz, tau, kappa)
    P.run_hsde(1, tol=0.0)
    sol = P.hsde_solution()
    rx, ry = P.hsde_raw()
    assert np.allclose(F.from_compact(rx), un[ix], atol=1e-10)
    assert np.allclose(cat(sol["s"]), un[is_], atol=1e-10)
    assert np.allclose(ry, un[iy], atol=1e-10)
    assert np.allclose(cat(sol["t"]), un[it_], atol=1e-10)
    assert np.isclose(sol["tau"], un[itau], atol=1e-12)
    assert np.allclose(cat(sol["z"]), vn[is_], atol=1e-10)
    assert np.isclose(sol["kappa"], vn[itau], atol=1e-12)
    # v stays in the dual cone's zero parts
    assert np.allclose(vn[ix], 0, atol=1e-10) and np.allclose(vn[iy], 0, atol=1e-10)


@pytest.mark.parametrize("n", [5, 7, 9])
def test_hsde_lovasz_theta(oracle_mod, n):
    inst = sdpgen.lovasz_theta_odd_cycle(n)
    P = oracle_mod.Problem(inst)
    P.hsde_setup()
    r = P.run_hsde(200000, tol=1e-10)
    assert r.status == 0
    sol = P.hsde_solution()
    exact = -n * np.cos(np.pi / n) / (1 + np.cos(np.pi / n))
    assert abs(np.sum(weights(inst) * inst.c * sol["x"]) - exact) <= 1e-7 * abs(exact)
    assert abs(inst.b @ sol["y"] - exact) <= 1e-7 * abs(exact)


def test_hsde_maxcut_tree(oracle_mod):
    inst = sdpgen.maxcut_tree(25, seed=1)
    P = oracle_mod.Problem(inst)
    P.hsde_setup()
    assert P.run_hsde(200000, tol=1e-10).status == 0
    exact = -np.abs(inst.meta["weights"]).sum()
    assert abs(np.sum(weights(inst) * inst.c * P.hsde_solution()["x"]) - exact) <= 1e-7 * abs(exact)


@pytest.mark.parametrize("shape", [(3, 3, 2, 6, 4), (4, 4, 2, 9, 7)])
def test_hsde_agrees_with_algorithm_1(oracle_mod, shape):
    l, d, h, m, seed = shape
    inst = sdpgen.block_arrow_instance(l, d, h, m, seed)
    P = oracle_mod.Problem(inst)
    P.hsde_setup()
    r = P.run_hsde(400000, tol=1e-10)
    assert r.status == 0
    Pp = oracle_mod.Problem(inst)
    assert Pp.run(400000, tol=1e-10, adaptive=True).status == 0
    sol = P.hsde_solution()
    obj = np.sum(weights(inst) * inst.c * sol["x"])
    assert abs(obj - Pp.objective()) <= 1e-6 * (1 + abs(Pp.objective()))
    assert max(sol["eps_p"], sol["eps_d"], sol["eps_g"], sol["eps_c"]) <= 1e-10
    Z = full_sym_from_lower(inst, inst.c - sol["y"] @ inst.a_val)
    assert np.linalg.eigvalsh(Z).min() >= -1e-6


def test_hsde_certifies_primal_infeasibility(oracle_mod):
    inst = sdpgen.primal_infeasible_instance(3, 3, 2, 5, seed=1)
    P = oracle_mod.Problem(inst)
    P.hsde_setup()
    r = P.run_hsde(100000, tol=1e-6)
    assert r.status == 2
    _, uy = P.hsde_raw()
    y = uy / (inst.b @ uy)
    assert np.isclose(inst.b @ y, 1.0)
    # Farkas: -sum y_i A_i is PSD (to the tolerance) while b^T y = 1 > 0
    S = full_sym_from_lower(inst, -(y @ inst.a_val))
    assert np.linalg.eigvalsh(S).min() >= -1e-4 * max(1.0, np.abs(S).max())


def test_hsde_certifies_dual_infeasibility(oracle_mod):
    inst = sdpgen.dual_infeasible_instance(3, 3, 2, 5, seed=2)
    P = oracle_mod.Problem(inst)
    P.hsde_setup()
    r = P.run_hsde(100000, tol=1e-6)
    assert r.status == 3
    ux, _ = P.hsde_raw()
    w = weights(inst)
    x = -ux / np.sum(w * inst.c * ux)
    assert np.isclose(np.sum(w * inst.c * x), -1.0)
    assert np.linalg.norm(inst.a_val @ (w * x)) <= 1e-4
    for k in range(inst.p):
        v = inst.clique(k)
        Xf = full_sym_from_lower(inst, x)[np.ix_(v, v)]
        assert np.linalg.eigvalsh(Xf).min() >= -1e-4 * max(1.0, np.abs(Xf).max())


def test_feasible_instances_are_not_reported_infeasible(oracle_mod):
    for seed in range(3):
        inst = sdpgen.block_arrow_instance(3, 3, 2, 5, seed)
        P = oracle_mod.Problem(inst)
        P.hsde_setup()
        assert P.run_hsde(20000, tol=1e-6).status == 0
