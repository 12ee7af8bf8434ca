"""Pins of the oracle's conjugate-gradient affine step (the iterative
alternative to factorising A D^-1 A^T named in Section 4.1.1) against what
the mathematics fixes:

* many PCG steps solve (A D^-1 A^T) y = rhs as a dense solve does, with the
  matrix built from the paper's definitions on the full vectorised pattern
  (both triangles, D = sum_k H_k^T H_k, no compact-coordinate weights);
* the recursive residuals equal rhs - M y_j recomputed explicitly;
* the M-norm of the error never grows (CG's optimality property);
* a diagonal A D^-1 A^T (the MaxCut family, Section 4.1.1) is solved in one
  step, since the Jacobi preconditioner is then the matrix itself;
* Algorithm 1 with PCG to a tight tolerance reproduces the factor-based
  iterates; with a few steps per iteration it reaches the same optimum.
"""
import numpy as np
import pytest

import sdpgen
from test_oracle_hsde import FullSpace


def gram_full(inst):
    F = FullSpace(inst)
    Dfull = np.diag(F.H.T @ F.H)
    return F.A @ np.diag(1.0 / Dfull) @ F.A.T


def cg_problem(oracle_mod, inst, K=1, tol=0.0):
    P = oracle_mod.Problem(inst)
    P.set_affine_cg(K, tol)
    return P


@pytest.mark.parametrize("shape", [(3, 4, 2, 8, 1), (4, 3, 3, 15, 2)])
def test_pcg_matches_dense_solve(oracle_mod, shape):
    l, d, h, m, seed = shape
    inst = sdpgen.block_arrow_instance(l, d, h, m, seed)
    M = gram_full(inst)
    rhs = np.random.default_rng(seed).standard_normal(m)
    P = cg_problem(oracle_mod, inst)
    y, hist = P.pcg(rhs, np.zeros(m), 200, 1e-13 * np.linalg.norm(rhs))
    assert np.allclose(y, np.linalg.solve(M, rhs), rtol=1e-10, atol=1e-11)
    assert hist[-1] <= 1e-13 * np.linalg.norm(rhs)
    assert len(hist) - 1 <= m + 5


def test_pcg_recursive_residual_is_the_true_residual(oracle_mod):
    inst = sdpgen.block_arrow_instance(4, 3, 3, 15, 2)
    M = gram_full(inst)
    rng = np.random.default_rng(3)
    rhs, y0 = rng.standard_normal(15), rng.standard_normal(15)
    P = cg_problem(oracle_mod, inst)
    for K in range(0, 7):
        y, hist = P.pcg(rhs, y0, K)
        assert len(hist) == K + 1
        assert np.isclose(hist[-1], np.linalg.norm(rhs - M @ y), rtol=1e-9, atol=1e-12)
    y, _ = P.pcg(rhs, y0, 0)
    assert np.array_equal(y, y0)


def test_pcg_energy_error_never_grows(oracle_mod):
    inst = sdpgen.block_arrow_instance(4, 3, 3, 15, 2)
    M = gram_full(inst)
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal(15)
    ystar = np.linalg.solve(M, rhs)
    P = cg_problem(oracle_mod, inst)
    errs = []
    for K in range(0, 16):        # m = 15: exact after at most 15 steps
        y, _ = P.pcg(rhs, np.zeros(15), K)
        e = y - ystar
        errs.append(float(np.sqrt(e @ M @ e)))
    assert all(b <= a * (1 + 1e-12) + 1e-14 for a, b in zip(errs, errs[1:]))
    assert errs[-1] <= 1e-8 * errs[0]


def test_diagonal_gram_is_solved_in_one_step(oracle_mod):
    """MaxCut on a tree: every A_i = e_i e_i^T, so A D^-1 A^T is diagonal."""
    inst = sdpgen.maxcut_tree(12, seed=2)
    M = gram_full(inst)
    assert np.allclose(M, np.diag(np.diag(M)))
    rhs = np.random.default_rng(1).standard_normal(inst.m)
    P = cg_problem(oracle_mod, inst)
    y, hist = P.pcg(rhs, np.zeros(inst.m), 1)
    assert np.allclose(y, rhs / np.diag(M), rtol=1e-13)
    # Algorithm 1 with one PCG step per iteration equals the factor-based run
    Pc, Pf = cg_problem(oracle_mod, inst, K=1), oracle_mod.Problem(inst)
    Pc.run(40, tol=0.0)
    Pf.run(40, tol=0.0)
    assert np.allclose(Pc.u(), Pf.u(), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("sparse", [False, True])
def test_tight_pcg_reproduces_factor_iterates(oracle_mod, sparse):
    inst = sdpgen.block_arrow_instance(4, 5, 2, 12, seed=3, density=0.3 if sparse else None)
    Pc, Pf = cg_problem(oracle_mod, inst, K=300, tol=1e-15), oracle_mod.Problem(inst)
    Pc.run(30, tol=0.0)
    Pf.run(30, tol=0.0)
    scale = np.abs(Pf.u()).max()
    assert np.abs(Pc.u() - Pf.u()).max() <= 1e-9 * scale
    assert np.abs(Pc.y_dual() - Pf.y_dual()).max() <= 1e-9 * np.abs(Pf.y_dual()).max()


def test_few_pcg_steps_reach_the_same_optimum(oracle_mod):
    inst = sdpgen.workload_small_blockarrow()
    Pc, Pf = cg_problem(oracle_mod, inst, K=3), oracle_mod.Problem(inst)
    rc, rf = Pc.run(20000, tol=1e-8), Pf.run(20000, tol=1e-8)
    assert rc.status == 0 and rf.status == 0
    assert abs(Pc.objective() - Pf.objective()) <= 1e-6 * abs(Pf.objective())
    assert Pc.cg_steps() <= 3 * rc.iters


def test_warm_start_at_the_solution_takes_no_step(oracle_mod):
    inst = sdpgen.block_arrow_instance(3, 4, 2, 8, 1)
    rhs = np.random.default_rng(2).standard_normal(8)
    ystar = np.linalg.solve(gram_full(inst), rhs)
    P = cg_problem(oracle_mod, inst)
    y, hist = P.pcg(rhs, ystar, 10, 1e-9)
    assert len(hist) == 1 and hist[0] <= 1e-9
    assert np.array_equal(y, ystar)


def test_invalid_cg_settings(oracle_mod):
    P = oracle_mod.Problem(sdpgen.block_arrow_instance(2, 2, 1, 3, 0))
    with pytest.raises(Exception):
        P.set_affine_cg(-1, 0.0)
    with pytest.raises(Exception):
        P.set_affine_cg(3, -1.0)


def test_factorless_problem_runs_the_same_cg_iterates(oracle_mod):
    """A problem created without the factor (the large-m case) runs Algorithm 1
    in conjugate-gradient mode exactly as a factored one does, and refuses
    the factor-based iteration."""
    inst = sdpgen.block_arrow_instance(4, 5, 2, 12, seed=3, density=0.3)
    Pa, Pb = oracle_mod.Problem(inst), oracle_mod.Problem(inst, factor=False)
    Pa.set_affine_cg(3, 0.0)
    Pb.set_affine_cg(3, 0.0)
    Pa.run(20, tol=0.0)
    Pb.run(20, tol=0.0)
    assert np.array_equal(Pa.u(), Pb.u())
    Pc = oracle_mod.Problem(inst, factor=False)
    assert Pc.run(5, tol=0.0).status == oracle_mod.ERR_ARG
