"""GPU parity of Algorithm 1 with the conjugate-gradient affine step (the
iterative alternative to the factor, Section 4.1.1) against the oracle's
PCG mode.

* Fixed-N parity with a fixed number of PCG steps per iteration (cg_tol = 0,
  so both sides take exactly the same steps): u, y_dual, the clique blocks and
  the residual history element by element (FP64: 1e-8 relative to the
  largest entry; FP32-eig: 2e-4), for dense A, sparse A and a batch of
  instances with different m; the step counts agree exactly.
* A tolerance-driven solve reaches the factor-based optimum.
* At the large-m workload (m = 40000, beyond the factor's reach) the oracle
  runs without a factor; a few iterations match it element by element, and
  with a tight PCG tolerance every x-update satisfies A(x) = b.
"""
import numpy as np
import pytest

import sdpgen

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def rel_err(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def compare_cg(sdp, oracle_mod, insts, n_iter, K, precision="fp64", tol_rel=1e-8, factor=True):
    log(f"cg fixed-N {[i.name for i in insts]} N={n_iter} K={K} {precision}")
    with sdp.Solver(insts, tol=0.0, max_iter=100000, precision=precision, cg_max_iter=K,
                    cg_tol=0.0) as S:
        S.step(n_iter)
        sols = [S.solution(i) for i in range(len(insts))]
        hists = [S.history(i) for i in range(len(insts))]
        steps = S.cg_steps()
    total = 0
    for inst, sol, (hc, hl, _) in zip(insts, sols, hists):
        P = oracle_mod.Problem(inst, factor=factor)
        P.set_affine_cg(K, 0.0)
        r = P.run(n_iter, tol=0.0)
        total += P.cg_steps()
        Xo, Lo = P.blocks()
        errs = dict(u=rel_err(sol["u"], P.u()), y=rel_err(sol["y_dual"], P.y_dual()),
                    X=rel_err(sol["X_packed"], sdp.pack_blocks(Xo)),
                    L=rel_err(sol["L_packed"], sdp.pack_blocks(Lo)),
                    eps_c=rel_err(hc, r.hist_eps_c), eps_l=rel_err(hl, r.hist_eps_l))
        log(f"  {inst.name}: {errs}")
        for k, v in errs.items():
            assert v <= tol_rel, (inst.name, k, v)
    assert steps == total, (steps, total)


def test_cg_fixed_n_dense(sdp, gpu, oracle_mod):
    compare_cg(sdp, oracle_mod, [sdpgen.workload_small_blockarrow()], 30, K=3)


def test_cg_fixed_n_fp32(sdp, gpu, oracle_mod):
    compare_cg(sdp, oracle_mod, [sdpgen.workload_small_blockarrow()], 10, K=3, precision="fp32",
               tol_rel=2e-4)


def test_cg_fixed_n_sparse_and_batch(sdp, gpu, oracle_mod):
    insts = [sdpgen.block_arrow_instance(4, 5, 2, 12, seed=3, density=0.3),
             sdpgen.block_arrow_instance(6, 9, 4, 150, seed=4),
             sdpgen.sparse_rows_instance(300, sdpgen.banded_cliques(300, 7), 700, 24, seed=5)]
    compare_cg(sdp, oracle_mod, insts, 15, K=4)


def test_cg_one_step_on_diagonal_gram(sdp, gpu, oracle_mod):
    """MaxCut on a tree: A D^-1 A^T is diagonal, one PCG step is exact, so the
    iterates equal the factor-based ones."""
    inst = sdpgen.maxcut_tree(40, seed=3)
    compare_cg(sdp, oracle_mod, [inst], 25, K=1)
    P = oracle_mod.Problem(inst)
    P.run(25, tol=0.0)
    with sdp.Solver([inst], tol=0.0, max_iter=1000, cg_max_iter=1) as S:
        S.step(25)
        u = S.solution(0)["u"]
    assert rel_err(u, P.u()) <= 1e-10


def test_cg_solve_reaches_factor_optimum(sdp, gpu, oracle_mod):
    inst = sdpgen.workload_small_blockarrow()
    P = oracle_mod.Problem(inst)
    assert P.run(20000, tol=1e-6).status == 0
    with sdp.Solver([inst], tol=1e-6, max_iter=20000, cg_max_iter=10, cg_tol=1e-10) as S:
        g = S.solve()[0]
        steps = S.cg_steps()
    log(f"cg solve: {g['iters']} it, {steps} PCG steps, obj {g['objective']:.10g} "
        f"(factor {P.objective():.10g})")
    assert g["status"] == 0
    assert abs(g["objective"] - P.objective()) <= 1e-5 * abs(P.objective())
    assert 0 < steps <= 10 * g["iters"]


def test_large_m_workload_parity_and_feasibility(sdp, gpu, oracle_mod):
    """m = 40000 sparse constraints (n = 20000, 19985 cliques of 16)."""
    inst = sdpgen.workload_large_m()
    compare_cg(sdp, oracle_mod, [inst], 3, K=3, factor=False)
    with sdp.Solver([inst], tol=0.0, max_iter=1000, cg_max_iter=200, cg_tol=1e-13) as S:
        S.step(2)
        u = S.solution(0)["u"]
    w = np.where(inst.pat_row == inst.pat_col, 1.0, 2.0)
    rows = np.repeat(np.arange(inst.m), np.diff(inst.a_rowptr))
    ax = np.bincount(rows, weights=inst.a_val * (w * u)[inst.a_col], minlength=inst.m)
    res = np.linalg.norm(ax - inst.b) / (1 + np.linalg.norm(inst.b))
    log(f"large-m: ||A(x) - b|| / (1 + ||b||) = {res:.3e}")
    assert res <= 1e-9


def test_cg_rejections(sdp, gpu):
    inst = sdpgen.block_arrow_instance(3, 3, 2, 5, seed=0)
    with pytest.raises(sdp.SdpError) as e:
        sdp.Solver([inst], cg_max_iter=3, algorithm="dual")
    assert e.value.code == -7
    with sdp.Solver([inst], cg_max_iter=3) as S:
        with pytest.raises(sdp.SdpError) as e:
            S.unrolled_forward(5, 5)
        assert e.value.code == -7
    # the factor path refuses what only the CG path can hold
    big = sdpgen.sparse_rows_instance(2200, sdpgen.banded_cliques(2200, 3), 20500, 4, seed=1)
    assert sdp.setup_status([big]) == -7
