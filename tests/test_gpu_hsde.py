"""GPU parity of Algorithm 3 (ADMM on the homogeneous self-dual embedding)
against the oracle.

Fixed-N parity from u = v = (0, ..., 0, 1): x = u_x / tau, y = u_y / tau, the
blocks u_s and v_z and the residual history agree element by element (FP64:
1e-8 relative to the largest entry; the GPU forms A u_x and A^T u_y from
quantities of the inner solve, the oracle multiplies directly, so the two
differ by rounding only; FP32-eig: 2e-4).  Solves: the same stopping
iteration (+-1) and <C, X> within 1e-6; infeasible instances end with the
same certificate status.
"""
import numpy as np
import pytest

import sdpgen
from cases import singleton_clique_instance

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def rel_err(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def hist_err(a, b):
    """rel_err over the finite entries; infinite residuals (a zero
    denominator in the consensus ratio) must sit at the same iterations."""
    a, b = np.asarray(a, float), np.asarray(b, float)
    if a.shape != b.shape or not np.array_equal(np.isinf(a), np.isinf(b)):
        return np.inf
    f = np.isfinite(b)
    return rel_err(a[f], b[f]) if f.any() else 0.0


def weights(inst):
    return np.where(inst.pat_row == inst.pat_col, 1.0, 2.0)


def oracle_hsde(oracle_mod, inst, n_iter, tol=0.0):
    P = oracle_mod.Problem(inst)
    assert P.hsde_setup() == 0
    r = P.run_hsde(n_iter, tol=tol)
    return P, r


def compare_fixed_n_hsde(sdp, oracle_mod, insts, n_iter, precision="fp64", tol_rel=1e-8):
    log(f"hsde fixed-N {[i.name for i in insts]} N={n_iter} {precision}")
    with sdp.Solver(insts, tol=0.0, max_iter=100000, precision=precision,
                    algorithm="hsde") as S:
        S.step(n_iter)
        sols = [S.solution(i) for i in range(len(insts))]
        hists = [S.history(i) for i in range(len(insts))]
    for inst, sol, (hc, he, ht) in zip(insts, sols, hists):
        P, r = oracle_hsde(oracle_mod, inst, n_iter)
        o = P.hsde_solution()
        errs = dict(x=rel_err(sol["u"], o["x"]), y=rel_err(sol["y_dual"], o["y"]),
                    s=rel_err(sol["X_packed"], sdp.pack_blocks(o["s"])),
                    z=rel_err(sol["L_packed"], sdp.pack_blocks(o["z"])),
                    eps_c=hist_err(hc, r.hist_c), eps_e=hist_err(he, r.hist_e))
        log(f"  {inst.name}: {errs} tau={o['tau']:.6g}")
        for k, v in errs.items():
            assert v <= tol_rel, (inst.name, k, v)


def test_hsde_fixed_n_small_blockarrow_fp64(sdp, gpu, oracle_mod):
    compare_fixed_n_hsde(sdp, oracle_mod, [sdpgen.workload_small_blockarrow()], 40)


def test_hsde_fixed_n_fp32(sdp, gpu, oracle_mod):
    compare_fixed_n_hsde(sdp, oracle_mod, [sdpgen.workload_small_blockarrow()], 10,
                         precision="fp32", tol_rel=2e-4)


def test_hsde_fixed_n_sparse_singleton_and_batch(sdp, gpu, oracle_mod):
    insts = [singleton_clique_instance(),
             sdpgen.block_arrow_instance(4, 6, 3, 30, seed=2, density=0.2),
             sdpgen.block_arrow_instance(6, 9, 4, 150, seed=3)]
    compare_fixed_n_hsde(sdp, oracle_mod, insts, 20)


def test_hsde_banded_workload_fixed_n(sdp, gpu, oracle_mod):
    compare_fixed_n_hsde(sdp, oracle_mod, [sdpgen.workload_banded()], 5)


@pytest.mark.parametrize("precision,obj_tol", [("fp64", 1e-6), ("fp32", 1e-4)])
def test_hsde_solve_small_blockarrow(sdp, gpu, oracle_mod, precision, obj_tol):
    inst = sdpgen.workload_small_blockarrow()
    P, r = oracle_hsde(oracle_mod, inst, 20000, tol=1e-4)
    o = P.hsde_solution()
    obj_o = float(np.sum(weights(inst) * inst.c * o["x"]))
    with sdp.Solver([inst], tol=1e-4, max_iter=20000, precision=precision,
                    algorithm="hsde") as S:
        g = S.solve()[0]
    log(f"hsde solve {precision}: oracle {r.iters} it obj={obj_o:.12g}; gpu {g['iters']} it "
        f"obj={g['objective']:.12g} eps_p={g['eps_p']:.2e} eps_d={g['eps_d']:.2e} "
        f"eps_g={g['eps_g']:.2e}")
    assert g["status"] == 0 and r.status == 0
    assert abs(g["objective"] - obj_o) <= obj_tol * abs(obj_o)
    if precision == "fp64":
        assert abs(g["iters"] - r.iters) <= 1
    assert max(g["eps_p"], g["eps_d"], g["eps_g"], g["eps_c"]) <= 1e-4


def test_hsde_lovasz_theta_on_gpu(sdp, gpu):
    n = 5
    inst = sdpgen.lovasz_theta_odd_cycle(n)
    exact = -n * np.cos(np.pi / n) / (1 + np.cos(np.pi / n))
    with sdp.Solver([inst], tol=1e-9, max_iter=200000, algorithm="hsde") as S:
        g = S.solve()[0]
    log(f"theta C5 via HSDE: {g['objective']:.12f} exact {exact:.12f} iters {g['iters']}")
    assert g["status"] == 0
    assert abs(g["objective"] - exact) <= 1e-7 * abs(exact)


def test_hsde_certificates_on_gpu(sdp, gpu, oracle_mod):
    """A feasible, a primal-infeasible and a dual-infeasible instance in one
    batch: each ends with the oracle's status and stopping iteration (+-1);
    the certificates satisfy their defining conditions."""
    insts = [sdpgen.block_arrow_instance(3, 3, 2, 5, seed=1),
             sdpgen.primal_infeasible_instance(3, 3, 2, 5, seed=1),
             sdpgen.dual_infeasible_instance(3, 3, 2, 5, seed=2)]
    with sdp.Solver(insts, tol=1e-6, max_iter=100000, algorithm="hsde") as S:
        gs = S.solve()
        sols = [S.solution(i) for i in range(3)]
    expect = [0, sdp.PRIMAL_INFEASIBLE, sdp.DUAL_INFEASIBLE]
    for inst, g, sol, e in zip(insts, gs, sols, expect):
        P, r = oracle_hsde(oracle_mod, inst, 100000, tol=1e-6)
        log(f"  {inst.name}: gpu status {g['status']} after {g['iters']}, oracle {r.status} "
            f"after {r.iters}")
        assert g["status"] == e and r.status == e
        assert abs(g["iters"] - r.iters) <= 1
    w = weights(insts[2])
    y = sols[1]["y_dual"] / (insts[1].b @ sols[1]["y_dual"])
    from test_oracle_pins import full_sym_from_lower
    Sm = full_sym_from_lower(insts[1], -(y @ insts[1].a_val))
    assert np.linalg.eigvalsh(Sm).min() >= -1e-4 * max(1.0, np.abs(Sm).max())
    x = -sols[2]["u"] / np.sum(w * insts[2].c * sols[2]["u"])
    assert np.linalg.norm(insts[2].a_val @ (w * x)) <= 1e-4


def test_hsde_fixed_n_fp32_blocks_of_64_with_decoupling(sdp, gpu, oracle_mod):
    """Algorithm 3 in the FP32-eig form on cliques of 64: the warm-started
    projections take the positive/negative decoupling (on by default)."""
    inst = sdpgen.block_arrow_instance(3, 58, 6, 40, seed=5)
    compare_fixed_n_hsde(sdp, oracle_mod, [inst], 40, precision="fp32", tol_rel=2e-4)
