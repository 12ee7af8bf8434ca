"""GPU parity of Algorithm 2 (range-space dual ADMM) against the oracle.

Fixed-N parity from the same start (z_k = lambda_k = v_k = 0): the primal
estimate -rho x, y, z_k, lambda_k and the residual history agree element by
element (FP64: 1e-8 relative to the largest entry; FP32-eig: 2e-4).  Solves
to 1e-4: same iteration count (+-1) and dual objective b^T y within 1e-6
(FP64) or 1e-4 (FP32-eig).  Closed-form optima (Lovasz theta) pin the GPU
path directly.
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


def weights(inst):
    return np.where(inst.pat_row == inst.pat_col, 1.0, 2.0)


def compare_fixed_n_dual(sdp, oracle_mod, insts, n_iter, precision="fp64", rho=1.0,
                         tol_rel=1e-8, **opts):
    log(f"dual fixed-N {[i.name for i in insts]} N={n_iter} {precision} {opts}")
    with sdp.Solver(insts, rho=rho, tol=0.0, max_iter=100000, precision=precision,
                    algorithm="dual", **opts) as S:
        S.step(n_iter)
        sols = [S.solution(i) for i in range(len(insts))]
        hists = [S.history(i) for i in range(len(insts))]
    for inst, sol, (hc, hl, _) in zip(insts, sols, hists):
        P = oracle_mod.Problem(inst, rho0=rho)
        r = P.run_dual(n_iter, tol=0.0)
        Z, L = P.blocks()
        errs = dict(u=rel_err(sol["u"], -P.rho * P.u()), y=rel_err(sol["y_dual"], P.y()),
                    Z=rel_err(sol["X_packed"], sdp.pack_blocks(Z)),
                    L=rel_err(sol["L_packed"], sdp.pack_blocks(L)),
                    eps_c=rel_err(hc, r.hist_eps_c), eps_l=rel_err(hl, r.hist_eps_l))
        log(f"  {inst.name}: {errs}")
        for k, v in errs.items():
            assert v <= tol_rel, (inst.name, k, v)


def test_dual_fixed_n_small_blockarrow_fp64(sdp, gpu, oracle_mod):
    compare_fixed_n_dual(sdp, oracle_mod, [sdpgen.workload_small_blockarrow()], 40)


def test_dual_fixed_n_fp32(sdp, gpu, oracle_mod):
    compare_fixed_n_dual(sdp, oracle_mod, [sdpgen.workload_small_blockarrow()], 10,
                         precision="fp32", tol_rel=2e-4)


def test_dual_fixed_n_sparse_a_singleton_cliques_and_batch(sdp, gpu, oracle_mod):
    insts = [singleton_clique_instance(),
             sdpgen.block_arrow_instance(4, 6, 3, 30, seed=2, density=0.2),
             sdpgen.block_arrow_instance(6, 9, 4, 150, seed=3)]
    compare_fixed_n_dual(sdp, oracle_mod, insts, 20, rho=0.7)


@pytest.mark.parametrize("method", ["scalar", "sign"])
def test_dual_fixed_n_both_projection_paths(sdp, gpu, oracle_mod, method):
    """The z-update on the warm-started Jacobi kernels and on the register
    sign-function kernels (cliques of 8, 13, 24 and 31: both block sizes),
    FP64 at 1e-8 and FP32-eig at 2e-4."""
    from test_gpu_admm_sign import arrow_with_blocks
    inst = arrow_with_blocks([4, 9, 20, 27], 4, 40, seed=11)
    with sdp.Solver([inst], algorithm="dual", projection_method=method) as S:
        dt = sdp.DTYPE_FP64
        kinds = {sdp.projection_variant_kind(dt, v) for v in S.projection_plan_variants()}
    assert kinds == ({2} if method == "sign" else {0})
    compare_fixed_n_dual(sdp, oracle_mod, [inst], 30, rho=0.9, projection_method=method)
    compare_fixed_n_dual(sdp, oracle_mod, [inst], 30, rho=0.9, precision="fp32", tol_rel=2e-4,
                         projection_method=method)


def test_dual_banded_workload_fixed_n(sdp, gpu, oracle_mod):
    """The n = 2000 banded workload at full size, 6 iterations of Algorithm 2."""
    compare_fixed_n_dual(sdp, oracle_mod, [sdpgen.workload_banded()], 6)


@pytest.mark.parametrize("precision,obj_tol", [("fp64", 1e-6), ("fp32", 1e-4)])
def test_dual_solve_small_blockarrow(sdp, gpu, oracle_mod, precision, obj_tol):
    inst = sdpgen.workload_small_blockarrow()
    P = oracle_mod.Problem(inst)
    r = P.run_dual(20000, tol=1e-4)
    with sdp.Solver([inst], tol=1e-4, max_iter=20000, precision=precision,
                    algorithm="dual") as S:
        g = S.solve()[0]
        d = S.diagnostics()[0]
    log(f"dual solve {precision}: oracle {r.iters} it b'y={P.dual_objective():.12g}; "
        f"gpu {g['iters']} it b'y={g['objective']:.12g}; eps_p={d['eps_p']:.2e}")
    assert g["status"] == 0 and r.status == 0
    assert abs(g["objective"] - P.dual_objective()) <= obj_tol * abs(P.dual_objective())
    if precision == "fp64":
        assert abs(g["iters"] - r.iters) <= 1
    # -rho x satisfies the constraints to rounding (A x = -b / rho in every iteration)
    assert d["eps_p"] <= 1e-9


@pytest.mark.parametrize("n", [5, 7])
def test_dual_lovasz_theta_closed_form_on_gpu(sdp, gpu, n):
    inst = sdpgen.lovasz_theta_odd_cycle(n)
    exact = -n * np.cos(np.pi / n) / (1 + np.cos(np.pi / n))
    with sdp.Solver([inst], tol=1e-10, max_iter=200000, adaptive_rho=1,
                    algorithm="dual") as S:
        g = S.solve()[0]
    log(f"theta C{n} via b'y: gpu {g['objective']:.12f} exact {exact:.12f}")
    assert g["status"] == 0
    assert abs(g["objective"] - exact) <= 1e-7 * abs(exact)


def test_dual_and_primal_reach_the_same_optimum_on_gpu(sdp, gpu):
    inst = sdpgen.block_arrow_instance(3, 4, 2, 7, seed=9)
    with sdp.Solver([inst], tol=1e-9, max_iter=400000, adaptive_rho=1,
                    algorithm="dual") as S:
        gd = S.solve()[0]
        xd = S.solution(0)["u"]
    with sdp.Solver([inst], tol=1e-9, max_iter=400000, adaptive_rho=1) as S:
        gp = S.solve()[0]
    assert abs(gd["objective"] - gp["objective"]) <= 1e-6 * (1 + abs(gp["objective"]))
    assert abs(np.sum(weights(inst) * inst.c * xd) - gp["objective"]) <= 1e-6 * (
        1 + abs(gp["objective"]))


def test_dual_rejects_unrolled_differentiation(sdp, gpu):
    import torch
    inst = sdpgen.workload_small_blockarrow()
    with sdp.Solver([inst], tol=0.0, algorithm="dual") as S:
        u = torch.zeros(S.total_nnz, dtype=torch.float64, device="cuda:0")
        with pytest.raises(sdp.SdpError) as e:
            S.unrolled_forward(5, 5, u)
        assert e.value.code == -7


def test_dual_fixed_n_fp32_blocks_of_64_with_decoupling(sdp, gpu, oracle_mod):
    """Algorithm 2 in the FP32-eig form on cliques of 64: the warm-started
    projections take the positive/negative decoupling (on by default)."""
    inst = sdpgen.block_arrow_instance(3, 58, 6, 40, seed=5)
    compare_fixed_n_dual(sdp, oracle_mod, [inst], 40, precision="fp32", tol_rel=2e-4)
