"""Algorithm 1 with the register-resident sign-function projection
(the default plan, or projection_method = "sign": cliques of up to 32
vertices, X_k = P+(W_k) =
(W_k + W_k sign(W_k)) / 2 in one wave's registers, Lambda_k += rho (X_k - H_k x)
and the residual partials in the same kernel) against the FP64 oracle.

Fixed-N bars as for the Jacobi kernels: FP64 1e-8 relative to the largest
entry (the sign iteration resolves eigenvalues down to 3^-30 ||W||_F and
converges to ~1e-15); FP32-eig 2e-4 (each projection accurate to ~1e-7 ||W||_F,
P+ is 1-Lipschitz, and the iterates amplify it at most like the Jacobi path's
1e-6 sweep tolerance)."""
import numpy as np
import pytest

import sdpgen
from test_gpu_admm import compare_fixed_n, log, rel_err, solve_both

pytestmark = pytest.mark.gpu


def arrow_with_blocks(blocks, h, m, seed):
    """Block-arrow pattern with blocks of the given sizes and a head of h
    vertices (listed last): clique k is block k plus the head."""
    cliques, v = [], 0
    n = sum(blocks) + h
    head = np.arange(n - h, n, dtype=np.int32)
    for d in blocks:
        cliques.append(np.concatenate([np.arange(v, v + d, dtype=np.int32), head]))
        v += d
    return sdpgen.random_instance(n, cliques, m, seed=seed,
                                  name=f"arrow_blocks{'_'.join(map(str, blocks))}_h{h}_m{m}")


def sign_plan(sdp, inst, precision):
    with sdp.Solver([inst], tol=0.0, precision=precision, projection_method="sign") as S:
        dt = sdp.DTYPE_FP32 if precision == "fp32" else sdp.DTYPE_FP64
        return [(n, t, c, sdp.projection_variant_kind(dt, v))
                for (n, t, c), v in zip(S.projection_plan(), S.projection_plan_variants())]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 2e-4)])
def test_sign_fixed_n_banded_blocks_of_16(sdp, gpu, oracle_mod, precision, tol):
    inst = sdpgen.banded_instance(300, 15, 120, seed=4)
    plan = sign_plan(sdp, inst, precision)
    log(f"  plan {plan}")
    assert plan == [(16, 64, inst.p, 2)]
    compare_fixed_n(sdp, oracle_mod, inst, 30, precision=precision, tol_rel=tol,
                    projection_method="sign")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 2e-4)])
def test_sign_fixed_n_mixed_blocks_up_to_32(sdp, gpu, oracle_mod, precision, tol):
    """Cliques of 9, 13, 16, 17, 24 and 31 vertices: both register kernels
    (16 and 32), padding inside each, odd sizes."""
    inst = arrow_with_blocks([5, 9, 12, 13, 20, 27], 4, 60, seed=7)
    sizes = np.diff(inst.clique_ptr)
    log(f"  clique sizes {sorted(set(sizes.tolist()))}")
    assert sizes.max() <= 32 and sizes.min() <= 16 < sizes.max()
    plan = sign_plan(sdp, inst, precision)
    assert all(k == 2 for *_, k in plan) and sum(c for _, _, c, _ in plan) == inst.p
    compare_fixed_n(sdp, oracle_mod, inst, 25, precision=precision, tol_rel=tol, rho=0.8,
                    projection_method="sign")


def test_sign_fixed_n_singleton_and_sparse(sdp, gpu, oracle_mod):
    from cases import singleton_clique_instance
    compare_fixed_n(sdp, oracle_mod, singleton_clique_instance(), 25, rho=0.7,
                    projection_method="sign")
    inst = sdpgen.block_arrow_instance(4, 6, 3, 30, seed=2, density=0.2)
    compare_fixed_n(sdp, oracle_mod, inst, 25, precision="fp32", tol_rel=2e-4,
                    projection_method="sign")


def test_sign_larger_cliques_keep_jacobi(sdp, gpu, oracle_mod):
    """Cliques above 32 vertices stay on the Jacobi variants under
    projection_method = "sign"; the mixed plan still matches the oracle."""
    inst = arrow_with_blocks([10, 30, 40, 7], 4, 50, seed=8)
    sizes = np.diff(inst.clique_ptr)
    plan = sign_plan(sdp, inst, "fp32")
    log(f"  sizes {sorted(set(sizes.tolist()))} plan {plan}")
    for n, t, c, k in plan:
        assert (k == 2) == (n <= 32)
    compare_fixed_n(sdp, oracle_mod, inst, 15, precision="fp32", tol_rel=2e-4,
                    projection_method="sign")


def test_sign_diagnostics_and_unrolled_use_eigen_paths(sdp, gpu, oracle_mod):
    """The minimum-eigenvalue pass of the diagnostics runs the Jacobi kernels
    of the same block size under a sign-function plan, with the same results
    as a Jacobi plan (the unrolled forward, which records eigenvectors, is
    covered by the adjoint tests, whose plans are sign-function plans too)."""
    inst = sdpgen.block_arrow_instance(5, 8, 3, 25, seed=6)
    out = {}
    for method in ("scalar", "sign"):
        with sdp.Solver([inst], tol=0.0, precision="fp64", projection_method=method) as S:
            S.step(12)
            out[method] = S.diagnostics()[0]
    for k in ("eps_p", "eps_d", "eps_g", "eps_alpha"):
        a, b = out["scalar"][k], out["sign"][k]
        assert abs(a - b) <= 1e-8 * max(abs(a), abs(b)) + 1e-12, (k, a, b)


@pytest.mark.timeout(600)
def test_sign_solve_banded_workload_matches_oracle(sdp, gpu, oracle_mod):
    """The banded workload (n = 2000, 1985 cliques of 16, m = 1000) solved to
    1e-4 with the sign-function projections: objective within 1e-4 of the
    oracle's (FP32) and 1e-6 (FP64), the oracle's iteration count +-1 in FP64."""
    inst = sdpgen.workload_banded()
    P = oracle_mod.Problem(inst)
    r = P.run(20000, tol=1e-4)
    for precision, obj_tol, it_tol in (("fp64", 1e-6, 1), ("fp32", 1e-4, 5)):
        with sdp.Solver([inst], tol=1e-4, max_iter=20000, precision=precision,
                        projection_method="sign") as S:
            g = S.solve()[0]
            u = S.solution(0)["u"]
        rel = abs(g["objective"] - P.objective()) / abs(P.objective())
        log(f"  {precision}: gpu iters={g['iters']} obj={g['objective']:.12g} | oracle iters="
            f"{r.iters} obj={P.objective():.12g} | rel={rel:.2e} u err={rel_err(u, P.u()):.2e}")
        assert g["status"] == 0 and r.status == 0
        assert rel <= obj_tol
        assert abs(g["iters"] - r.iters) <= it_tol
