"""The two-level (block) Jacobi variants inside the iteration, forced with
projection_method = 2 (the autotuner picks them only where they are faster):

* the launch plan uses two-level variants for the large cliques;
* fixed-N parity with the oracle, FP64 (1e-8 relative to the largest entry)
  on cliques of 64 and 72 (blocks of 64 and 80) and FP32-eig (2e-4) on cliques
  of 120 (blocks of 128), with warm-started eigensolves and the Newton-Schulz
  basis update;
* the unrolled differentiation (eigenvectors stored by the forward sweep)
  gives the same VJP as with the scalar method: the projection adjoint does
  not depend on the eigenvector basis the solver returns.
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


def plan_kinds(sdp, S, precision):
    dt = sdp.DTYPE_FP32 if precision == "fp32" else sdp.DTYPE_FP64
    return [(n, sdp.projection_variant_two_level(dt, v))
            for (n, _, _), v in zip(S.projection_plan(), S.projection_plan_variants())]


def parity(sdp, oracle_mod, inst, n_iter, precision, tol_rel):
    P = oracle_mod.Problem(inst)
    r = P.run(n_iter, tol=0.0)
    with sdp.Solver([inst], tol=0.0, max_iter=100000, precision=precision,
                    projection_method="two_level") as S:
        kinds = plan_kinds(sdp, S, precision)
        S.step(n_iter)
        sol = S.solution(0)
        hc, hl, _ = S.history(0)
    log(f"{inst.name} {precision}: plan {kinds}")
    assert all(k for n, k in kinds if n >= 64), kinds
    Xo, Lo = P.blocks()
    assert max(np.abs(x).max() for x in Xo) > 0, "projections all zero: nothing tested"
    errs = dict(u=rel_err(sol["u"], P.u()), y=rel_err(sol["y_dual"], P.y_dual()),
                X=rel_err(sol["X_packed"], sdp.pack_blocks(Xo)),
                L=rel_err(sol["L_packed"], sdp.pack_blocks(Lo)),
                eps_c=rel_err(hc, r.hist_eps_c), eps_l=rel_err(hl, r.hist_eps_l))
    log(f"  errors {errs}")
    for k, v in errs.items():
        assert v <= tol_rel, (k, v)


@pytest.mark.parametrize("d,h", [(58, 6), (66, 6)])
def test_two_level_fixed_n_fp64(sdp, gpu, oracle_mod, d, h):
    inst = sdpgen.block_arrow_instance(3, d, h, 40, seed=5)
    parity(sdp, oracle_mod, inst, 12, "fp64", 1e-8)


def test_two_level_fixed_n_fp32_blocks_of_128(sdp, gpu, oracle_mod):
    inst = sdpgen.block_arrow_instance(3, 112, 8, 60, seed=6, density=0.05)
    parity(sdp, oracle_mod, inst, 40, "fp32", 2e-4)


def test_two_level_vjp_matches_scalar_method(sdp, gpu):
    import torch
    dev = torch.device("cuda:0")
    inst = sdpgen.block_arrow_instance(3, 58, 6, 30, seed=7)
    rng = np.random.default_rng(1)
    ubar = torch.from_numpy(rng.standard_normal(inst.nnz)).to(dev)
    res = {}
    for method in ("scalar", "two_level"):
        with sdp.Solver([inst], rho=1.0, tol=0.0, max_iter=10 ** 6,
                        projection_method=method) as S:
            u = torch.zeros(S.total_nnz, dtype=torch.float64, device=dev)
            S.unrolled_forward(20, 5, u)
            cb = torch.zeros(S.total_nnz, dtype=torch.float64, device=dev)
            bb = torch.zeros(S.total_m, dtype=torch.float64, device=dev)
            S.vjp(ubar, cb, bb)
            torch.cuda.synchronize()
            res[method] = (u.cpu().numpy(), cb.cpu().numpy(), bb.cpu().numpy())
    for name, a, b in zip(("u", "c_bar", "b_bar"), res["two_level"], res["scalar"]):
        e = rel_err(a, b)
        log(f"two-level vs scalar {name}: {e:.2e}")
        assert e <= 1e-8, (name, e)
