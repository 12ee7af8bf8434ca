"""Positive/negative decoupling of warm-started projections (option decouple;
FP32-eig, blocks padded to 64 and more): the refinements replace the Jacobi
sweeps only where a Gershgorin bound certifies the result, so the iterates
must match the oracle as closely as with sweeps alone:

* fixed-N parity with the oracle (FP32-eig: 2e-4 relative to the largest
  entry) for blocks of 64 and 128 and for a batch of mixed clique sizes; with
  FP64 or small blocks the option changes nothing (FP64: 1e-8);
* the decoupled path is taken: far fewer Jacobi sweeps per projection than
  with sweeps alone;
* a solve to 1e-4 stops within a few iterations of the sweep-only solve and
  reaches the same objective.
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


def parity(sdp, oracle_mod, insts, n_iter, precision, tol_rel):
    with sdp.Solver(insts, tol=0.0, max_iter=100000, precision=precision, decouple=1) as S:
        S.step(n_iter)
        sols = [S.solution(i) for i in range(len(insts))]
        hists = [S.history(i) for i in range(len(insts))]
        st = S.stats()
    log(f"{[i.name for i in insts]} {precision}: sweeps per projection "
        f"{st['jacobi_sweeps'] / max(st['projections'], 1):.3f}")
    for inst, sol, (hc, hl, _) in zip(insts, sols, hists):
        P = oracle_mod.Problem(inst)
        r = P.run(n_iter, tol=0.0)
        Xo, Lo = P.blocks()
        assert max(np.abs(x).max() for x in Xo) > 0, "projections all zero: nothing tested"
        errs = dict(u=rel_err(sol["u"], P.u()), y=rel_err(sol["y_dual"], P.y_dual()),
                    X=rel_err(sol["X_packed"], sdp.pack_blocks(Xo)),
                    L=rel_err(sol["L_packed"], sdp.pack_blocks(Lo)),
                    eps_c=rel_err(hc, r.hist_eps_c), eps_l=rel_err(hl, r.hist_eps_l))
        log(f"  {inst.name}: {errs}")
        for k, v in errs.items():
            assert v <= tol_rel, (inst.name, k, v)
    return st


@pytest.mark.parametrize("precision,tol_rel", [("fp64", 1e-8), ("fp32", 2e-4)])
def test_decouple_leaves_blocks_of_16_alone(sdp, gpu, oracle_mod, precision, tol_rel):
    inst = sdpgen.sparse_rows_instance(300, sdpgen.banded_cliques(300, 15), 200, 30, seed=4)
    parity(sdp, oracle_mod, [inst], 60, precision, tol_rel)


@pytest.mark.parametrize("precision,tol_rel", [("fp64", 1e-8), ("fp32", 2e-4)])
def test_decouple_fixed_n_blocks_of_64(sdp, gpu, oracle_mod, precision, tol_rel):
    inst = sdpgen.block_arrow_instance(3, 58, 6, 40, seed=5)
    parity(sdp, oracle_mod, [inst], 40, precision, tol_rel)


def test_decouple_fixed_n_fp32_blocks_of_128(sdp, gpu, oracle_mod):
    inst = sdpgen.block_arrow_instance(3, 112, 8, 60, seed=6, density=0.05)
    parity(sdp, oracle_mod, [inst], 40, "fp32", 2e-4)


def test_decouple_fixed_n_mixed_batch(sdp, gpu, oracle_mod):
    insts = [sdpgen.block_arrow_instance(4, 5, 2, 12, seed=3),
             sdpgen.block_arrow_instance(3, 26, 4, 50, seed=8),
             sdpgen.block_arrow_instance(2, 70, 6, 30, seed=9)]
    parity(sdp, oracle_mod, insts, 50, "fp32", 2e-4)


def test_decouple_takes_the_refinement_path(sdp, gpu):
    """Once the warm start settles, most projections are certified after the
    refinements and run no sweep."""
    inst = sdpgen.block_arrow_instance(6, 58, 6, 100, seed=1)
    rates = {}
    for dec in (0, 1):
        with sdp.Solver([inst], tol=0.0, max_iter=100000, precision="fp32", decouple=dec,
                        projection_method="scalar") as S:
            S.step(150)
            before = S.stats()
            S.step(50)
            after = S.stats()
        rates[dec] = ((after["jacobi_sweeps"] - before["jacobi_sweeps"])
                      / max(after["projections"] - before["projections"], 1))
    log(f"sweeps per projection, iterations 150-200: sweeps only {rates[0]:.3f}, "
        f"with decoupling {rates[1]:.3f}")
    assert rates[1] < rates[0] and rates[1] <= 0.5


def test_decouple_solve_matches_sweeps(sdp, gpu):
    inst = sdpgen.block_arrow_instance(4, 58, 6, 60, seed=2)
    out = {}
    for dec in (0, 1):
        with sdp.Solver([inst], tol=1e-4, max_iter=20000, precision="fp32",
                        projection_method="scalar", decouple=dec) as S:
            out[dec] = S.solve()[0]
    log(f"solve fp32: sweeps only {out[0]['iters']} it obj {out[0]['objective']:.10g}; "
        f"decoupling {out[1]['iters']} it obj {out[1]['objective']:.10g}")
    assert out[1]["status"] == 0
    assert abs(out[1]["iters"] - out[0]["iters"]) <= max(3, 0.01 * out[0]["iters"])
    assert abs(out[1]["objective"] - out[0]["objective"]) <= 1e-6 * abs(out[0]["objective"])


def test_decouple_plans_scalar_variants_for_large_blocks(sdp, gpu):
    """With the decoupling on (the default) the FP32 blocks of 64 and more take
    the scalar variants, which carry it; with it off the autotuner may take
    the two-level ones."""
    inst = sdpgen.block_arrow_instance(3, 70, 6, 30, seed=9)
    with sdp.Solver([inst], precision="fp32") as S:
        kinds = [sdp.projection_variant_two_level(sdp.DTYPE_FP32, v)
                 for v in S.projection_plan_variants()]
    log(f"decouple on: two-level per bucket {kinds}")
    assert not any(kinds)


def test_decouple_with_failing_certificates_reaches_oracle_optimum(sdp, gpu, oracle_mod):
    """The nonchordal workload's extension in the FP32-eig form: its cliques
    of 64 to 76 vertices fail the decoupling certificate near convergence
    (both eigenvalue groups reach zero), so the attempts back off, and after
    two failures in a row the matrix sign function carries those cliques
    (blocks of up to 96) while they wait.  The solve to 1e-4 still stops
    within a few iterations of the FP64 oracle and reaches its objective to
    1e-4."""
    from cases import as_instance
    ext = as_instance(sdp.extend_instance(sdpgen.workload_nonchordal()))
    P = oracle_mod.Problem(ext)
    r = P.run(20000, tol=1e-4)
    assert r.status == 0
    with sdp.Solver([ext], tol=1e-4, max_iter=20000, precision="fp32", decouple=1) as S:
        g = S.solve()[0]
        st = S.stats()
    log(f"nonchordal fp32: gpu {g['iters']} it obj {g['objective']:.10g} "
        f"(sweeps per projection {st['jacobi_sweeps'] / max(st['projections'], 1):.3f}, "
        f"{st['sign_fallbacks']} sign-function fallbacks); "
        f"oracle {r.iters} it obj {P.objective():.10g}")
    assert st["sign_fallbacks"] > 0
    assert g["status"] == 0
    assert abs(g["iters"] - r.iters) <= max(3, 0.01 * r.iters)
    assert abs(g["objective"] - P.objective()) <= 1e-4 * abs(P.objective())


def _nonchordal_extension(sdp):
    from cases import as_instance
    return as_instance(sdp.extend_instance(sdpgen.workload_nonchordal()))


def test_sign_fallback_fixed_n_matches_oracle(sdp, gpu, oracle_mod):
    """Fixed-N parity through the sign-function fallback: 1400 FP32-eig
    iterations of the nonchordal extension, long enough for its cliques of
    65 to 76 vertices (padded to 80) to fail the certificate twice in a row
    and take the fallback (counted in the stats); X, Lambda, u and the
    residual history then match the FP64 oracle.  Bar: each FP32 projection
    is accurate to ~1e-6 ||W||_F (sweep tolerance, sign iteration resolving
    eigenvalues down to 3^-13 ||W||_F) and the ADMM map is nonexpansive, so
    N iterations differ by at most ~N * 1e-6 relative: 1.5e-6 N."""
    ext = _nonchordal_extension(sdp)
    n_iter = 1400
    st = parity(sdp, oracle_mod, [ext], n_iter, "fp32", 1.5e-6 * n_iter)
    log(f"  sign-function fallbacks: {st['sign_fallbacks']}")
    assert st["sign_fallbacks"] > 0


def test_reset_restores_decoupling_back_off_bitwise(sdp, gpu):
    """sdp_reset returns every clique's decoupling back-off to its initial
    state: after a run long enough for certificate failures (and sign-function
    fallbacks), a reset and the same run again reproduce a fresh handle's
    iterates bit for bit; so does sdp_set_state with the zero state."""
    ext = _nonchordal_extension(sdp)
    n = 1400
    with sdp.Solver([ext], tol=0.0, max_iter=100000, precision="fp32", decouple=1) as S:
        S.step(n)
        first = S.solution(0)
        st1 = S.stats()
        S.reset()
        S.step(n)
        second = S.solution(0)
        st2 = S.stats()
        S.set_state(0, np.zeros(S.npk[0]), np.zeros(S.npk[0]), 1.0)
        S.step(n)
        third = S.solution(0)
    log(f"  fallbacks: first run {st1['sign_fallbacks']}, after reset {st2['sign_fallbacks']}")
    assert st1["sign_fallbacks"] > 0 and st2["sign_fallbacks"] == st1["sign_fallbacks"]
    for key in ("u", "X_packed", "L_packed", "y_dual"):
        assert np.array_equal(first[key], second[key]), key
        assert np.array_equal(first[key], third[key]), key
