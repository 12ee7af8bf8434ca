"""GPU parity of the whole Algorithm 1 iteration against the oracle.

Fixed-N parity: after N iterations from the same start (X_k = Lambda_k = 0,
same rho), u, y_dual, X_k, Lambda_k and the residual history agree element by
element (FP64: 1e-8 relative to the largest entry; the two sides sum in
different orders).  Solve parity at 1e-4: FP64 objective within 1e-6
relative (the bar for the plain form), FP32-eig within 1e-4 (the bar for the
FP32 form).  Closed-form optima (Lovasz theta, MaxCut on trees) pin the GPU
path directly.
"""
import numpy as np
import pytest

import sdpgen
from cases import rank_deficient_instance, singleton_clique_instance

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def packed_oracle_blocks(P):
    import paper_1707_05058_amd as sdp
    X, L = P.blocks()
    return sdp.pack_blocks(X), sdp.pack_blocks(L)


def rel_err(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def compare_fixed_n(sdp, oracle_mod, inst, n_iter, precision="fp64", rho=1.0, tol_rel=1e-8,
                    graph_chunk=25, **opts):
    log(f"fixed-N parity {inst.name} N={n_iter} precision={precision} {opts}")
    P = oracle_mod.Problem(inst, rho0=rho)
    r = P.run(n_iter, tol=0.0)
    with sdp.Solver([inst], rho=rho, tol=0.0, max_iter=100000, precision=precision,
                    graph_chunk=graph_chunk, **opts) as S:
        S.step(n_iter)
        sol = S.solution(0)
        hc, hl, hr = S.history(0)
    Xo, Lo = packed_oracle_blocks(P)
    errs = dict(u=rel_err(sol["u"], P.u()), y=rel_err(sol["y_dual"], P.y_dual()),
                X=rel_err(sol["X_packed"], Xo), L=rel_err(sol["L_packed"], Lo),
                eps_c=rel_err(hc, r.hist_eps_c), eps_l=rel_err(hl, r.hist_eps_l))
    log(f"  errors {errs}")
    for k, v in errs.items():
        assert v <= tol_rel, (k, v)
    assert len(hc) == n_iter


def test_fixed_n_small_blockarrow_fp64(sdp, gpu, oracle_mod):
    compare_fixed_n(sdp, oracle_mod, sdpgen.workload_small_blockarrow(), 40)


def test_fixed_n_without_graphs_matches(sdp, gpu, oracle_mod):
    compare_fixed_n(sdp, oracle_mod, sdpgen.workload_small_blockarrow(), 7, graph_chunk=0)


def test_fixed_n_small_blockarrow_fp32(sdp, gpu, oracle_mod):
    compare_fixed_n(sdp, oracle_mod, sdpgen.workload_small_blockarrow(), 10, precision="fp32",
                    tol_rel=2e-4)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 2e-4)])
def test_fixed_n_small_blockarrow_jacobi_path(sdp, gpu, oracle_mod, precision, tol):
    """The warm-started Jacobi kernels of the small blocks (the path that
    projection_method = "scalar", Algorithms 2 and 3 and the unrolled
    iterations take; the default plan runs the sign function there)."""
    compare_fixed_n(sdp, oracle_mod, sdpgen.workload_small_blockarrow(), 30,
                    precision=precision, tol_rel=tol, projection_method="scalar")


def test_fixed_n_singleton_and_odd_cliques(sdp, gpu, oracle_mod):
    compare_fixed_n(sdp, oracle_mod, singleton_clique_instance(), 25, rho=0.7)


def test_fixed_n_sparse_a(sdp, gpu, oracle_mod):
    inst = sdpgen.block_arrow_instance(4, 6, 3, 30, seed=2, density=0.2)
    assert inst.a_format == sdpgen.A_CSR
    compare_fixed_n(sdp, oracle_mod, inst, 25)


def test_fixed_n_many_rows_and_multi_block_factor(sdp, gpu, oracle_mod):
    """m = 150 > 128 exercises several 64-blocks of the Cholesky/inverse and
    several row tiles; |E_l| > 128 several column tiles with a ragged tail."""
    inst = sdpgen.block_arrow_instance(6, 9, 4, 150, seed=3)
    compare_fixed_n(sdp, oracle_mod, inst, 20)


def solve_both(sdp, oracle_mod, inst, precision, tol=1e-4, adaptive=False, rho=1.0):
    P = oracle_mod.Problem(inst, rho0=rho)
    r = P.run(20000, tol=tol, adaptive=adaptive)
    with sdp.Solver([inst], rho=rho, tol=tol, max_iter=20000, precision=precision,
                    adaptive_rho=int(adaptive)) as S:
        g = S.solve()[0]
    return P, r, g


@pytest.mark.parametrize("precision,obj_tol", [("fp64", 1e-6), ("fp32", 1e-4)])
def test_solve_small_blockarrow(sdp, gpu, oracle_mod, precision, obj_tol):
    inst = sdpgen.workload_small_blockarrow()
    log(f"solve {inst.name} {precision}")
    P, r, g = solve_both(sdp, oracle_mod, inst, precision)
    log(f"  oracle iters={r.iters} obj={P.objective():.12g}  gpu iters={g['iters']} "
        f"obj={g['objective']:.12g}")
    assert g["status"] == 0 and r.status == 0
    assert abs(g["objective"] - P.objective()) <= obj_tol * abs(P.objective())
    if precision == "fp64":
        assert abs(g["iters"] - r.iters) <= 1
    assert max(g["eps_c"], g["eps_lambda"]) <= 1e-4


def test_adaptive_rho_decisions_match(sdp, gpu, oracle_mod):
    inst = sdpgen.workload_small_blockarrow()
    P, r, g = solve_both(sdp, oracle_mod, inst, "fp64", adaptive=True, rho=40.0)
    assert np.any(r.hist_rho != 40.0)
    with sdp.Solver([inst], rho=40.0, tol=1e-4, precision="fp64", adaptive_rho=1) as S:
        S.solve()
        _, _, hr = S.history(0)
    k = min(len(hr), len(r.hist_rho))
    assert np.array_equal(hr[:k], r.hist_rho[:k])
    assert abs(g["objective"] - P.objective()) <= 1e-6 * abs(P.objective())


@pytest.mark.parametrize("n", [5, 7, 9])
def test_lovasz_theta_closed_form_on_gpu(sdp, gpu, n):
    inst = sdpgen.lovasz_theta_odd_cycle(n)
    exact = -n * np.cos(np.pi / n) / (1 + np.cos(np.pi / n))
    with sdp.Solver([inst], tol=1e-10, max_iter=200000, adaptive_rho=1) as S:
        g = S.solve()[0]
    log(f"theta C{n}: gpu {g['objective']:.12f} exact {exact:.12f} iters {g['iters']}")
    assert g["status"] == 0
    assert abs(g["objective"] - exact) <= 1e-7 * abs(exact)


def test_maxcut_tree_closed_form_on_gpu(sdp, gpu):
    inst = sdpgen.maxcut_tree(40, seed=4)
    exact = -np.abs(inst.meta["weights"]).sum()
    with sdp.Solver([inst], tol=1e-10, max_iter=200000, adaptive_rho=1) as S:
        g = S.solve()[0]
    assert abs(g["objective"] - exact) <= 1e-7 * abs(exact)


def test_batched_uneven_instances_match_individual_oracle_runs(sdp, gpu, oracle_mod):
    insts = [sdpgen.uneven_block_arrow_instance(s, l_range=(2, 6), d_range=(3, 12),
                                                h_range=(1, 4)) for s in range(6)]
    log("batched: " + ", ".join(i.name for i in insts))
    with sdp.Solver(insts, tol=1e-4, max_iter=20000, precision="fp64") as S:
        gs = S.solve()
        sols = [S.solution(i) for i in range(len(insts))]
    for inst, g, sol in zip(insts, gs, sols):
        P = oracle_mod.Problem(inst)
        r = P.run(20000, tol=1e-4)
        assert abs(g["iters"] - r.iters) <= 1, (inst.name, g["iters"], r.iters)
        assert abs(g["objective"] - P.objective()) <= 1e-6 * max(1.0, abs(P.objective()))
        assert rel_err(sol["u"], P.u()) <= 1e-5


def test_diagnostics_match_oracle(sdp, gpu, oracle_mod):
    inst = sdpgen.workload_small_blockarrow()
    P = oracle_mod.Problem(inst)
    P.run(20000, tol=1e-4)
    do = P.diagnostics()
    with sdp.Solver([inst], tol=1e-4) as S:
        S.solve()
        g = S.diagnostics()[0]
    for k in ("eps_p", "eps_d", "eps_g", "eps_alpha"):
        log(f"  {k}: gpu {g[k]:.6e} oracle {do[k]:.6e}")
    assert abs(g["eps_d"] - do["eps_d"]) <= 1e-6 * max(do["eps_d"], 1e-12) + 1e-12
    assert abs(g["eps_g"] - do["eps_g"]) <= 1e-6 * max(do["eps_g"], 1e-12) + 1e-12
    assert abs(g["eps_alpha"] - do["eps_alpha"]) <= 1e-6 * max(do["eps_alpha"], 1e-12) + 1e-12
    assert g["eps_p"] <= 1e-9 and do["eps_p"] <= 1e-9


def test_reset_reproduces_bitwise(sdp, gpu):
    inst = sdpgen.workload_small_blockarrow()
    with sdp.Solver([inst], tol=1e-4) as S:
        a = S.solve()[0]
        ua = S.solution(0)["u"]
        S.reset()
        b = S.solve()[0]
        ub = S.solution(0)["u"]
    assert a["iters"] == b["iters"] and a["objective"] == b["objective"]
    assert np.array_equal(ua, ub)


def test_rank_deficient_detected_on_gpu(sdp, gpu):
    assert sdp.setup_status([rank_deficient_instance()]) == -5


def test_warm_start_state_roundtrip(sdp, gpu, oracle_mod):
    """sdp_set_state then one step equals the oracle's step from the same state."""
    inst = sdpgen.workload_small_blockarrow()
    P = oracle_mod.Problem(inst)
    P.run(15, tol=0.0)
    Xo, Lo = packed_oracle_blocks(P)
    with sdp.Solver([inst], tol=0.0, max_iter=1000) as S:
        S.set_state(0, Xo, Lo, P.rho)
        S.step(3)
        sol = S.solution(0)
    P.run(3, tol=0.0)
    assert rel_err(sol["u"], P.u()) <= 1e-9


def test_banded_workload_fixed_n_fp64_and_fp32(sdp, gpu, oracle_mod):
    """The n=2000 banded workload (1985 cliques of 16, m=1000) at full size:
    8 iterations element by element in FP64; FP32-eig within 1e-4."""
    inst = sdpgen.workload_banded()
    compare_fixed_n(sdp, oracle_mod, inst, 8, tol_rel=1e-8)
    compare_fixed_n(sdp, oracle_mod, inst, 8, precision="fp32", tol_rel=1e-4)
    compare_fixed_n(sdp, oracle_mod, inst, 8, precision="fp32", tol_rel=1e-4,
                    projection_method="scalar")


def test_large_clique_workload_fixed_n_fp32(sdp, gpu, oracle_mod):
    """n=4808 block-arrow with 40 cliques of 128 and sparse A (m=4000, 0.5%
    density) at full size: FP32-eig iterates against the FP64 oracle."""
    inst = sdpgen.workload_large_cliques()
    compare_fixed_n(sdp, oracle_mod, inst, 2, precision="fp32", tol_rel=2e-4)


def test_batched_workload_shapes_fixed_n_fp64(sdp, gpu, oracle_mod):
    """The first 6 instances of the 512-instance batched workload (uneven
    clique sizes 10..50, m up to ~1000) in one handle, iterate by iterate."""
    insts = sdpgen.workload_batched(range(6))
    log("batched shapes: " + ", ".join(i.name for i in insts))
    n_iter = 6
    with sdp.Solver(insts, tol=0.0, max_iter=1000, precision="fp64") as S:
        S.step(n_iter)
        sols = [S.solution(i) for i in range(len(insts))]
    for inst, sol in zip(insts, sols):
        P = oracle_mod.Problem(inst)
        P.run(n_iter, tol=0.0)
        Xo, Lo = packed_oracle_blocks(P)
        errs = dict(u=rel_err(sol["u"], P.u()), y=rel_err(sol["y_dual"], P.y_dual()),
                    X=rel_err(sol["X_packed"], Xo), L=rel_err(sol["L_packed"], Lo))
        log(f"  {inst.name}: {errs}")
        for k, v in errs.items():
            assert v <= 1e-8, (inst.name, k, v)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotuned_plan_covers_every_clique_and_matches_default(sdp, gpu, precision):
    """The launch plan (autotuned or default) holds every clique once, in a
    block size that fits it; both plans give the same iterates up to rounding."""
    insts = [sdpgen.uneven_block_arrow_instance(s, l_range=(2, 6), d_range=(3, 40),
                                                h_range=(1, 8)) for s in range(4)]
    sizes = np.concatenate([np.diff(i.clique_ptr) for i in insts])
    res = {}
    for tune in (0, 1):
        with sdp.Solver(insts, tol=0.0, max_iter=1000, precision=precision,
                        autotune=tune) as S:
            plan = S.projection_plan()
            log(f"autotune={tune} plan={plan}")
            assert sum(c for _, _, c in plan) == len(sizes)
            assert min(N for N, _, _ in plan) >= 16
            S.step(12)
            res[tune] = np.concatenate([S.solution(i)["u"] for i in range(len(insts))])
    tol = 1e-9 if precision == "fp64" else 1e-4
    assert rel_err(res[1], res[0]) <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_warm_started_eigensolves_match_cold_and_take_fewer_sweeps(sdp, gpu, oracle_mod,
                                                                   precision, tol):
    """Starting each clique's Jacobi from last iteration's basis computes the
    same projection (fixed-N parity against the oracle) with fewer sweeps."""
    inst = sdpgen.workload_small_blockarrow()
    P = oracle_mod.Problem(inst)
    P.run(60, tol=0.0)
    sweeps = {}
    for warm in (0, 1):
        with sdp.Solver([inst], tol=0.0, max_iter=1000, precision=precision,
                        warm_start=warm, projection_method="scalar") as S:
            S.step(60)
            u = S.solution(0)["u"]
            st = S.stats()
            sweeps[warm] = st["jacobi_sweeps"] / st["projections"]
        assert rel_err(u, P.u()) <= tol, (warm, rel_err(u, P.u()))
    log(f"sweeps per projection: cold {sweeps[0]:.2f} warm {sweeps[1]:.2f}")
    assert sweeps[1] < 0.8 * sweeps[0]


def run_batch(sdp, insts, n, single_steps, **opts):
    with sdp.Solver(insts, tol=1e-3, max_iter=100000, **opts) as S:
        if single_steps:
            for _ in range(n):
                res = S.step(1)
        else:
            res = S.step(n)
        out = []
        for i in range(len(insts)):
            sol = S.solution(i)
            out.append((res[i]["iters"], res[i]["status"], sol["u"], sol["X_packed"],
                        sol["L_packed"], np.asarray(S.history(i)[0]), np.asarray(S.history(i)[1])))
    return out


@pytest.mark.parametrize("opts", [dict(graph_chunk=25), dict(graph_chunk=0),
                                  dict(graph_chunk=25, cg_max_iter=3)])
def test_folded_residuals_equal_single_steps(sdp, gpu, opts):
    """With a fixed penalty the scatter kernel of an iteration also finishes
    the previous one; a sequence of n iterations must equal n separate calls
    (each a sequence of one, no folding) bit for bit, including instances of
    a batch that stop at different iterations inside the sequence."""
    insts = [sdpgen.block_arrow_instance(3, 5, 2, 12, seed=1),
             sdpgen.block_arrow_instance(5, 8, 3, 40, seed=2),
             sdpgen.workload_small_blockarrow()]
    n = 130
    a = run_batch(sdp, insts, n, False, **opts)
    b = run_batch(sdp, insts, n, True, **opts)
    iters = [x[0] for x in a]
    log(f"folded vs single steps {opts}: iterations {iters}, status {[x[1] for x in a]}")
    assert len(set(iters)) > 1 and min(iters) < n, "instances should stop at different iterations"
    for x, y in zip(a, b):
        assert x[0] == y[0] and x[1] == y[1]
        for p, q in zip(x[2:], y[2:]):
            assert np.array_equal(p, q)
