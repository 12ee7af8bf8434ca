"""The solver on preprocessed instances: nonchordal patterns given their
chordal extension by the library (Theorem 1; Section 7.1.1) and data scaled
by the library (Section 7.1.3).

* Fixed-N parity of the GPU iterates on the extended instances against the
  oracle run on the same extended instance (FP64 1e-8, FP32-eig 2e-4), at
  small size and on the 45 x 45 grid workload (cliques of 3 to 76 vertices).
* The GPU solve on the extension reaches the optimum the oracle finds for the
  undecomposed SDP (the single clique V).
* A badly scaled instance, scaled by the library and solved on the GPU with
  the adaptive penalty, maps back to the original optimum and needs far
  fewer iterations than the unscaled solve.
"""
import numpy as np
import pytest

import sdpgen
from cases import as_instance
from test_gpu_admm import compare_fixed_n

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def weights(inst):
    return np.where(inst.pat_row == inst.pat_col, 1.0, 2.0)


def small_grid_instance():
    pr, pc = sdpgen.grid_pattern(6, 6)
    return sdpgen.instance_on_pattern(36, pr, pc, 12, seed=7, name="grid6x6_m12_s7")


def test_extended_grid_fixed_n(sdp, gpu, oracle_mod):
    ext = as_instance(sdp.extend_instance(small_grid_instance()))
    log(f"grid 6x6 extension: p={ext.p} sizes {sorted(set(np.diff(ext.clique_ptr).tolist()))}")
    compare_fixed_n(sdp, oracle_mod, ext, 30, tol_rel=1e-8)
    compare_fixed_n(sdp, oracle_mod, ext, 10, precision="fp32", tol_rel=2e-4)


def test_nonchordal_workload_fixed_n(sdp, gpu, oracle_mod):
    """The 45 x 45 grid (n = 2025, m = 200, sparse A) on its extension:
    1540 cliques of 3 to 76 vertices."""
    ext = as_instance(sdp.extend_instance(sdpgen.workload_nonchordal()))
    sz = np.diff(ext.clique_ptr)
    log(f"nonchordal workload: nnz {ext.nnz} p={ext.p} sizes {sz.min()}..{sz.max()}")
    compare_fixed_n(sdp, oracle_mod, ext, 5, tol_rel=1e-8)
    compare_fixed_n(sdp, oracle_mod, ext, 5, precision="fp32", tol_rel=2e-4)


def test_extension_solve_reaches_undecomposed_optimum(sdp, gpu, oracle_mod):
    pr, pc = sdpgen.grid_pattern(3, 5)
    inst = sdpgen.instance_on_pattern(15, pr, pc, 8, seed=11)
    one = sdpgen.as_single_clique(inst)
    Pu = oracle_mod.Problem(one)
    assert Pu.run(400000, tol=1e-10, adaptive=True).status == 0
    ext = sdp.extend_instance(inst)
    with sdp.Solver([ext], tol=1e-7, max_iter=200000, adaptive_rho=1) as S:
        g = S.solve()[0]
    log(f"grid 3x5: gpu {g['iters']} it obj {g['objective']:.10g}; undecomposed {Pu.objective():.10g}")
    assert g["status"] == 0
    assert abs(g["objective"] - Pu.objective()) <= 1e-5 * (1 + abs(Pu.objective()))


def test_scaled_solve_maps_back(sdp, gpu, oracle_mod):
    base = sdpgen.block_arrow_instance(3, 4, 2, 8, seed=1)
    bad = sdpgen.rescaled_instance(base, seed=3)
    Pb = oracle_mod.Problem(base)
    assert Pb.run(400000, tol=1e-10, adaptive=True).status == 0
    target = bad.meta["g"] * Pb.objective()          # the copy's optimal value
    S = sdp.scale_instance(bad, iters=10)
    with sdp.Solver([S.scaled], tol=1e-6, max_iter=50000, adaptive_rho=1) as Sv:
        gs = Sv.solve()[0]
        sol = Sv.solution(0)
    x, y, _ = S.recover(sol["u"], sol["y_dual"])
    obj = float(np.sum(weights(bad) * bad.c * x))
    with sdp.Solver([bad], tol=1e-6, max_iter=50000, adaptive_rho=1) as Sv:
        gb = Sv.solve()[0]
    log(f"scaled: {gs['iters']} it, recovered obj {obj:.10g} (target {target:.10g}); "
        f"unscaled: {gb['iters']} it status {gb['status']}")
    assert gs["status"] == 0
    assert abs(obj - target) <= 1e-4 * abs(target)
    assert abs(float(bad.b @ y) - target) <= 1e-4 * abs(target)
    assert gs["iters"] * 5 <= gb["iters"]
