"""Pins of the oracle's Algorithm 2 (ADMM for the range-space decomposition
of the dual-form SDP, Section 4.2) against what the paper and the mathematics
fix, independently of the oracle's own arithmetic:

* one iteration against a full-vector reference built from explicit Kronecker
  selectors, numpy.linalg.solve on the KKT system (OptCondMinYDual) and an
  eigh-based projection (zkUpdate, vkEqn, MultUpdateDualSDP);
* closed-form optima through the dual objective b^T y (Lovasz theta of odd
  cycles, MaxCut on trees) and strong duality with Algorithm 1;
* invariants of every iterate: lambda_k = -rho H_k x (vkEqn substituted in the
  multiplier update), A(-rho x) = b, residuals as DualConsensusResidual
  defines them; dual feasibility C - sum y_i A_i >= 0 at convergence.
"""
import numpy as np
import pytest

import sdpgen
from test_oracle_pins import full_sym_from_lower, numpy_psd, rand_sym, selector, vec


def weights(inst):
    return np.where(inst.pat_row == inst.pat_col, 1.0, 2.0)


@pytest.mark.parametrize("shape", [(2, 2, 1, 3), (3, 3, 2, 6)])
def test_one_dual_iteration_matches_full_vector_reference(oracle_mod, shape):
    l, d, h, m = shape
    inst = sdpgen.block_arrow_instance(l, d, h, m, seed=5)
    n, p = inst.n, inst.p
    rng = np.random.default_rng(3)
    rho = 0.8
    Zs = [rand_sym(rng, len(inst.clique(k))) for k in range(p)]
    Ls = [rand_sym(rng, len(inst.clique(k))) for k in range(p)]
    Vs = [rand_sym(rng, len(inst.clique(k))) for k in range(p)]
    # ---- reference on n^2 variables ----
    Afull = np.stack([vec(full_sym_from_lower(inst, inst.a_val[i])) for i in range(m)])
    cfull = vec(full_sym_from_lower(inst, inst.c))
    Hs = [np.kron(selector(inst.clique(k), n), selector(inst.clique(k), n)) for k in range(p)]
    D = sum(np.diag(H.T @ H) for H in Hs)
    Zn = [numpy_psd(Vs[k] - Ls[k] / rho) for k in range(p)]                  # zkUpdate
    rhs = cfull - sum(Hs[k].T @ vec(Zn[k] + Ls[k] / rho) for k in range(p))
    S = np.nonzero(D > 0)[0]
    K = np.zeros((len(S) + m, len(S) + m))
    K[:len(S), :len(S)] = np.diag(D[S])
    K[:len(S), len(S):] = Afull[:, S].T
    K[len(S):, :len(S)] = Afull[:, S]
    sol = np.linalg.solve(K, np.concatenate([rhs[S], -inst.b / rho]))      # OptCondMinYDual
    x = np.zeros(n * n)
    x[S] = sol[:len(S)]
    y = sol[len(S):]
    Vn = [Zn[k] + Ls[k] / rho + (Hs[k] @ x).reshape(Zn[k].shape, order="F") for k in range(p)]
    Ln = [Ls[k] + rho * (Zn[k] - Vn[k]) for k in range(p)]                   # MultUpdateDualSDP
    # ---- oracle ----
    P = oracle_mod.Problem(inst, rho0=rho)
    P.set_blocks(Zs, Ls)
    P.set_v_blocks(Vs)
    P.run_dual(1, tol=0.0)
    Zo, Lo = P.blocks()
    Vo = P.v_blocks()
    for k in range(p):
        assert np.allclose(Zo[k], Zn[k], atol=1e-11)
        assert np.allclose(Vo[k], Vn[k], atol=1e-10)
        assert np.allclose(Lo[k], Ln[k], atol=1e-10)
    assert np.allclose(P.u(), x[inst.pat_col * n + inst.pat_row], atol=1e-10)
    assert np.allclose(P.y(), y, atol=1e-10)


@pytest.mark.parametrize("n", [5, 7, 9])
def test_dual_objective_gives_lovasz_theta(oracle_mod, n):
    inst = sdpgen.lovasz_theta_odd_cycle(n)
    P = oracle_mod.Problem(inst)
    r = P.run_dual(200000, tol=1e-10, adaptive=True)
    assert r.status == oracle_mod.OK
    exact = -n * np.cos(np.pi / n) / (1 + np.cos(np.pi / n))
    assert abs(P.dual_objective() - exact) <= 1e-7 * abs(exact)


@pytest.mark.parametrize("seed", [0, 1])
def test_dual_objective_on_maxcut_tree(oracle_mod, seed):
    inst = sdpgen.maxcut_tree(25, seed)
    P = oracle_mod.Problem(inst)
    r = P.run_dual(200000, tol=1e-10, adaptive=True)
    assert r.status == oracle_mod.OK
    exact = -np.abs(inst.meta["weights"]).sum()
    assert abs(P.dual_objective() - exact) <= 1e-7 * abs(exact)


@pytest.mark.parametrize("shape", [(3, 3, 2, 6, 4), (4, 4, 2, 9, 7)])
def test_strong_duality_with_algorithm_1_and_dual_feasibility(oracle_mod, shape):
    """Both algorithms reach the common optimum; the dual iterate is a valid
    certificate (C - sum y_i A_i PSD by dense eigh) and -rho x is a primal
    point with the same objective."""
    l, d, h, m, seed = shape
    inst = sdpgen.block_arrow_instance(l, d, h, m, seed)
    Pd = oracle_mod.Problem(inst)
    Pp = oracle_mod.Problem(inst)
    assert Pd.run_dual(400000, tol=1e-10, adaptive=True).status == 0
    assert Pp.run(400000, tol=1e-10, adaptive=True).status == 0
    bty, ctx = Pd.dual_objective(), Pp.objective()
    assert abs(bty - ctx) <= 1e-6 * (1 + abs(ctx))
    Z = full_sym_from_lower(inst, inst.c - Pd.y() @ inst.a_val)
    assert np.linalg.eigvalsh(Z).min() >= -1e-6
    xp = -Pd.rho * Pd.u()
    assert abs(np.sum(weights(inst) * inst.c * xp) - ctx) <= 1e-6 * (1 + abs(ctx))


def test_dual_iterate_invariants(oracle_mod):
    """After every iteration: lambda_k = -rho H_k x and A(-rho x) = b; the
    residuals follow DualConsensusResidual."""
    inst = sdpgen.block_arrow_instance(3, 4, 2, 7, seed=9)
    P = oracle_mod.Problem(inst, rho0=1.3)
    w = weights(inst)
    A = inst.a_val
    for it in range(6):
        Zp, _ = P.blocks()
        r = P.run_dual(1, tol=0.0)
        Z, L = P.blocks()
        V = P.v_blocks()
        x = P.u()
        G = P.gather(x)
        for k in range(inst.p):
            assert np.allclose(L[k], -P.rho * G[k], atol=1e-10)
        assert np.allclose(A @ (w * (-P.rho * x)), inst.b, atol=1e-9)
        num = np.sqrt(sum(np.sum((Z[k] - V[k]) ** 2) for k in range(inst.p)))
        den = max(np.sqrt(sum(np.sum(Z[k] ** 2) for k in range(inst.p))),
                  np.sqrt(sum(np.sum(V[k] ** 2) for k in range(inst.p))))
        eps_c = num / den if den > 0 else (0.0 if num == 0 else np.inf)
        dz = np.sqrt(sum(np.sum((Z[k] - Zp[k]) ** 2) for k in range(inst.p)))
        nl = np.sqrt(sum(np.sum(L[k] ** 2) for k in range(inst.p)))
        eps_l = P.rho * dz / nl if nl > 0 else (0.0 if dz == 0 else np.inf)
        assert np.isclose(r.eps_c, eps_c, rtol=1e-10, atol=1e-14)
        assert np.isclose(r.eps_l, eps_l, rtol=1e-10, atol=1e-14)


def test_dual_small_workload_converges(oracle_mod):
    inst = sdpgen.workload_small_blockarrow()
    P = oracle_mod.Problem(inst)
    r = P.run_dual(20000, tol=1e-4)
    assert r.status == oracle_mod.OK
    assert max(r.eps_c, r.eps_l) <= 1e-4
