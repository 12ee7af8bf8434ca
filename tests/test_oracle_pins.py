"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test names what pins it: a worked example printed in the paper, a library
routine that solves the same mathematical problem, a closed form, or an
invariant of the projection/ADMM that a dropped term, a wrong sign or a
transposed operand would break.
"""
import json
import os

import numpy as np
import pytest

import sdpgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# helpers (independent of the oracle): explicit selector matrices, full vec
# ----------------------------------------------------------------------------

def selector(clique, n):
    """E_C with (E_C)_ij = 1 iff C(i) = j (Section 'Sparse matrix cones')."""
    E = np.zeros((len(clique), n))
    for i, v in enumerate(clique):
        E[i, v] = 1.0
    return E


def vec(M):
    return M.flatten(order="F")


def full_sym_from_lower(inst, vals):
    n = inst.n
    M = np.zeros((n, n))
    M[inst.pat_row, inst.pat_col] = vals
    M[inst.pat_col, inst.pat_row] = vals
    return M


def numpy_psd(W):
    ev, V = np.linalg.eigh(0.5 * (W + W.T))
    return (V * np.maximum(ev, 0)) @ V.T


def rand_sym(rng, s):
    g = rng.standard_normal((s, s))
    return 0.5 * (g + g.T)


# ----------------------------------------------------------------------------
# Jacobi eigensolver and the PSD projection (XkUpdate)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("s", [1, 2, 3, 7, 16, 24, 33, 64])
def test_jacobi_matches_library_eigh(oracle_mod, s):
    """Pinned to numpy.linalg.eigh (LAPACK) on GOE blocks."""
    W = sdpgen.goe_blocks([s], seed=100 + s)[0]
    th, V, sweeps = oracle_mod.jacobi_eig(W)
    ref = np.linalg.eigvalsh(W)
    scale = np.linalg.norm(W)
    assert np.allclose(np.sort(th), ref, atol=1e-12 * scale, rtol=0)
    assert np.allclose(V.T @ V, np.eye(s), atol=1e-13)
    assert np.allclose((V * th) @ V.T, W, atol=1e-12 * scale)
    assert sweeps <= 20


def test_jacobi_2x2_closed_form(oracle_mod):
    """Eigenvalues of [[a, b], [b, c]] are (a+c)/2 +- sqrt(((a-c)/2)^2 + b^2)."""
    rng = np.random.default_rng(7)
    for _ in range(50):
        a, b, c = rng.standard_normal(3) * 10 ** rng.uniform(-3, 3, 3)
        th, V, _ = oracle_mod.jacobi_eig(np.array([[a, b], [b, c]]))
        r = np.sqrt(((a - c) / 2) ** 2 + b ** 2)
        exact = np.array([(a + c) / 2 - r, (a + c) / 2 + r])
        assert np.allclose(np.sort(th), exact, rtol=1e-14, atol=1e-14 * (abs(a) + abs(b) + abs(c)))


def test_projection_diagonal_input_is_clamp(oracle_mod):
    d = np.array([3.0, -1.0, 0.0, 2.5, -7.0, 1e-300])
    X = oracle_mod.psd_project(np.diag(d))
    assert np.array_equal(X, np.diag(np.maximum(d, 0)))


@pytest.mark.parametrize("s", [2, 5, 16, 24, 50])
def test_projection_matches_library_and_invariants(oracle_mod, s):
    """Against numpy eigh; Moreau decomposition; idempotence; PSD output;
    positive homogeneity; orthogonal equivariance; nonexpansiveness; and
    optimality against random PSD matrices."""
    rng = np.random.default_rng(s)
    W = rand_sym(rng, s)
    P = oracle_mod.psd_project
    X = P(W)
    nrm = np.linalg.norm(W)
    assert np.allclose(X, numpy_psd(W), atol=1e-12 * nrm)
    Xm = P(-W)
    assert np.allclose(X - Xm, W, atol=1e-12 * nrm)                  # Moreau
    assert abs(np.sum(X * Xm)) <= 1e-12 * nrm ** 2                   # <P+X, P+(-X)> = 0
    assert np.allclose(P(X), X, atol=1e-12 * nrm)                    # idempotent
    assert np.linalg.eigvalsh(X).min() >= -1e-12 * nrm               # PSD
    assert np.allclose(P(3.5 * W), 3.5 * X, atol=1e-11 * nrm)        # homogeneous
    Q, _ = np.linalg.qr(rng.standard_normal((s, s)))
    assert np.allclose(P(Q @ W @ Q.T), Q @ X @ Q.T, atol=1e-11 * nrm)
    W2 = rand_sym(rng, s)
    assert np.linalg.norm(P(W2) - X) <= np.linalg.norm(W2 - W) * (1 + 1e-12)
    for _ in range(5):
        G = rng.standard_normal((s, s))
        Y = G @ G.T / s
        assert np.linalg.norm(W - X) <= np.linalg.norm(W - Y) + 1e-12


def test_projection_padding_is_exact(oracle_mod):
    """P+(diag(W, 0)) = diag(P+(W), 0): a zero-padded block projects exactly."""
    rng = np.random.default_rng(3)
    W = rand_sym(rng, 5)
    Wp = np.zeros((8, 8))
    Wp[:5, :5] = W
    Xp = oracle_mod.psd_project(Wp)
    assert np.allclose(Xp[:5, :5], oracle_mod.psd_project(W), atol=1e-13)
    assert np.all(Xp[5:, :] == 0) and np.all(Xp[:, 5:] == 0)


# ----------------------------------------------------------------------------
# Cholesky and substitutions (the cached factor)
# ----------------------------------------------------------------------------

def test_cholesky_and_solve_match_library(oracle_mod):
    rng = np.random.default_rng(0)
    G = rng.standard_normal((40, 60))
    M = G @ G.T
    rc, L = oracle_mod.cholesky(M)
    assert rc == 0
    assert np.allclose(L, np.linalg.cholesky(M), atol=1e-10)
    r = rng.standard_normal(40)
    assert np.allclose(oracle_mod.chol_solve(L, r), np.linalg.solve(M, r), atol=1e-10)


def test_cholesky_reports_rank_deficiency(oracle_mod):
    G = np.random.default_rng(1).standard_normal((5, 3))
    rc, _ = oracle_mod.cholesky(G @ G.T)
    assert rc == oracle_mod.ERR_RANK_DEFICIENT


# ----------------------------------------------------------------------------
# Entry selectors: the paper's worked example and explicit H_k = E_k (x) E_k
# ----------------------------------------------------------------------------

def _example_instance():
    g = json.load(open(os.path.join(GOLDEN, "paper_selector_example.json")))
    n = g["n"]
    cliques = [np.array(c) - 1 for c in g["cliques_1based"]]
    pr, pc = sdpgen.pattern_from_cliques(n, cliques)
    ptr, vert = sdpgen.cliques_to_csr(cliques)
    nnz = pr.shape[0]
    diag = (pr == pc).astype(float)
    inst = sdpgen.Instance(n=n, m=1, pat_row=pr, pat_col=pc, clique_ptr=ptr,
                           clique_vert=vert, a_format=0, a_val=diag[None, :].copy(),
                           b=np.array([float(n)]), c=np.zeros(nnz))
    return g, inst


def test_selector_matches_paper_example(oracle_mod):
    g, inst = _example_instance()
    E1 = selector(inst.clique(0), inst.n)
    assert np.array_equal(E1, np.array(g["E_C1"], dtype=float))
    P = oracle_mod.Problem(inst)
    # gather: E_C1 X E_C1^T has the printed entries X_{ab}
    X = np.arange(1, 17, dtype=float).reshape(4, 4)
    X = X + X.T
    u = X[inst.pat_row, inst.pat_col]
    U1 = P.gather(u)[0]
    for a, row in enumerate(g["E_C1_X_E_C1T_entries_1based"]):
        for b, (i, j) in enumerate(row):
            assert U1[a, b] == X[i - 1, j - 1]
    # scatter: sum_k H_k^T x_k with x_2 = 0, lambda = 0, c = 0, rho = 1 places
    # Y where the printed E_C1^T Y E_C1 says (on the pattern coordinates)
    Y = np.array([[1.0, 2.0, 3.0], [2.0, 5.0, 6.0], [3.0, 6.0, 9.0]])
    bhat = P.form_bhat([Y, np.zeros((3, 3))], [np.zeros((3, 3))] * 2, 1.0)
    full = np.zeros((4, 4))
    full[inst.pat_row, inst.pat_col] = bhat
    full[inst.pat_col, inst.pat_row] = bhat
    for i, row in enumerate(g["E_C1T_Y_E_C1_entries_1based"]):
        for j, ent in enumerate(row):
            expect = 0.0 if ent is None else Y[ent[0] - 1, ent[1] - 1]
            assert full[i, j] == expect


def test_overlap_counts_equal_explicit_sum_of_HkT_Hk(oracle_mod):
    inst = sdpgen.block_arrow_instance(3, 3, 2, 4, seed=5)
    n = inst.n
    Dfull = np.zeros(n * n)
    for k in range(inst.p):
        E = selector(inst.clique(k), n)
        H = np.kron(E, E)
        assert np.allclose(H @ H.T, np.eye(H.shape[0]))     # orthonormal rows
        Dfull += np.diag(H.T @ H)
    P = oracle_mod.Problem(inst)
    # vec stacks columns: entry (r, c) sits at c*n + r
    assert np.array_equal(P.D(), Dfull[inst.pat_col * n + inst.pat_row])
    assert np.all(Dfull[Dfull > 0] >= 1)


# ----------------------------------------------------------------------------
# Affine step: the full-vector KKT system (OptCondMinYPrimal) solved densely
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(2, 2, 1, 3), (3, 3, 2, 6), (2, 4, 2, 9)])
def test_affine_step_matches_full_kkt_solve(oracle_mod, shape):
    """Pinned to numpy.linalg.solve on [[D, A^T], [A, 0]] over n^2 variables.

    Entries outside the pattern have D = 0 and appear in no data; the system is
    solved on the pattern entries E* (both triangles).
    """
    l, d, h, m = shape
    inst = sdpgen.block_arrow_instance(l, d, h, m, seed=11)
    n = inst.n
    rng = np.random.default_rng(1)
    rho = 0.7
    Xs = [rand_sym(rng, len(inst.clique(k))) for k in range(inst.p)]
    Ls = [rand_sym(rng, len(inst.clique(k))) for k in range(inst.p)]
    # independent full-vector construction
    Afull = np.stack([vec(full_sym_from_lower(inst, inst.a_val[i])) for i in range(m)])
    cfull = vec(full_sym_from_lower(inst, inst.c))
    D = np.zeros(n * n)
    rhs = -cfull / rho
    for k in range(inst.p):
        E = selector(inst.clique(k), n)
        H = np.kron(E, E)
        D += np.diag(H.T @ H)
        rhs += H.T @ (vec(Xs[k]) + vec(Ls[k]) / rho)
    S = np.nonzero(D > 0)[0]
    K = np.zeros((len(S) + m, len(S) + m))
    K[:len(S), :len(S)] = np.diag(D[S])
    K[:len(S), len(S):] = Afull[:, S].T
    K[len(S):, :len(S)] = Afull[:, S]
    sol = np.linalg.solve(K, np.concatenate([rhs[S], inst.b]))
    x = np.zeros(n * n)
    x[S] = sol[:len(S)]
    y_ref = sol[len(S):]
    # oracle
    P = oracle_mod.Problem(inst)
    bhat = P.form_bhat(Xs, Ls, rho)
    assert np.allclose(bhat, rhs[inst.pat_col * n + inst.pat_row], atol=1e-12)
    u, y = P.affine(bhat)
    assert np.allclose(u, x[inst.pat_col * n + inst.pat_row], atol=1e-10)
    assert np.allclose(y, y_ref, atol=1e-10)
    # the x-update satisfies Ax = b exactly (up to rounding)
    assert np.allclose(Afull @ x, inst.b, atol=1e-10)


def test_maxcut_pattern_gives_diagonal_factor(oracle_mod):
    """For MaxCut-type problems A D^-1 A^T is diagonal (Section 'Minimization
    over X'), so its Cholesky factor is diagonal too."""
    inst = sdpgen.maxcut_tree(12, seed=2)
    L = oracle_mod.Problem(inst).L()
    assert np.count_nonzero(L - np.diag(np.diag(L))) == 0


# ----------------------------------------------------------------------------
# Whole Algorithm 1 against closed-form optima
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n", [5, 7, 9])
def test_lovasz_theta_of_odd_cycles(oracle_mod, n):
    """theta(C_n) = n cos(pi/n) / (1 + cos(pi/n)) for odd n (C_5: sqrt 5)."""
    inst = sdpgen.lovasz_theta_odd_cycle(n)
    P = oracle_mod.Problem(inst)
    r = P.run(200000, tol=1e-10, adaptive=True)
    assert r.status == oracle_mod.OK
    exact = -n * np.cos(np.pi / n) / (1 + np.cos(np.pi / n))
    assert abs(P.objective() - exact) <= 1e-7 * abs(exact)
    if n == 5:
        assert abs(P.objective() + np.sqrt(5.0)) <= 1e-7


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_maxcut_on_tree(oracle_mod, seed):
    """On a tree the relaxation is tight: optimum -sum |w_ij|."""
    inst = sdpgen.maxcut_tree(25, seed)
    P = oracle_mod.Problem(inst)
    r = P.run(200000, tol=1e-10, adaptive=True)
    assert r.status == oracle_mod.OK
    exact = -np.abs(inst.meta["weights"]).sum()
    assert abs(P.objective() - exact) <= 1e-7 * abs(exact)


@pytest.mark.parametrize("shape", [(3, 3, 2, 5, 0), (4, 2, 3, 8, 1), (2, 5, 2, 7, 2)])
def test_decomposed_equals_undecomposed(oracle_mod, shape):
    """Theorem 1: decomposing over the maximal cliques leaves the optimum
    unchanged; the one-clique problem is the undecomposed SDP."""
    l, d, h, m, seed = shape
    inst = sdpgen.block_arrow_instance(l, d, h, m, seed)
    one = sdpgen.as_single_clique(inst)
    Pd = oracle_mod.Problem(inst)
    Pu = oracle_mod.Problem(one)
    rd = Pd.run(400000, tol=1e-10, adaptive=True)
    ru = Pu.run(400000, tol=1e-10, adaptive=True)
    assert rd.status == 0 and ru.status == 0
    od, ou = Pd.objective(), Pu.objective()
    assert abs(od - ou) <= 1e-6 * (1 + abs(ou))
    # the undecomposed solution is a genuine PSD matrix: check with eigh
    X = full_sym_from_lower(one, Pu.u())
    assert np.linalg.eigvalsh(X).min() >= -1e-6


def test_dual_certificate_on_small_instance(oracle_mod):
    """At convergence y_dual = -rho*y gives Z = C - sum y_i A_i PSD (dense
    eigh) and a vanishing duality gap, so b^T y_dual is a valid lower bound."""
    inst = sdpgen.block_arrow_instance(3, 3, 2, 6, seed=4)
    P = oracle_mod.Problem(inst)
    P.run(400000, tol=1e-10, adaptive=True)
    yd = P.y_dual()
    Zl = inst.c - yd @ inst.a_val
    Z = full_sym_from_lower(inst, Zl)
    assert np.linalg.eigvalsh(Z).min() >= -1e-6
    diag = P.diagnostics()
    assert diag["eps_g"] <= 1e-7 and diag["eps_p"] <= 1e-10 and diag["eps_d"] <= 1e-7
    assert inst.b @ yd <= P.objective() + 1e-6


# ----------------------------------------------------------------------------
# Invariants of every iterate
# ----------------------------------------------------------------------------

def test_multiplier_is_projection_of_minus_w(oracle_mod):
    """lambda_k^+ = lambda_k + rho (x_k - H_k x) with x_k = P+(W_k),
    W_k = H_k x - lambda_k/rho, equals rho P+(-W_k) (Moreau): after every
    iteration Lambda_k is PSD and orthogonal to X_k."""
    inst = sdpgen.block_arrow_instance(4, 5, 3, 20, seed=8)
    P = oracle_mod.Problem(inst, rho0=0.5)
    for _ in range(6):
        W = P.next_w()
        rho = P.rho
        P.run(1, tol=0.0)
        Xs, Ls = P.blocks()
        for Wk, Xk, Lk in zip(W, Xs, Ls):
            assert np.allclose(Xk, numpy_psd(Wk), atol=1e-11)
            assert np.allclose(Lk, rho * numpy_psd(-Wk), atol=1e-10)
            assert np.linalg.eigvalsh(Lk).min() >= -1e-10
            assert abs(np.sum(Xk * Lk)) <= 1e-9


def test_residuals_follow_their_definition(oracle_mod):
    """eps_c and eps_lambda recomputed from the full blocks (PrimalConsensusResidual)."""
    inst = sdpgen.block_arrow_instance(3, 4, 2, 10, seed=9)
    P = oracle_mod.Problem(inst)
    P.run(3, tol=0.0)
    Xp, _ = P.blocks()
    rho = P.rho
    r = P.run(1, tol=0.0)
    X, L = P.blocks()
    U = P.gather(P.u())
    num = np.sqrt(sum(np.sum((x - u) ** 2) for x, u in zip(X, U)))
    den = max(np.sqrt(sum(np.sum(x ** 2) for x in X)), np.sqrt(sum(np.sum(u ** 2) for u in U)))
    assert np.isclose(r.eps_c, num / den, rtol=1e-12)
    el = rho * np.sqrt(sum(np.sum((x - xp) ** 2) for x, xp in zip(X, Xp))) / \
        np.sqrt(sum(np.sum(l ** 2) for l in L))
    assert np.isclose(r.eps_l, el, rtol=1e-12)


def test_adaptive_penalty_rule(oracle_mod):
    """rho <- mu rho if eps_c >= nu eps_l; rho <- rho/mu if eps_l >= nu eps_c."""
    inst = sdpgen.lovasz_theta_odd_cycle(7)
    P = oracle_mod.Problem(inst, rho0=50.0)
    r = P.run(400, tol=1e-12, adaptive=True, mu=2.0, nu=10.0)
    hc, hl, hr = r.hist_eps_c, r.hist_eps_l, r.hist_rho
    changed = 0
    for it in range(len(hr) - 1):
        if hc[it] >= 10 * hl[it]:
            assert hr[it + 1] == 2 * hr[it]
        elif hl[it] >= 10 * hc[it]:
            assert hr[it + 1] == hr[it] / 2
        else:
            assert hr[it + 1] == hr[it]
        changed += hr[it + 1] != hr[it]
    assert changed > 0


def test_fixed_rho_never_changes(oracle_mod):
    inst = sdpgen.workload_small_blockarrow()
    P = oracle_mod.Problem(inst, rho0=1.0)
    r = P.run(50, tol=0.0, adaptive=False)
    assert np.all(r.hist_rho == 1.0)


def test_small_blockarrow_workload_converges(oracle_mod):
    """n=105 block-arrow workload reaches the 1e-4 residual; the x-update keeps
    Ax = b to rounding (the paper's remark on the primal residual)."""
    inst = sdpgen.workload_small_blockarrow()
    P = oracle_mod.Problem(inst)
    r = P.run(20000, tol=1e-4, adaptive=False)
    assert r.status == 0 and r.iters < 2000
    dg = P.diagnostics()
    assert dg["eps_p"] < 1e-10
    assert dg["eps_g"] < 1e-3


# ----------------------------------------------------------------------------
# Validation status codes
# ----------------------------------------------------------------------------

from cases import invalid_instances, rank_deficient_instance  # noqa: E402


@pytest.mark.parametrize("case", invalid_instances(), ids=lambda c: c[0])
def test_oracle_validation_codes(oracle_mod, case):
    name, inst, code = case
    assert oracle_mod.create_status(inst) == code


def test_oracle_rank_deficient(oracle_mod):
    assert oracle_mod.create_status(rank_deficient_instance()) == oracle_mod.ERR_RANK_DEFICIENT


# ----------------------------------------------------------------------------
# Diagnostics: HSDEerror (relative primal/dual residuals and gap, Section 5.2.3)
# and the PSD-violation bound eps_alpha (Section 7.2)
# ----------------------------------------------------------------------------

def _full_diagnostics(inst, u, y_dual, lam_blocks, b):
    """eps_p, eps_d, eps_g and eps_alpha from explicit n x n matrices: X, C and
    every A_i built on both triangles, Z = sum_k E_k^T Lambda_k E_k with the
    selector matrices, Frobenius norms of the full matrices (no compact
    weights anywhere)."""
    n, m = inst.n, inst.m
    X = full_sym_from_lower(inst, u)
    C = full_sym_from_lower(inst, inst.c)
    A = [full_sym_from_lower(inst, row) for row in inst.a_dense()]
    Z = np.zeros((n, n))
    cliques = [inst.clique_vert[inst.clique_ptr[k]:inst.clique_ptr[k + 1]]
               for k in range(len(inst.clique_ptr) - 1)]
    lmin = []
    for k, cl in enumerate(cliques):
        E = selector(cl, n)
        Z += E.T @ lam_blocks[k] @ E
        lmin.append(np.linalg.eigvalsh(E @ X @ E.T).min())
    ax = np.array([np.sum(Ai * X) for Ai in A])
    eps_p = np.linalg.norm(ax - b) / (1.0 + np.linalg.norm(b))
    dres = sum(y_dual[i] * A[i] for i in range(m)) + Z - C
    eps_d = np.linalg.norm(dres) / (1.0 + np.linalg.norm(C))
    ctx, bty = np.sum(C * X), b @ y_dual
    eps_g = abs(ctx - bty) / (1.0 + abs(ctx) + abs(bty))
    alpha = -min(0.0, min(lmin))
    eps_alpha = alpha / (1.0 + np.linalg.norm(X))
    return dict(eps_p=eps_p, eps_d=eps_d, eps_g=eps_g, eps_alpha=eps_alpha,
                objective=ctx, dual_objective=bty), alpha, X, cliques


@pytest.mark.parametrize("iters,seed", [(2, 11), (5, 12), (9, 13)])
def test_diagnostics_follow_their_definitions(oracle_mod, iters, seed):
    """The oracle's eps_p, eps_d, eps_g (HSDEerror) and eps_alpha (PSD-violation)
    on a non-converged iterate, against the definitions evaluated on explicit
    full matrices.  b is replaced after the iteration, so that A x != b and the
    primal residual's normalisation 1 + ||b|| is exercised (the x-update alone
    keeps A x = b to rounding); the early iterate has clique blocks with
    negative eigenvalues and large dual residuals, so a lambda_max for
    lambda_min, a missing off-diagonal weight in ||X||_F or ||C||_F, or a
    dropped 1 + in any denominator changes the result."""
    inst = sdpgen.block_arrow_instance(4, 5, 3, 12, seed=seed)
    P = oracle_mod.Problem(inst, rho0=0.7)
    P.run(iters, tol=0.0)
    rng = np.random.default_rng(seed)
    b2 = inst.b + rng.standard_normal(inst.m)
    P.set_cb(b=b2)
    got = P.diagnostics()
    _, Ls = P.blocks()
    ref, alpha, X, cliques = _full_diagnostics(inst, P.u(), -P.rho * P.y(), Ls, b2)
    assert alpha > 1e-3, "the test needs a clique block with a negative eigenvalue"
    assert ref["eps_p"] > 1e-2 and ref["eps_d"] > 1e-3
    for key in ("eps_p", "eps_d", "eps_g", "eps_alpha", "objective", "dual_objective"):
        assert np.isclose(got[key], ref[key], rtol=1e-10, atol=1e-14), key


def test_eps_alpha_is_the_smallest_completable_shift(oracle_mod):
    """Section 7.2: alpha is the smallest non-negative shift with X + alpha I
    PSD-completable; by the chordal completion theorem that means every clique
    block of X + alpha I is PSD.  Checked with dense eigh on the blocks: alpha
    makes them all PSD, 0.99 alpha leaves one indefinite; the normalisation
    uses the full Frobenius norm of the partial matrix X."""
    inst = sdpgen.banded_instance(30, 4, 15, seed=5)
    P = oracle_mod.Problem(inst)
    P.run(3, tol=0.0)
    X = full_sym_from_lower(inst, P.u())
    alpha = P.diagnostics()["eps_alpha"] * (1.0 + np.linalg.norm(X))
    assert alpha > 1e-3
    n = inst.n
    cl = [inst.clique_vert[inst.clique_ptr[k]:inst.clique_ptr[k + 1]]
          for k in range(len(inst.clique_ptr) - 1)]
    mins = [np.linalg.eigvalsh(selector(c, n) @ (X + alpha * np.eye(n)) @ selector(c, n).T).min()
            for c in cl]
    assert min(mins) >= -1e-10 * alpha
    mins99 = [np.linalg.eigvalsh(selector(c, n) @ (X + 0.99 * alpha * np.eye(n)) @ selector(c, n).T).min()
              for c in cl]
    assert min(mins99) < 0


def test_eps_alpha_zero_for_psd_blocks(oracle_mod):
    """With every clique block of X positive definite the bound is exactly 0:
    after convergence of a MaxCut relaxation on a tree (optimum attained by a
    rank-one +-1 matrix, blocks [[1, +-1], [+-1, 1]] shifted by the iterate's
    rounding) alpha vanishes up to the 1e-10 residual."""
    inst = sdpgen.maxcut_tree(12, 3)
    P = oracle_mod.Problem(inst)
    P.run(200000, tol=1e-11, adaptive=True)
    d = P.diagnostics()
    _, Ls = P.blocks()
    ref, alpha, _, _ = _full_diagnostics(inst, P.u(), P.y_dual(), Ls, inst.b)
    assert d["eps_alpha"] <= 1e-8
    assert np.isclose(d["eps_alpha"], ref["eps_alpha"], rtol=1e-6, atol=1e-14)
