"""Pins of the oracle's reverse mode (differentiation of the unrolled
iteration w.r.t. C and b) against central finite differences.

The projection derivative (Daleckii-Krein form) is pinned to finite
differences of a projection computed with LAPACK (numpy.linalg.eigh); the
whole vector-Jacobian product of T unrolled iterations is pinned to central
differences of the oracle's forward map (FP64, step 1e-6), and at
convergence to the envelope theorem (the gradient of the optimal value w.r.t.
b is the dual multiplier).
"""
import copy

import numpy as np
import pytest

import sdpgen


def numpy_psd(W):
    ev, V = np.linalg.eigh(0.5 * (W + W.T))
    return (V * np.maximum(ev, 0)) @ V.T


def sym(rng, s):
    g = rng.standard_normal((s, s))
    return 0.5 * (g + g.T)


@pytest.mark.parametrize("s", [2, 5, 12, 24])
def test_projection_derivative_matches_library_fd(oracle_mod, s):
    rng = np.random.default_rng(s)
    W = sym(rng, s)
    G = sym(rng, s)
    X, th, V, _ = oracle_mod.psd_project(W, return_eig=True)
    assert np.min(np.abs(th)) > 1e-3          # no eigenvalue at the kink
    dk = oracle_mod.psd_project_derivative(V, th, G)
    h = 1e-6
    fd = (numpy_psd(W + h * G) - numpy_psd(W - h * G)) / (2 * h)
    assert np.abs(dk - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())
    # self-adjoint: <D[G], H> = <G, D[H]>
    H = sym(rng, s)
    dh = oracle_mod.psd_project_derivative(V, th, H)
    assert abs(np.sum(dk * H) - np.sum(G * dh)) <= 1e-12 * s * s


def test_projection_derivative_special_cases(oracle_mod):
    """All eigenvalues positive: identity map; all negative: zero map."""
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    G = sym(rng, 6)
    th = np.array([1.0, 2.0, 3.0, 0.5, 4.0, 2.0])
    assert np.allclose(oracle_mod.psd_project_derivative(Q, th, G), G, atol=1e-13)
    assert np.allclose(oracle_mod.psd_project_derivative(Q, -th, G), 0.0, atol=1e-13)


def weighted(inst, x, y):
    w = np.where(inst.pat_row == inst.pat_col, 1.0, 2.0)
    return float(np.sum(w * x * y))


def fd_check(oracle_mod, inst, T, rho, seed, h=1e-6):
    rng = np.random.default_rng(seed)
    P = oracle_mod.Problem(inst)
    ubar = rng.standard_normal(inst.nnz)
    uT, cbar, bbar = P.unrolled_vjp(T, rho, ubar)
    dc = rng.standard_normal(inst.nnz)
    db = rng.standard_normal(inst.m)

    def g(sign):
        P.set_cb(inst.c + sign * h * dc, inst.b + sign * h * db)
        u = P.unrolled_forward(T, rho)
        return weighted(inst, ubar, u)

    fd = (g(+1) - g(-1)) / (2 * h)
    P.set_cb(inst.c, inst.b)
    an = weighted(inst, cbar, dc) + float(bbar @ db)
    return an, fd, uT, P


@pytest.mark.parametrize("shape,T", [((3, 3, 2, 6, 0), 5), ((4, 4, 3, 12, 1), 20),
                                     ((2, 6, 2, 9, 2), 40)])
def test_unrolled_vjp_matches_central_differences(oracle_mod, shape, T):
    l, d, h, m, seed = shape
    inst = sdpgen.block_arrow_instance(l, d, h, m, seed)
    an, fd, uT, P = fd_check(oracle_mod, inst, T, rho=0.8, seed=seed)
    assert abs(an - fd) <= 1e-6 * max(1.0, abs(fd)), (an, fd)
    assert np.allclose(uT, P.unrolled_forward(T, 0.8), atol=0)   # same forward


def test_unrolled_vjp_with_singleton_and_sparse(oracle_mod):
    from cases import singleton_clique_instance
    inst = singleton_clique_instance()
    an, fd, _, _ = fd_check(oracle_mod, inst, 15, rho=1.3, seed=4)
    assert abs(an - fd) <= 1e-6 * max(1.0, abs(fd))
    inst = sdpgen.block_arrow_instance(3, 5, 2, 10, seed=6, density=0.3)
    an, fd, _, _ = fd_check(oracle_mod, inst, 15, rho=1.0, seed=5)
    assert abs(an - fd) <= 1e-6 * max(1.0, abs(fd))


def test_objective_gradient_envelope_theorem(oracle_mod):
    """For the converged iterate, d<C,X*>/db = y_dual (the dual multipliers)
    and d/dc = X*: the unrolled gradient approaches both as T grows."""
    inst = sdpgen.block_arrow_instance(3, 3, 2, 5, seed=7)
    P = oracle_mod.Problem(inst)
    T = 1500
    uT = P.unrolled_forward(T, 1.0)
    yd = P.y_dual()
    # gradient of f = <c, u_T>: ubar = c, plus the direct term u_T in cbar
    _, cbar, bbar = P.unrolled_vjp(T, 1.0, inst.c)
    cbar = cbar + uT
    assert np.allclose(bbar, yd, atol=1e-4 * max(1.0, np.abs(yd).max()))
    assert np.allclose(cbar, uT, atol=1e-4 * max(1.0, np.abs(uT).max()))
