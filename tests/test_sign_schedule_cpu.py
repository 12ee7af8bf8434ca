"""The sign iteration's schedule (sdp_sign_schedule, host only, no GPU).

X0 = W / ||W||_F; k1 fast steps x <- 3x - 3.2x^3 + 1.2x^5, k2 Newton-Schulz
steps x <- x (3 - x^2) / 2; P+(W) = (W + W s(X0)) / 2.  Each eigenvalue
follows the scalar maps, so eigenvalue delta is off by
e(delta) = delta |1 - s(delta)| / 2 (units of ||W||_F), and at most n - 1
eigenvalues can sit at the worst point.  Checked here, independently of the
library's own grid:

* the schedule meets sqrt(n - 1) max e <= tol / 2 on a grid ten times finer;
* no schedule with fewer products (and k2 >= 2) meets 2 sqrt(n - 1) max e <=
  tol, so the library takes no more steps than the bound needs;
* on real symmetric matrices whose n - 1 small eigenvalues all sit at the
  scalar worst point (the case the bound is tight for), the FP64 matrix
  iteration gives P+(W) within tol ||W||_F / 2 of the eigendecomposition;
* the schedule never takes more products than the rule it replaces,
  k1 = ceil(log(1/tol) / log 3) with k2 = 3 (FP32) or 4 (FP64), which bounds
  each eigenvalue's error by 3^-k1 alone.
"""
import math

import numpy as np
import pytest

import paper_1707_05058_amd as sdp

GRID = np.concatenate([np.logspace(-18, 0, 18 * 2560 + 1), np.linspace(0, 1, 10241)[1:]])


def fast(x):
    return x * (3.0 - 3.2 * x * x + 1.2 * x ** 4)


def newton_schulz(x):
    return x * (3.0 - x * x) / 2.0


def worst_error(k1, k2, d=GRID):
    x = d.copy()
    for _ in range(k1):
        x = fast(x)
    for _ in range(k2):
        x = newton_schulz(x)
    e = d * np.abs(1.0 - x) / 2.0
    j = int(np.argmax(e))
    return e[j], d[j]


CASES = [(1e-4, 16), (1e-6, 16), (1e-6, 32), (1e-8, 96), (1e-10, 16), (1e-14, 16), (1e-14, 128)]


@pytest.mark.parametrize("tol,n", CASES)
def test_schedule_meets_the_bound(tol, n):
    k1, k2 = sdp.sign_schedule(tol, n)
    assert k2 >= 2
    e, _ = worst_error(k1, k2)
    assert math.sqrt(n - 1) * e <= tol / 2 * 1.02, (k1, k2, e)


@pytest.mark.parametrize("tol,n", CASES)
def test_schedule_is_minimal(tol, n):
    k1, k2 = sdp.sign_schedule(tol, n)
    products = 3 * k1 + 2 * k2
    d = GRID[::4]
    x = d.copy()
    for a in range(k1 + 1):
        if a > 0:
            x = fast(x)
        y = x.copy()
        for b in range(1, 9):
            y = newton_schulz(y)
            if b >= 2 and 3 * a + 2 * b < products:
                e = np.max(d * np.abs(1.0 - y) / 2.0)
                assert 2 * math.sqrt(n - 1) * e > tol * 0.98, (a, b, e)


def matrix_sign_project(W, k1, k2):
    X = W / np.linalg.norm(W)
    for it in range(k1 + k2):
        Y = X @ X
        X = X @ ((3 * np.eye(len(W)) - 3.2 * Y + 1.2 * Y @ Y) if it < k1
                 else (1.5 * np.eye(len(W)) - 0.5 * Y))
        X = (X + X.T) / 2
    P = (W + W @ X) / 2
    return (P + P.T) / 2


@pytest.mark.parametrize("tol,n", [(1e-6, 16), (1e-6, 32), (1e-10, 16)])
def test_worst_case_matrices(tol, n):
    k1, k2 = sdp.sign_schedule(tol, n)
    _, dstar = worst_error(k1, k2)
    rng = np.random.default_rng(7)
    for trial in range(3):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        small = dstar * rng.choice([-1.0, 1.0], n - 1)
        lam = np.concatenate([[math.sqrt(1.0 - np.sum(small ** 2))], small]) * 10.0 ** trial
        W = (Q * lam) @ Q.T
        W = (W + W.T) / 2
        exact = (Q * np.maximum(lam, 0.0)) @ Q.T
        err = np.linalg.norm(matrix_sign_project(W, k1, k2) - exact) / np.linalg.norm(W)
        assert err <= tol / 2, (trial, err)
        # the bound is nearly attained: the schedule is not loose by much
        assert err >= tol / 2 / 3 ** 2, (trial, err)


@pytest.mark.parametrize("tol,n", CASES)
def test_never_more_than_the_earlier_rule(tol, n):
    k1, k2 = sdp.sign_schedule(tol, n)
    old_k1 = max(4, math.ceil(math.log(1.0 / tol) / math.log(3.0)))
    old_k2 = 3 if tol >= 1e-8 else 4
    assert 3 * k1 + 2 * k2 <= 3 * old_k1 + 2 * old_k2


def test_schedule_arguments():
    assert sdp.sign_schedule(1e-6, 1)[1] >= 2
    assert sdp.sign_schedule(0.0, 16) == sdp.sign_schedule(1e-16, 16)
    with pytest.raises(sdp.SdpError):
        sdp.sign_schedule(1e-6, 0)
