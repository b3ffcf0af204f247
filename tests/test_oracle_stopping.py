"""Pins of the oracle's stopping test (Section 5.1.5): the full primal and
dual residuals, and the runs stopped by their norms.

* The primal residual with the exact z is -grad f(w): checked against central
  differences of the objective (f is quadratic, so they are exact up to
  rounding), and it vanishes at the closed-form optimum.
* It bounds the objective error from both sides: with H = X X^T/n + lam I,
  f(w) - f* = 1/2 g^T H^{-1} g, so ||g||^2 / (2 L) <= f(w) - f* <= ||g||^2 / (2 lam)
  with L the largest eigenvalue of H (the paper uses the residual as an
  upper bound on the objective error).
* The dual residual with w = -X alpha/(lam n) is n grad D(alpha), and it
  vanishes at alpha* = X^T w* - y.
* A stopped run ends at the first check whose norm is <= tol and its iterate
  is the plain run's iterate after that many inner iterations (bitwise).
"""

import numpy as np
import pytest

from oracle import bcd
import synth


@pytest.fixture(scope="module")
def prob():
    X, y, _ = synth.gaussian_ridge(24, 300, 31)
    return X.numpy(), y.numpy(), 0.03


def _fd_grad(f, x, h=1e-3):
    g = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x)
        e[i] = h
        g[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


def test_primal_residual_is_minus_gradient(prob):
    X, y, lam = prob
    w = np.random.default_rng(1).standard_normal(X.shape[0])
    rho = bcd.primal_residual(X, y, lam, w, X.T @ w)
    g = _fd_grad(lambda v: bcd.primal_objective(X, y, lam, v), w)
    assert np.linalg.norm(rho + g) <= 1e-7 * np.linalg.norm(g)


def test_primal_residual_vanishes_at_optimum(prob):
    X, y, lam = prob
    ws = bcd.ridge_closed_form(X, y, lam)
    rho = bcd.primal_residual(X, y, lam, ws, X.T @ ws)
    assert np.linalg.norm(rho) <= 1e-12 * np.linalg.norm(X @ y / X.shape[1])


def test_primal_residual_brackets_objective_error(prob):
    X, y, lam = prob
    d, n = X.shape
    ws = bcd.ridge_closed_form(X, y, lam)
    fs = bcd.primal_objective(X, y, lam, ws)
    L = np.linalg.eigvalsh(X @ X.T / n + lam * np.eye(d))[-1]
    rng = np.random.default_rng(2)
    for scale in (1e-3, 1e-1, 1.0):
        w = ws + scale * rng.standard_normal(d)
        g2 = float(np.sum(bcd.primal_residual(X, y, lam, w, X.T @ w) ** 2))
        err = bcd.primal_objective(X, y, lam, w) - fs
        assert g2 / (2 * L) * (1 - 1e-9) <= err <= g2 / (2 * lam) * (1 + 1e-9)


def test_dual_residual_is_scaled_dual_gradient(prob):
    X, y, lam = prob
    n = X.shape[1]
    a = np.random.default_rng(3).standard_normal(n)
    w = -(X @ a) / (lam * n)
    rho = bcd.dual_residual(X, y, a, w)
    g = _fd_grad(lambda v: bcd.dual_objective(X, y, lam, v), a)
    assert np.linalg.norm(rho - n * g) <= 1e-7 * np.linalg.norm(n * g)


def test_dual_residual_vanishes_at_optimum(prob):
    X, y, lam = prob
    n = X.shape[1]
    ws = bcd.ridge_closed_form(X, y, lam)
    a = X.T @ ws - y
    rho = bcd.dual_residual(X, y, a, -(X @ a) / (lam * n))
    assert np.linalg.norm(rho) <= 1e-11 * np.linalg.norm(y)


@pytest.mark.parametrize("s,every", [(1, 1), (4, 3), (8, 2)])
def test_primal_stop_is_first_check_below_tol(prob, s, every):
    X, y, lam = prob
    H, b, seed = 4000, 4, 9
    norms = {}
    bcd.primal_bcd(X, y, lam, b, s, H, seed, monitor=lambda h, w, z: norms.__setitem__(
        h, float(np.linalg.norm(bcd.primal_residual(X, y, lam, w, z)))))
    hs = sorted(norms)
    tol = 1e-6 * norms[hs[0]]
    checks = [h for k, h in enumerate(hs, 1) if k % every == 0]
    want = next(h for h in checks if norms[h] <= tol)
    w, z, h, nrm = bcd.primal_bcd_tol(X, y, lam, b, s, H, seed, tol, every)
    assert h == want and nrm == norms[want]
    assert all(norms[c] > tol for c in checks if c < want)
    w2, z2 = bcd.primal_bcd(X, y, lam, b, s, want, seed)
    assert np.array_equal(w, w2) and np.array_equal(z, z2)
    # an unreachable tolerance runs all H iterations
    _, _, h, _ = bcd.primal_bcd_tol(X, y, lam, b, s, 40, seed, 0.0, every)
    assert h == 40


@pytest.mark.parametrize("s,every", [(1, 1), (5, 2)])
def test_dual_stop_is_first_check_below_tol(prob, s, every):
    X, y, lam = prob
    H, b, seed = 6000, 6, 4
    norms = {}
    bcd.dual_bcd(X, y, lam, b, s, H, seed, monitor=lambda h, a, w: norms.__setitem__(
        h, float(np.linalg.norm(bcd.dual_residual(X, y, a, w)))))
    hs = sorted(norms)
    tol = 1e-4 * np.linalg.norm(y)
    checks = [h for k, h in enumerate(hs, 1) if k % every == 0]
    want = next(h for h in checks if norms[h] <= tol)
    a, w, h, nrm = bcd.dual_bcd_tol(X, y, lam, b, s, H, seed, tol, every)
    assert h == want and nrm == norms[want]
    a2, w2 = bcd.dual_bcd(X, y, lam, b, s, want, seed)
    assert np.array_equal(a, a2) and np.array_equal(w, w2)
