"""Calibration of the oracle's own rounding (CPU): the oracle self-spread.

The oracle sums in the order its matrix library chooses.  Permuting the
columns of X (the data points; y permuted alike) leaves every quantity of the
primal method unchanged in exact arithmetic (the Gram, Y z and the residual
update are sums over data points) but changes the order of every one of those
sums; permuting the rows of X does the same for the dual.  The distance
between the two runs is how far reordering alone moves the iterates, the
scale against which the GPU's 1e-10 bar is set: it must sit well below it.
"""

import numpy as np
import pytest

from oracle import bcd
import synth


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name,maker,lam,b,s,H", [
    ("gaussian 64x1024", lambda: synth.gaussian_ridge(64, 1024, 1000), 1e-3, 4, 8, 2000),
    ("spectral 256x8192 (spectrum 1..1e3)", lambda: synth.spectral_ridge(256, 8192, 1001), 1e-4,
     8, 32, 1024),
])
def test_primal_self_spread(name, maker, lam, b, s, H):
    X, y, _ = maker()
    X, y = X.numpy(), y.numpy()
    perm = np.random.default_rng(5).permutation(X.shape[1])
    w1, z1 = bcd.primal_bcd(X, y, lam, b, s, H, 2000)
    w2, z2 = bcd.primal_bcd(np.ascontiguousarray(X[:, perm]), y[perm], lam, b, s, H, 2000)
    sw, sz = _rel(w2, w1), _rel(z2[np.argsort(perm)], z1)
    print(f"{name}: self-spread w {sw:.2e}, z {sz:.2e}")
    assert 0.0 < sw <= 1e-12 and sz <= 1e-12


def test_dual_self_spread():
    X, y, _ = synth.gaussian_ridge(600, 300, 44)
    X, y = X.numpy(), y.numpy()
    perm = np.random.default_rng(6).permutation(X.shape[0])
    a1, w1 = bcd.dual_bcd(X, y, 1e-3, 8, 16, 1024, 7)
    a2, w2 = bcd.dual_bcd(np.ascontiguousarray(X[perm]), y, 1e-3, 8, 16, 1024, 7)
    sa, sw = _rel(a2, a1), _rel(w2[np.argsort(perm)], w1)
    print(f"dual 600x300: self-spread alpha {sa:.2e}, w {sw:.2e}")
    assert 0.0 < sa <= 1e-12 and sw <= 1e-12
