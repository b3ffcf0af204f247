"""The stability study on the oracle (CPU): with one block sequence, the
s-step method's relative objective and solution errors match those of s = 1 at
every monitor point (exact-arithmetic equivalence, Section 3, up to rounding),
and the run reaches the FP64 floor.  Small stand-in with the paper's
regularisation rule (lambda = 1000 x the smallest eigenvalue of X X^T / n)."""

import numpy as np
import pytest

from oracle import bcd
import synth


def _curve(X, y, lam, b, s, H, points, seed, dual):
    wstar = bcd.ridge_closed_form(X, y, lam)
    fstar = bcd.primal_objective(X, y, lam, wstar)
    chunk = H // points
    pts = []

    def mon(h, a_or_w, v):
        if h % chunk == 0:
            w = v if dual else a_or_w
            pts.append((h, (bcd.primal_objective(X, y, lam, w) - fstar) / fstar,
                        np.linalg.norm(w - wstar) / np.linalg.norm(wstar)))
    run = bcd.dual_bcd if dual else bcd.primal_bcd
    run(X, y, lam, b, s, H, seed, monitor=mon)
    return pts


@pytest.mark.parametrize("dual", [False, True])
def test_oracle_curves_equal_across_s_and_converge(dual):
    if dual:
        X, y, _ = synth.spectral_ridge(32, 256, 1013, sigma_max=1e2)
        H = 4096
    else:
        X, y, _ = synth.spectral_ridge(64, 1024, 1012, sigma_max=1e2)
        H = 4096
    X, y = X.numpy(), y.numpy()
    lam = 1000.0 / X.shape[1]
    base = _curve(X, y, lam, 8, 1, H, 8, 3, dual)
    assert len(base) == 8
    for s in (2, 4, 8, 16):
        c = _curve(X, y, lam, 8, s, H, 8, 3, dual)
        assert [p[0] for p in c] == [p[0] for p in base]
        for (h, o1, e1), (_, o2, e2) in zip(base, c):
            assert abs(o2 - o1) <= 1e-12 + 1e-9 * abs(o1), (s, h)
            assert abs(e2 - e1) <= 1e-12, (s, h)
    assert base[-1][1] <= 1e-14 and base[-1][2] <= 1e-10
