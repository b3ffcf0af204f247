"""The reference values the benchmark computes on the GPU, checked against the
oracle: the closed-form optimum and f* (used for every time-to-1e-6 record and
for the stability study), and the stability curves themselves (relative
objective and solution error per monitor point) on a small case.

Tolerances: f* to 1e-12 relative (f is flat at its minimum); w* to 1e-8
(a Cholesky solve of a matrix with condition number up to ~1e7); curve points:
solution errors within 1e-10 absolute (the FP64 iterate bar), objective errors
within 1e-12 + 1e-9 of their value."""

import numpy as np
import pytest
import torch

import bench
from oracle import bcd
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.mark.parametrize("fmt", ["f64", "bf16", "fp8"])
def test_closed_form_matches_oracle(gpu_lib, fmt):
    print("closed form", fmt, flush=True)
    X, y, _, _ = synth.colscaled_ridge(256, 16384, 31)
    lam = 1e-4
    Xd = X.to(DEV)
    if fmt != "f64":
        code = gpu_lib.BF16 if fmt == "bf16" else gpu_lib.FP8_E4M3
        Xd = gpu_lib.quantize(Xd, code).dequantize()
    w, f = bench.closed_form(gpu_lib, torch, Xd, y.to(DEV), lam)
    Xh, yn = Xd.cpu().numpy(), y.numpy()
    wo = bcd.ridge_closed_form(Xh, yn, lam)
    fo = bcd.primal_objective(Xh, yn, lam, wo)
    assert abs(f - fo) <= 1e-12 * fo
    assert np.linalg.norm(w.cpu().numpy() - wo) <= 1e-8 * np.linalg.norm(wo)


@pytest.mark.parametrize("dual", [False, True])
@pytest.mark.parametrize("s", [1, 8])
def test_stability_curve_matches_oracle(gpu_lib, dual, s):
    print("stability curve", dual, s, flush=True)
    if dual:
        X, y, _ = synth.spectral_ridge(32, 256, 1013, sigma_max=1e2)
    else:
        X, y, _ = synth.spectral_ridge(64, 1024, 1012, sigma_max=1e2)
    Xn, yn = X.numpy(), y.numpy()
    lam = 1000.0 / Xn.shape[1]
    H, points, b, seed = 4096, 8, 8, 3
    wstar = bcd.ridge_closed_form(Xn, yn, lam)
    fstar = bcd.primal_objective(Xn, yn, lam, wstar)
    A = (X.t().contiguous() if dual else X).to(DEV)
    got = bench.stability_curve(gpu_lib, torch, A, y.to(DEV), lam, b, s, H, points, seed,
                                torch.tensor(wstar, device=DEV), fstar, dual=dual)
    want = []
    chunk = H // points

    def mon(h, a_or_w, v):
        if h % chunk == 0:
            w = v if dual else a_or_w
            want.append((h, (bcd.primal_objective(Xn, yn, lam, w) - fstar) / fstar,
                         np.linalg.norm(w - wstar) / np.linalg.norm(wstar)))
    (bcd.dual_bcd if dual else bcd.primal_bcd)(Xn, yn, lam, b, s, H, seed, monitor=mon)
    assert [p[0] for p in got] == [p[0] for p in want]
    for (h, og, sg), (_, ow, sw) in zip(got, want):
        assert abs(og - ow) <= 1e-12 + 1e-9 * abs(ow), (h, og, ow)
        assert abs(sg - sw) <= 1e-10, (h, sg, sw)
