"""The residual stopping test (Section 5.1.5) on the GPU against the oracle.

* Full residuals through cabcd_primal_residual / cabcd_dual_residual, element
  by element: dense FP64 (aligned, unaligned rows, rows long enough to be cut
  into parts), BF16 / FP8 storage (against the oracle on the dequantised
  matrix) and CSR.  Bound per entry: 1e-12 x the sum of the magnitudes that
  enter it (n u = 2e-12 at the largest n here is the worst case of a sum of n
  terms; the typical error is sqrt(n) u).
* Stopped runs: the tolerance is placed between two consecutive check norms
  of the oracle's run (so that a decision cannot flip on rounding), and the
  GPU run must stop after the same number of inner iterations as
  oracle.primal_bcd_tol / dual_bcd_tol, with iterates within 1e-10 relative.
"""

import numpy as np
import pytest
import scipy.sparse
import torch

from oracle import bcd
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _absX(X):
    return abs(X) if scipy.sparse.issparse(X) else np.abs(X)


@pytest.mark.parametrize("d,n,ld_pad", [(40, 3000, 0), (37, 20001, 0), (33, 50000, 3),
                                        (1, 9, 0), (300, 1000, 1)])
def test_primal_residual_dense_matches_oracle(gpu_lib, d, n, ld_pad):
    _say("primal residual dense", d, n, ld_pad)
    X, y, _ = synth.gaussian_ridge(d, n, 40 + d)
    Xc, yc = X.numpy(), y.numpy()
    rng = np.random.default_rng(d)
    w = rng.standard_normal(d)
    r = rng.standard_normal(n)
    lam = 3e-3
    Xd = X.to(DEV)
    if ld_pad:
        big = torch.zeros(d, n + ld_pad, dtype=torch.float64, device=DEV)
        big[:, :n] = Xd
        Xd = big[:, :n]
    norm, rho = gpu_lib.primal_residual(Xd, lam, torch.tensor(w, device=DEV),
                                        torch.tensor(r, device=DEV))
    ro = bcd.primal_residual(Xc, yc, lam, w, r + yc)
    bound = np.abs(Xc) @ np.abs(r) / n + lam * np.abs(w)
    assert np.all(np.abs(rho.cpu().numpy() - ro) <= 1e-12 * bound)
    assert abs(norm.item() - np.linalg.norm(ro)) <= 1e-12 * np.linalg.norm(bound)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
@pytest.mark.parametrize("d,n", [(24, 5000), (19, 70001)])
def test_primal_residual_lowp_matches_oracle(gpu_lib, dtype, d, n):
    _say("primal residual", dtype, d, n)
    X, y, _ = synth.gaussian_ridge(d, n, 60 + d)
    code = gpu_lib.BF16 if dtype == "bf16" else gpu_lib.FP8_E4M3
    Q = gpu_lib.quantize(X.to(DEV), code)
    Xh = Q.dequantize().cpu().numpy()
    rng = np.random.default_rng(n)
    w, r, lam = rng.standard_normal(d), rng.standard_normal(n), 1e-2
    norm, rho = gpu_lib.primal_residual(Q, lam, torch.tensor(w, device=DEV),
                                        torch.tensor(r, device=DEV))
    ro = bcd.primal_residual(Xh, y.numpy(), lam, w, r + y.numpy())
    bound = np.abs(Xh) @ np.abs(r) / n + lam * np.abs(w)
    assert np.all(np.abs(rho.cpu().numpy() - ro) <= 1e-12 * bound)
    assert abs(norm.item() - np.linalg.norm(ro)) <= 1e-12 * np.linalg.norm(bound)


def test_residuals_csr_match_oracle(gpu_lib):
    _say("residuals csr")
    rng = np.random.default_rng(5)
    S = scipy.sparse.random(400, 3000, density=0.02, format="csr", random_state=rng,
                            data_rvs=rng.standard_normal)
    S.sort_indices()
    y = rng.standard_normal(3000)
    w = rng.standard_normal(400)
    r = rng.standard_normal(3000)
    A = gpu_lib.CSR.from_scipy(S, DEV)
    norm, rho = gpu_lib.primal_residual(A, 1e-3, torch.tensor(w, device=DEV),
                                        torch.tensor(r, device=DEV))
    ro = bcd.primal_residual(S, y, 1e-3, w, r + y)
    bound = np.asarray(abs(S) @ np.abs(r)).ravel() / 3000 + 1e-3 * np.abs(w)
    assert np.all(np.abs(rho.cpu().numpy() - ro) <= 1e-12 * bound + 1e-300)
    # dual on A = X^T (rows = data points): X = S^T here
    XT = gpu_lib.CSR.from_scipy(S, DEV)            # n = 400 data points, d = 3000
    a = rng.standard_normal(400)
    yd = rng.standard_normal(400)
    wd = rng.standard_normal(3000)
    norm, rho = gpu_lib.dual_residual(XT, torch.tensor(yd, device=DEV),
                                      torch.tensor(a, device=DEV), torch.tensor(wd, device=DEV))
    ro = bcd.dual_residual(S.T.tocsr(), yd, a, wd)
    bound = np.asarray(abs(S) @ np.abs(wd)).ravel() + np.abs(a) + np.abs(yd)
    assert np.all(np.abs(rho.cpu().numpy() - ro) <= 1e-12 * bound)
    assert abs(norm.item() - np.linalg.norm(ro)) <= 1e-12 * np.linalg.norm(bound)


@pytest.mark.parametrize("d,n", [(64, 3000), (48, 20001)])
def test_dual_residual_dense_matches_oracle(gpu_lib, d, n):
    _say("dual residual dense", d, n)
    X, y, _ = synth.gaussian_ridge(d, n, 70 + d)
    Xc, yc = X.numpy(), y.numpy()
    rng = np.random.default_rng(7)
    a, w = rng.standard_normal(n), rng.standard_normal(d)
    XT = X.t().contiguous().to(DEV)
    norm, rho = gpu_lib.dual_residual(XT, y.to(DEV), torch.tensor(a, device=DEV),
                                      torch.tensor(w, device=DEV))
    ro = bcd.dual_residual(Xc, yc, a, w)
    bound = np.abs(Xc.T) @ np.abs(w) + np.abs(a) + np.abs(yc)
    assert np.all(np.abs(rho.cpu().numpy() - ro) <= 1e-12 * bound)


def _tol_between_checks(norms, target):
    """A tolerance strictly between the first check norm <= target and every
    earlier check norm (geometric mean with the smallest earlier one)."""
    c = next(i for i, v in enumerate(norms) if v <= target)
    prev = min(norms[:c])
    tol = float(np.sqrt(prev * norms[c]))
    assert prev / norms[c] > 1.002, "check norms too close for a robust decision"
    return tol


@pytest.mark.parametrize("s,every", [(1, 4), (5, 2), (8, 1)])
def test_primal_stops_where_oracle_stops(gpu_lib, s, every):
    _say("primal stop", s, every)
    d, n, b, lam, seed, H = 60, 4001, 4, 1e-3, 31, 1000
    X, y, _ = synth.gaussian_ridge(d, n, 77)
    Xc, yc = X.numpy(), y.numpy()
    norms = []
    k = [0]

    def mon(h, w, z):
        k[0] += 1
        if k[0] % every == 0:
            norms.append(float(np.linalg.norm(bcd.primal_residual(Xc, yc, lam, w, z))))

    bcd.primal_bcd(Xc, yc, lam, b, s, H, seed, monitor=mon)
    rho0 = np.linalg.norm(Xc @ yc / n)
    tol = _tol_between_checks(norms, 1e-5 * rho0)
    wo, zo, ho, no = bcd.primal_bcd_tol(Xc, yc, lam, b, s, H, seed, tol, every)
    assert ho < H
    st = {}
    w, r = gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), lam, b, s, H, seed, tol=tol,
                              check_every=every, stats=st)
    _say(f"  oracle stops at h = {ho} (norm {no:.3e}, tol {tol:.3e}); gpu at {st['h']}")
    assert st["h"] == ho
    assert _rel(w.cpu(), wo) <= 1e-10
    assert _rel(r.cpu(), zo - yc) <= 1e-10
    assert abs(st["resid_norm"] - no) <= 1e-6 * no


def test_primal_checks_without_tolerance_run_to_h(gpu_lib):
    _say("primal checks, tol 0")
    X, y, _ = synth.gaussian_ridge(30, 2000, 5)
    st = {}
    w, r = gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), 1e-2, 3, 4, 101, 9, tol=0.0,
                              check_every=3, stats=st)
    assert st["h"] == 101
    wo, zo, h, no = bcd.primal_bcd_tol(X.numpy(), y.numpy(), 1e-2, 3, 4, 101, 9, 0.0, 3)
    assert h == 101 and _rel(w.cpu(), wo) <= 1e-10
    assert abs(st["resid_norm"] - no) <= 1e-8 * no
    tm = gpu_lib.new_timing()
    gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), 1e-2, 3, 4, 40, 9, check_every=2, timing=tm)
    assert gpu_lib.timing_dict(tm)["check"]["launches"] == 5   # ceil(40/4) = 10 steps
    # a timing mask brackets the selected phases only
    tm = gpu_lib.new_timing()
    gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), 1e-2, 3, 4, 40, 9, check_every=2, timing=tm,
                       timing_mask=1 << gpu_lib.PHASES.index("gram"))
    counts = {k: v["launches"] for k, v in gpu_lib.timing_dict(tm).items()}
    # ten steps: one Gram launch each, or fewer when Grams are computed ahead
    assert 1 <= counts["gram"] <= 10 and sum(counts.values()) == counts["gram"]


def test_primal_lowp_stops_where_oracle_stops(gpu_lib):
    _say("primal bf16 stop")
    d, n, b, s, lam, seed, H, every = 40, 6000, 8, 4, 1e-3, 3, 4000, 2
    X, y, _ = synth.gaussian_ridge(d, n, 91)
    Q = gpu_lib.quantize(X.to(DEV), gpu_lib.BF16)
    Xh, yc = Q.dequantize().cpu().numpy(), y.numpy()
    st = {}
    w, r = gpu_lib.primal_bcd(Q, y.to(DEV), lam, b, s, H, seed, tol=1e-6 * np.linalg.norm(
        Xh @ yc / n), check_every=every, stats=st)
    assert st["h"] < H
    # the stopping claim itself: the full residual of the returned w is small
    norm, _ = gpu_lib.primal_residual(Q, lam, w, r)
    assert norm.item() == st["resid_norm"]
    ro = bcd.primal_residual(Xh, yc, lam, w.cpu().numpy(), Xh.T @ w.cpu().numpy())
    assert np.linalg.norm(ro) <= 1.01e-6 * np.linalg.norm(Xh @ yc / n)


@pytest.mark.parametrize("s,every", [(1, 3), (6, 1)])
def test_dual_stops_where_oracle_stops(gpu_lib, s, every):
    _say("dual stop", s, every)
    d, n, b, lam, seed, H = 40, 1500, 6, 1e-2, 17, 8000
    X, y, _ = synth.gaussian_ridge(d, n, 78)
    Xc, yc = X.numpy(), y.numpy()
    norms = []
    k = [0]

    def mon(h, a, w):
        k[0] += 1
        if k[0] % every == 0:
            norms.append(float(np.linalg.norm(bcd.dual_residual(Xc, yc, a, w))))

    bcd.dual_bcd(Xc, yc, lam, b, s, H, seed, monitor=mon)
    tol = _tol_between_checks(norms, 1e-3 * np.linalg.norm(yc))
    ao, wo, ho, no = bcd.dual_bcd_tol(Xc, yc, lam, b, s, H, seed, tol, every)
    assert ho < H
    st = {}
    a, w = gpu_lib.dual_bcd(X.t().contiguous().to(DEV), y.to(DEV), lam, b, s, H, seed, tol=tol,
                            check_every=every, stats=st)
    _say(f"  oracle stops at h = {ho}; gpu at {st['h']}")
    assert st["h"] == ho
    assert _rel(a.cpu(), ao) <= 1e-10
    assert _rel(w.cpu(), wo) <= 1e-10
    assert abs(st["resid_norm"] - no) <= 1e-6 * no


def test_nonfinite_residual_stops_and_is_reported(gpu_lib):
    _say("nan residual")
    X, y, _ = synth.gaussian_ridge(20, 500, 8)
    Xd = X.to(DEV)
    Xd[4, 7] = float("nan")
    st = {}
    with pytest.raises(gpu_lib.CabcdError) as e:
        gpu_lib.primal_bcd(Xd, y.to(DEV), 1e-2, 4, 2, 400, 1, tol=1e-3, check_every=1, stats=st)
    assert e.value.status in (gpu_lib.ENOTSPD, gpu_lib.ENONFINITE)
