"""HIP path vs the CPU oracle, element by element, through the C-ABI.

Tolerances (FP64 path):
* sampler: bit-exact (integer work);
* Gram: |G_gpu - G_oracle| <= 1e-12 * scale * (|Y| |Y|^T) elementwise: both sides
  sum the same products in different orders, so the difference is bounded by a
  few multiples of sqrt(K) u |Y||Y|^T (Higham's dot-product bound is K u), far
  below 1e-12 for K <= 2^20;
* iterates: ||w_gpu - w_oracle|| / ||w_oracle|| <= 1e-10 after H iterations on
  the same blocks (the same for alpha and for the companion vector).
"""

import numpy as np
import pytest
import torch

from oracle import bcd, sampler
import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ------------------------------------------------------------------ sampler

@pytest.mark.parametrize("seed,h0,count,b,rng", [
    (2000, 0, 300, 8, 2048), (1, 12345, 50, 16, 20000), (7, 0, 40, 4, 4),
    (2**63 + 5, 999, 30, 3, 262144), (42, 0, 5, 64, 64), (3, 77, 64, 1, 1)])
def test_sampler_bit_exact(gpu_lib, seed, h0, count, b, rng):
    _say("sampler", seed, h0, count, b, rng)
    got = gpu_lib.sample(seed, h0, count, b, rng).cpu().numpy()
    want = np.array(sampler.sample_blocks(seed, h0, count, b, rng), dtype=np.int32)
    assert np.array_equal(got, want)


# ------------------------------------------------------------------ Gram

@pytest.mark.parametrize("m,cols", [(1, 1), (5, 7), (16, 300), (17, 301), (32, 4097),
                                    (33, 1000), (64, 2049), (100, 5000), (128, 777),
                                    (200, 3001), (256, 20000), (256, 65),
                                    # LDS-DMA path (128 < m <= 256, even cols): one, two
                                    # and three tiles per slab, a partial last tile
                                    (129, 16), (256, 32), (256, 48), (160, 1000),
                                    (250, 4098),
                                    # three tiles in rotation: four and five tiles per
                                    # slab, and many with a partial last one
                                    (256, 64), (256, 80), (192, 4130),
                                    # LDS-DMA path for m <= 128 (even cols): every block
                                    # class, several tiles per slab, partial tiles
                                    (8, 770), (32, 4096), (20, 5000), (64, 2048),
                                    (128, 778), (100, 40000), (128, 65536)])
def test_gram_matches_oracle(gpu_lib, m, cols):
    _say("gram", m, cols)
    rows = max(m + 3, 40)
    g = torch.Generator().manual_seed(m * 1000 + cols)
    A = torch.randn(rows, cols, generator=g, dtype=torch.float64)
    u = torch.randn(cols, generator=g, dtype=torch.float64)
    idx = torch.randint(0, rows, (m,), generator=g, dtype=torch.int32)
    scale, shift = 1.0 / cols, 0.37
    G, Yu = gpu_lib.gram(A.to(DEV), idx.to(DEV), scale, shift, u.to(DEV))
    G = G.cpu().numpy()
    Yu = Yu.cpu().numpy()
    Go, Yo = bcd.gram(A.numpy(), idx.numpy(), scale, shift, u.numpy())
    Y = np.abs(A.numpy()[idx.numpy()])
    bound = 1e-12 * scale * (Y @ Y.T) + 1e-300
    assert np.all(np.abs(G - Go) <= bound)
    assert np.array_equal(G, G.T)
    ubound = 1e-12 * (Y @ np.abs(u.numpy())) + 1e-300
    assert np.all(np.abs(Yu - Yo) <= ubound)


def test_gram_unaligned_leading_dimension(gpu_lib):
    _say("gram unaligned ld")
    g = torch.Generator().manual_seed(5)
    base = torch.randn(50, 1001, generator=g, dtype=torch.float64)
    A = base[:, 1:]
    Ad = base.to(DEV)[:, 1:]   # odd ld and every row start misaligned by 8 bytes
    assert Ad.stride(0) == 1001 and Ad.data_ptr() % 16 == 8
    idx = torch.tensor([3, 49, 0, 17, 3], dtype=torch.int32)
    G, _ = gpu_lib.gram(Ad, idx.to(DEV), 1.0, 0.0)
    Go, _ = bcd.gram(A.numpy(), idx.numpy(), 1.0, 0.0)
    Y = np.abs(A.numpy()[idx.numpy()])
    assert np.all(np.abs(G.cpu().numpy() - Go) <= 1e-12 * (Y @ Y.T))


# ------------------------------------------------------------------ primal

PRIMAL_CASES = [
    # d, n, b, s, H, lam, seed
    (64, 1024, 4, 8, 400, 1e-3, 2000),     # the small dense configuration's shape
    (64, 1024, 4, 1, 120, 1e-3, 2000),     # BCD (s = 1)
    (300, 5000, 8, 4, 37, 1e-2, 11),       # ragged last outer step, several tiles
    (20, 333, 3, 5, 23, 0.05, 3),          # odd n (unaligned rows), overlapping blocks
    (40, 777, 16, 16, 33, 1e-3, 9),        # sb = 256, overlaps across blocks
    (9, 50, 9, 1, 2, 0.1, 1),              # b = d: one Newton step
    (10, 400, 8, 32, 70, 0.1, 4),          # sb = 256 over 10 coordinates: ~25 repeats each
    (30, 300, 17, 15, 40, 0.1, 8),         # b = 17, one row per thread: ~8.5 repeats each
]


@pytest.mark.parametrize("d,n,b,s,H,lam,seed", PRIMAL_CASES)
def test_primal_matches_oracle(gpu_lib, d, n, b, s, H, lam, seed):
    _say("primal", d, n, b, s, H, lam, seed)
    X, y, _ = synth.gaussian_ridge(d, n, 100 + d)
    w, r = gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), lam, b, s, H, seed)
    wo, zo = bcd.primal_bcd(X.numpy(), y.numpy(), lam, b, s, H, seed)
    assert _rel(w.cpu(), wo) <= 1e-10
    assert _rel(r.cpu(), zo - y.numpy()) <= 1e-10


def test_primal_s_steps_equal_classical_on_gpu(gpu_lib):
    _say("primal s-equivalence")
    X, y, _ = synth.gaussian_ridge(64, 1024, 1000)
    Xd, yd = X.to(DEV), y.to(DEV)
    w1, _ = gpu_lib.primal_bcd(Xd, yd, 1e-3, 4, 1, 256, 2000)
    w8, _ = gpu_lib.primal_bcd(Xd, yd, 1e-3, 4, 8, 256, 2000)
    assert _rel(w8.cpu(), w1.cpu()) <= 1e-12


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_dual_s_steps_equal_classical_on_gpu(gpu_lib, kind):
    """The s-step dual reproduces BDCD (s = 1) on the same blocks: FP64 iterates
    agree to rounding (Section 3's claim, checked on the GPU path itself)."""
    _say("dual s-equivalence", kind)
    X, y, _ = synth.gaussian_ridge(80, 600, 44)
    XT = X.t().contiguous()
    if kind == "csr":
        import scipy.sparse
        A = gpu_lib.CSR.from_scipy(scipy.sparse.csr_matrix(XT.numpy()), DEV)
    else:
        A = XT.to(DEV)
    yd = y.to(DEV)
    a1, w1 = gpu_lib.dual_bcd(A, yd, 1e-2, 6, 1, 360, 9)
    for s in (3, 12, 40):
        a, w = gpu_lib.dual_bcd(A, yd, 1e-2, 6, s, 360, 9)
        assert _rel(a.cpu(), a1.cpu()) <= 1e-12
        assert _rel(w.cpu(), w1.cpu()) <= 1e-12


def test_primal_converges_to_closed_form(gpu_lib):
    _say("primal convergence")
    X, y, _ = synth.gaussian_ridge(64, 1024, 1000)
    wstar = bcd.ridge_closed_form(X.numpy(), y.numpy(), 1e-3)
    w, _ = gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), 1e-3, 4, 8, 2000, 2000)
    assert _rel(w.cpu(), wstar) <= 1e-10


def test_primal_resume_is_exact(gpu_lib):
    _say("primal resume")
    X, y, _ = synth.gaussian_ridge(50, 600, 4)
    Xd, yd = X.to(DEV), y.to(DEV)
    wa, ra = gpu_lib.primal_bcd(Xd, yd, 1e-2, 5, 4, 80, 17)
    wb, rb = gpu_lib.primal_bcd(Xd, yd, 1e-2, 5, 4, 40, 17)
    wb, rb = gpu_lib.primal_bcd(Xd, yd, 1e-2, 5, 4, 40, 17, w=wb, r=rb, h0=40,
                                flags=gpu_lib.FLAG_STATE_VALID)
    assert torch.equal(wa, wb) and torch.equal(ra, rb)


def test_primal_explicit_indices(gpu_lib):
    _say("primal explicit idx")
    X, y, _ = synth.gaussian_ridge(12, 100, 5)
    blocks = [[0, 1, 2], [2, 3, 4], [4, 5, 0], [6, 7, 8], [9, 10, 11], [11, 0, 3], [1, 5, 9]]
    idx = torch.tensor(blocks, dtype=torch.int32, device=DEV)
    w, _ = gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), 0.1, 3, 3, len(blocks), 0,
                              explicit_idx=idx)
    wo, _ = bcd.primal_bcd(X.numpy(), y.numpy(), 0.1, 3, 3, len(blocks), 0,
                           explicit_idx=blocks)
    assert _rel(w.cpu(), wo) <= 1e-12
    bad = torch.tensor([[0, 0, 1]], dtype=torch.int32, device=DEV)
    with pytest.raises(gpu_lib.CabcdError):
        gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), 0.1, 3, 1, 1, 0, explicit_idx=bad)


def test_primal_monitor_and_recompute(gpu_lib):
    _say("primal monitor")
    X, y, _ = synth.gaussian_ridge(30, 400, 6)
    lam = 1e-2
    trace = torch.zeros(5, dtype=torch.float64, device=DEV)
    w, r = gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), lam, 3, 4, 40, 8, resid_every=2,
                              monitor_every=2, trace=trace)
    fs = []
    bcd.primal_bcd(X.numpy(), y.numpy(), lam, 3, 4, 40, 8,
                   monitor=lambda h, w_, z_: fs.append(bcd.primal_objective(X.numpy(), y.numpy(), lam, w_)))
    want = np.array(fs[1::2])
    assert np.allclose(trace.cpu().numpy(), want, rtol=1e-12, atol=0)
    # after an exact recompute the residual equals X^T w - y
    r_exact = X.numpy().T @ w.cpu().numpy() - y.numpy()
    assert _rel(r.cpu(), r_exact) <= 1e-12


def test_primal_monitor_from_maintained_residual(gpu_lib):
    _say("primal monitor, maintained residual")
    X, y, _ = synth.gaussian_ridge(30, 400, 6)
    lam = 1e-2
    trace = torch.zeros(10, dtype=torch.float64, device=DEV)
    gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), lam, 3, 4, 40, 8, monitor_every=1, trace=trace,
                       flags=gpu_lib.FLAG_MONITOR_MAINTAINED)
    fs = []
    bcd.primal_bcd(X.numpy(), y.numpy(), lam, 3, 4, 40, 8,
                   monitor=lambda h, w_, z_: fs.append(bcd.primal_objective(X.numpy(), y.numpy(), lam, w_)))
    assert np.allclose(trace.cpu().numpy(), np.array(fs), rtol=1e-12, atol=0)


def test_primal_nan_is_reported(gpu_lib):
    _say("primal nan")
    X, y, _ = synth.gaussian_ridge(10, 64, 7)
    X[3, 5] = float("nan")
    with pytest.raises(gpu_lib.CabcdError) as e:
        gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), 0.1, 10, 1, 1, 0)
    assert e.value.status in (gpu_lib.ENOTSPD, gpu_lib.ENONFINITE)


def test_primal_h_zero_keeps_w(gpu_lib):
    X, y, _ = synth.gaussian_ridge(10, 64, 7)
    w0 = torch.linspace(-1, 1, 10, dtype=torch.float64, device=DEV)
    w, r = gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), 0.1, 2, 2, 0, 0, w=w0.clone())
    assert torch.equal(w, w0)
    assert _rel(r.cpu(), X.numpy().T @ w0.cpu().numpy() - y.numpy()) <= 1e-14


# ------------------------------------------------------------------ dual

DUAL_CASES = [
    # d, n, b, s, H, lam, seed
    (30, 200, 8, 6, 300, 0.05, 77),
    (30, 200, 8, 1, 100, 0.05, 77),
    (500, 300, 16, 8, 45, 1e-3, 5),        # d > n: the dual's natural shape
    (77, 1001, 5, 7, 33, 1e-2, 2),         # odd d (unaligned rows of X^T)
    (12, 30, 30, 1, 2, 0.03, 1),           # b' = n: one exact step
    (40, 12, 4, 32, 40, 0.1, 6),           # 128 rows over 12 samples: ~11 repeats each
    (200, 300, 20, 4, 40, 1e-2, 12),       # b = 20: Grams ahead, one row per thread
]


@pytest.mark.parametrize("d,n,b,s,H,lam,seed", DUAL_CASES)
def test_dual_matches_oracle(gpu_lib, d, n, b, s, H, lam, seed):
    _say("dual", d, n, b, s, H, lam, seed)
    X, y, _ = synth.gaussian_ridge(d, n, 300 + d)
    XT = X.t().contiguous()
    a, w = gpu_lib.dual_bcd(XT.to(DEV), y.to(DEV), lam, b, s, H, seed)
    ao, wo = bcd.dual_bcd(X.numpy(), y.numpy(), lam, b, s, H, seed)
    assert _rel(a.cpu(), ao) <= 1e-10
    assert _rel(w.cpu(), wo) <= 1e-10


def test_dual_link_and_objective(gpu_lib):
    _say("dual link")
    X, y, _ = synth.gaussian_ridge(30, 200, 21)
    lam = 0.05
    XT = X.t().contiguous().to(DEV)
    a, w = gpu_lib.dual_bcd(XT, y.to(DEV), lam, 8, 6, 3000, 77)
    w_link = gpu_lib.dual_to_primal(XT, a, lam)
    assert _rel(w.cpu(), w_link.cpu()) <= 1e-10
    wstar = bcd.ridge_closed_form(X.numpy(), y.numpy(), lam)
    assert _rel(w.cpu(), wstar) <= 1e-10
    f, _ = gpu_lib.primal_objective_t(XT, y.to(DEV), lam, w)
    fo = bcd.primal_objective(X.numpy(), y.numpy(), lam, w.cpu().numpy())
    assert abs(f.item() - fo) <= 1e-13 * fo


def test_primal_objective_matches(gpu_lib):
    X, y, _ = synth.gaussian_ridge(70, 3001, 8)
    w = torch.randn(70, dtype=torch.float64)
    f, r = gpu_lib.primal_objective(X.to(DEV), y.to(DEV), 0.3, w.to(DEV))
    fo = bcd.primal_objective(X.numpy(), y.numpy(), 0.3, w.numpy())
    assert abs(f.item() - fo) <= 1e-13 * fo
    assert _rel(r.cpu(), X.numpy().T @ w.numpy() - y.numpy()) <= 1e-14
