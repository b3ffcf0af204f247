"""Whole outer steps through the driver paths the benchmarks time, the b = 1
case of the paper's headline speedups, and the solver's edge cases, against the
CPU oracle through the C-ABI.

Which driver path a run took is read from the phase launch counts that
`opts.timing` returns:
* one Gram per outer step (gathered rows of more than 8 MiB, or a ragged last
  step): `gram` and `reduce` once per outer step, no `yu` pass;
* Grams computed ahead (short rows, CSR): one `gram` launch for many outer
  steps and a separate `yu` row-product pass per step.

Tolerances:
* FP64 iterates: 1e-10 relative (the bar of the FP64 path); where a block is
  ill-conditioned the bound is stated from kappa u (see the test);
* mixed precision: relative objective error 1e-6 on the dequantised problem
  (X^, y, lambda) and an exact residual recomputation to 1e-12.
"""

import numpy as np
import pytest
import scipy.sparse
import torch

from oracle import bcd
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
U64 = 2.0 ** -53


def _say(*a):
    print(*a, flush=True)


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _launches(gpu_lib, t):
    return {k: v["launches"] for k, v in gpu_lib.timing_dict(t).items()}


def _assert_per_step(gpu_lib, t, steps, updates=None):
    n = _launches(gpu_lib, t)
    _say("  launches", n)
    assert n["yu"] == 0, "expected one fused Gram per outer step"
    assert n["gram"] == steps and n["reduce"] == steps and n["solve"] == steps
    if updates is not None:   # updates not left to the next step's Gram
        assert n["update"] == updates


# ------------------------------------------------------------------ one Gram per step

@pytest.mark.parametrize("fold", [False, True])
def test_primal_fp64_per_step_path_full_steps(gpu_lib, fold):
    """Headline path at a shard shape: b = 8, s = 32 (sb = 256), rows of
    32768 FP64 values (64 MiB gathered per step), three full outer steps and a
    ragged one; the spectrum of the headline matrix (1 .. 1e3).  With and
    without the companion update folded into the next step's Gram."""
    d, n, b, s, lam, seed = 512, 32768, 8, 32, 1e-4, 2001
    H = 3 * s + 5
    _say("primal per-step", d, n, b, s, H, "fold" if fold else "")
    X, y, _ = synth.spectral_ridge(d, n, 1001)
    t = gpu_lib.new_timing()
    w, r = gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), lam, b, s, H, seed, timing=t,
                              flags=gpu_lib.FLAG_FOLD_UPDATE if fold else 0)
    # folded: the updates of steps 1 and 2 run inside the Grams of steps 2
    # and 3; step 3's runs alone (no full step follows), as does the ragged
    # step's
    _assert_per_step(gpu_lib, t, 4, updates=2 if fold else 4)
    trace = []
    wo, zo = bcd.primal_bcd(X.numpy(), y.numpy(), lam, b, s, H, seed,
                            monitor=lambda h, w_, z_: trace.append(h))
    assert trace == [32, 64, 96, 101]
    e_w, e_r = _rel(w.cpu(), wo), _rel(r.cpu(), zo - y.numpy())
    _say(f"  rel err w {e_w:.2e}, r {e_r:.2e}")
    assert e_w <= 1e-10 and e_r <= 1e-10


@pytest.fixture(scope="module")
def headline_matrix(gpu_lib):
    """The benchmark's headline matrix: d = 2048, n = 2^18, spectrum 1 .. 1e3,
    generated as the benchmark generates it, stored with its rows leading_dim
    apart on the GPU; with its host copy for the oracle."""
    d, n = 2048, 1 << 18
    X, y, _ = synth.spectral_ridge(d, n, 1001, device=DEV)
    Xc, yc = X.cpu().numpy(), y.cpu().numpy()
    Xp = gpu_lib.empty_dense(d, n, DEV)
    Xp.copy_(X)
    del X
    torch.cuda.empty_cache()
    yield Xp, y, Xc, yc
    del Xp
    torch.cuda.empty_cache()


def test_primal_headline_size_full_steps(gpu_lib, headline_matrix):
    """The benchmark's own workload and launch configuration: d = 2048,
    n = 2^18, b = 8, s = 32 (sb = 256), lambda = 1e-4, X stored with its rows
    leading_dim apart; three full outer steps through the one-Gram-per-step
    path, without and with the update folded into the next step's Gram; every
    entry of w and r against the oracle's run of the same steps."""
    Xp, y, Xc, yc = headline_matrix
    d, n = Xc.shape
    b, s, lam, seed = 8, 32, 1e-4, 7
    H = 3 * s
    _say("primal headline size", d, n, b, s, H)
    assert Xp.stride(0) == gpu_lib.leading_dim(n, gpu_lib.F64) != n
    wo, zo = bcd.primal_bcd(Xc, yc, lam, b, s, H, seed)
    for fold in (False, True):
        t = gpu_lib.new_timing()
        w, r = gpu_lib.primal_bcd(Xp, y, lam, b, s, H, seed, timing=t,
                                  flags=gpu_lib.FLAG_FOLD_UPDATE if fold else 0)
        _assert_per_step(gpu_lib, t, 3, updates=1 if fold else 3)
        e_w, e_r = _rel(w.cpu(), wo), _rel(r.cpu(), zo - yc)
        _say(f"  {'fold' if fold else 'plain'}: rel err w {e_w:.2e}, r {e_r:.2e}")
        assert e_w <= 1e-10 and e_r <= 1e-10


@pytest.mark.parametrize("s", [1, 4, 16])
def test_primal_headline_matrix_s_sweep(gpu_lib, headline_matrix, s):
    """The s sweep of the benchmark on the headline matrix (b = 8, s = 1, 4,
    16: one Gram per outer step of 8 to 128 gathered rows of 2 MiB), four
    outer steps against the oracle."""
    Xp, y, Xc, yc = headline_matrix
    b, lam, seed = 8, 1e-4, 2001
    H = 4 * s
    _say("primal headline matrix, s =", s)
    w, r = gpu_lib.primal_bcd(Xp, y, lam, b, s, H, seed)
    wo, zo = bcd.primal_bcd(Xc, yc, lam, b, s, H, seed)
    e_w, e_r = _rel(w.cpu(), wo), _rel(r.cpu(), zo - yc)
    _say(f"  rel err w {e_w:.2e}, r {e_r:.2e}")
    assert e_w <= 1e-10 and e_r <= 1e-10


def test_dual_headline_matrix(gpu_lib, headline_matrix):
    """The benchmark's dense dual: A = X^T of the headline matrix (2^18 data
    points of 2048 features), b = 8, s = 1, 4, 16, 32 (the Grams of future
    steps computed ahead), four outer steps each against the oracle."""
    Xp, y, Xc, yc = headline_matrix
    XT = Xp.t().contiguous()
    b, lam, seed = 8, 1e-4, 2001
    for s in (1, 4, 16, 32):
        H = 4 * s
        a, w = gpu_lib.dual_bcd(XT, y, lam, b, s, H, seed)
        ao, wo = bcd.dual_bcd(Xc, yc, lam, b, s, H, seed)
        e_a, e_w = _rel(a.cpu(), ao), _rel(w.cpu(), wo)
        _say(f"  dual s={s}: rel err alpha {e_a:.2e}, w {e_w:.2e}")
        assert e_a <= 1e-10 and e_w <= 1e-10
    del XT
    torch.cuda.empty_cache()


def test_dual_fp64_per_step_path_full_steps(gpu_lib):
    """Dual on A = X^T with rows of 6000 features: 12 MiB gathered per step at
    sb = 256, so each outer step forms its own Gram with Y w fused."""
    d, n, b, s, lam, seed = 6000, 3000, 8, 32, 1e-3, 7
    H = 3 * s + 5
    _say("dual per-step", d, n, b, s, H)
    X, y, _ = synth.gaussian_ridge(d, n, 606)
    XT = X.t().contiguous()
    t = gpu_lib.new_timing()
    a, w = gpu_lib.dual_bcd(XT.to(DEV), y.to(DEV), lam, b, s, H, seed, timing=t)
    _assert_per_step(gpu_lib, t, 4)
    ao, wo = bcd.dual_bcd(X.numpy(), y.numpy(), lam, b, s, H, seed)
    e_a, e_w = _rel(a.cpu(), ao), _rel(w.cpu(), wo)
    _say(f"  rel err alpha {e_a:.2e}, w {e_w:.2e}")
    assert e_a <= 1e-10 and e_w <= 1e-10


def test_folded_update_resume_is_bitwise(gpu_lib):
    """CABCD_FLAG_FOLD_UPDATE at s b = 256 with one Gram per step: a full
    step's companion update is applied inside the next step's Gram kernel, or
    on its own before a ragged step, a check or the end of a call, by the
    same device code.  The same run in one call and split in two (h0, state
    passed on) is bitwise equal, though the split moves one update from folded
    to alone; both match the oracle, and the unfolded run to rounding.
    Primal and dual."""
    d, n, b, s, lam, seed = 512, 8192, 8, 32, 1e-4, 2003
    X, y, _ = synth.spectral_ridge(d, n, 1003)
    Xd, yd = X.to(DEV), y.to(DEV)
    H = 5 * s
    fold = gpu_lib.FLAG_FOLD_UPDATE
    w1, r1 = gpu_lib.primal_bcd(Xd, yd, lam, b, s, H, seed, flags=fold)
    w2, r2 = gpu_lib.primal_bcd(Xd, yd, lam, b, s, 2 * s, seed, flags=fold)
    gpu_lib.primal_bcd(Xd, yd, lam, b, s, 3 * s, seed, w=w2, r=r2, h0=2 * s,
                       flags=gpu_lib.FLAG_STATE_VALID | fold)
    assert torch.equal(w1, w2) and torch.equal(r1, r2)
    wo, zo = bcd.primal_bcd(X.numpy(), y.numpy(), lam, b, s, H, seed)
    assert _rel(w1.cpu(), wo) <= 1e-10 and _rel(r1.cpu(), zo - y.numpy()) <= 1e-10
    w0, r0 = gpu_lib.primal_bcd(Xd, yd, lam, b, s, H, seed)
    assert _rel(w1.cpu(), w0.cpu()) <= 1e-12 and _rel(r1.cpu(), r0.cpu()) <= 1e-12
    # dual with the same 512 x 8192 matrix as A = X^T: 512 data points of
    # 8192 features (16 MiB gathered per step)
    yt = torch.tensor(np.random.default_rng(9).standard_normal(d))
    ytd = yt.to(DEV)
    a1, v1 = gpu_lib.dual_bcd(Xd, ytd, 1e-2, b, s, 4 * s, seed, flags=fold)
    a2, v2 = gpu_lib.dual_bcd(Xd, ytd, 1e-2, b, s, 3 * s, seed, flags=fold)
    gpu_lib.dual_bcd(Xd, ytd, 1e-2, b, s, s, seed, alpha=a2, w=v2, h0=3 * s,
                     flags=gpu_lib.FLAG_STATE_VALID | fold)
    assert torch.equal(a1, a2) and torch.equal(v1, v2)
    ao, vo = bcd.dual_bcd(X.numpy().T.copy(), yt.numpy(), 1e-2, b, s, 4 * s, seed)
    assert _rel(a1.cpu(), ao) <= 1e-10 and _rel(v1.cpu(), vo) <= 1e-10


def test_folded_update_with_monitor_and_checks(gpu_lib):
    """Monitor points, exact recomputations and residual checks read the
    companion, so with CABCD_FLAG_FOLD_UPDATE the steps before them apply
    their update on their own; the objective trace and the stopping
    iteration match the oracle's."""
    d, n, b, s, lam, seed = 512, 8192, 8, 32, 1e-4, 2004
    X, y, _ = synth.spectral_ridge(d, n, 1004)
    Xd, yd = X.to(DEV), y.to(DEV)
    H = 7 * s
    fold = gpu_lib.FLAG_FOLD_UPDATE
    trace = torch.zeros(3, dtype=torch.float64, device=DEV)
    w, r = gpu_lib.primal_bcd(Xd, yd, lam, b, s, H, seed, monitor_every=3, resid_every=5,
                              trace=trace, flags=fold)
    fs = []
    wo, zo = bcd.primal_bcd(X.numpy(), y.numpy(), lam, b, s, H, seed,
                            monitor=lambda h, w_, z_: fs.append(
                                bcd.primal_objective(X.numpy(), y.numpy(), lam, w_)))
    assert np.allclose(trace.cpu().numpy(), np.array(fs[2::3][:2] + [0.0]), rtol=1e-11, atol=0)
    assert _rel(w.cpu(), wo) <= 1e-10 and _rel(r.cpu(), zo - y.numpy()) <= 1e-10
    # a residual check every 2 outer steps: the run stops where the oracle's
    # residual first falls below the tolerance
    st = {}
    w3, _ = gpu_lib.primal_bcd(Xd, yd, lam, b, s, H, seed, tol=1e300, check_every=2, stats=st,
                               flags=fold)
    assert st["h"] == 2 * s
    w4, _ = gpu_lib.primal_bcd(Xd, yd, lam, b, s, 2 * s, seed, flags=fold)
    assert torch.equal(w3, w4)


def test_folded_update_with_explicit_blocks(gpu_lib):
    """CABCD_FLAG_FOLD_UPDATE with caller-given blocks (explicit_idx): the
    pending update reads the previous step's rows from the caller's array;
    blocks that repeat coordinates within and across steps.  Equal to the
    unfolded run to rounding and to the oracle."""
    d, n, b, s, lam = 600, 8192, 8, 32, 1e-3
    X, y, _ = synth.gaussian_ridge(d, n, 1005)
    Xd, yd = X.to(DEV), y.to(DEV)
    H = 3 * s
    rng = np.random.default_rng(17)
    blocks = np.stack([rng.choice(d, b, replace=False) for _ in range(H)])
    blocks[5] = blocks[4]                      # a block repeated inside a step
    blocks[s + 3] = blocks[3]                  # and one repeated across steps
    idx = torch.tensor(blocks, dtype=torch.int32, device=DEV)
    wf, rf = gpu_lib.primal_bcd(Xd, yd, lam, b, s, H, 0, explicit_idx=idx,
                                flags=gpu_lib.FLAG_FOLD_UPDATE)
    w0, r0 = gpu_lib.primal_bcd(Xd, yd, lam, b, s, H, 0, explicit_idx=idx)
    assert _rel(wf.cpu(), w0.cpu()) <= 1e-12 and _rel(rf.cpu(), r0.cpu()) <= 1e-12
    wo, zo = bcd.primal_bcd(X.numpy(), y.numpy(), lam, b, s, H, 0,
                            explicit_idx=blocks.tolist())
    assert _rel(wf.cpu(), wo) <= 1e-10 and _rel(rf.cpu(), zo - y.numpy()) <= 1e-10


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_mixed_primal_per_step_path(gpu_lib, dtype):
    """The mixed-precision step at sb = 256 (b = 16, s = 16) on rows of 65536
    codes (32 MiB of BF16, 16 MiB of FP8 gathered per step), with the exact
    residual recomputed every 4 outer steps as in the mixed workload."""
    d, n, b, s, lam, seed = 512, 65536, 16, 16, 1e-4, 3
    steps = 48
    H = steps * s
    _say("mixed per-step", dtype, d, n, b, s, H)
    X, y, _, _ = synth.colscaled_ridge(d, n, 9)
    code = gpu_lib.BF16 if dtype == "bf16" else gpu_lib.FP8_E4M3
    Q = gpu_lib.quantize(X.to(DEV), code)
    Xh = Q.dequantize().cpu().numpy()
    yn = y.numpy()
    wstar = bcd.ridge_closed_form(Xh, yn, lam)
    fstar = bcd.primal_objective(Xh, yn, lam, wstar)
    t = gpu_lib.new_timing()
    w, r = gpu_lib.primal_bcd(Q, y.to(DEV), lam, b, s, H, seed, resid_every=4, timing=t)
    _assert_per_step(gpu_lib, t, steps)
    wn = w.cpu().numpy()
    rel_obj = (bcd.primal_objective(Xh, yn, lam, wn) - fstar) / fstar
    _say(f"  rel obj error {rel_obj:.2e}")
    assert rel_obj <= 1e-6
    # the last outer step recomputed r = X^ T w - y exactly (48 steps, every 4th)
    ro = Xh.T @ wn - yn
    bound = np.abs(Xh).T @ np.abs(wn) + np.abs(yn)
    assert np.all(np.abs(r.cpu().numpy() - ro) <= 1e-12 * bound)
    # the FP64 path on X^ with the same blocks (pinned to the oracle by the
    # tests above): the distance is the FP32 Gram accumulation's, reported
    w64, _ = gpu_lib.primal_bcd(torch.tensor(Xh, device=DEV), y.to(DEV), lam, b, s, H, seed)
    _say(f"  ||w_mixed - w_fp64|| / ||w_fp64|| = {_rel(wn, w64.cpu()):.2e} (reported)")


# ------------------------------------------------------------------ b = 1

def _csr(M):
    S = scipy.sparse.csr_matrix(M)
    S.sort_indices()
    return S


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("s,H", [(1, 300), (8, 300), (32, 101)])
def test_primal_b1_matches_oracle(gpu_lib, kind, s, H):
    """b = 1 (single-coordinate BCD, the regime of the paper's largest CA
    speedups) on a matrix with a few exact zeros per row."""
    _say("primal b=1", kind, s, H)
    X, y, _ = synth.gaussian_ridge(64, 1024, 71)
    X[np.abs(X.numpy()) < 0.3] = 0.0
    lam = 1e-3
    A = gpu_lib.CSR.from_scipy(_csr(X.numpy()), DEV) if kind == "csr" else X.to(DEV)
    w, r = gpu_lib.primal_bcd(A, y.to(DEV), lam, 1, s, H, 5)
    wo, zo = bcd.primal_bcd(X.numpy(), y.numpy(), lam, 1, s, H, 5)
    assert _rel(w.cpu(), wo) <= 1e-10
    assert _rel(r.cpu(), zo - y.numpy()) <= 1e-10


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("s,H", [(1, 300), (8, 300), (32, 101)])
def test_dual_b1_matches_oracle(gpu_lib, kind, s, H):
    _say("dual b=1", kind, s, H)
    X, y, _ = synth.gaussian_ridge(300, 200, 72)
    X[np.abs(X.numpy()) < 0.3] = 0.0
    lam = 1e-2
    XT = X.t().contiguous()
    A = gpu_lib.CSR.from_scipy(_csr(XT.numpy()), DEV) if kind == "csr" else XT.to(DEV)
    a, w = gpu_lib.dual_bcd(A, y.to(DEV), lam, 1, s, H, 6)
    ao, wo = bcd.dual_bcd(X.numpy(), y.numpy(), lam, 1, s, H, 6)
    assert _rel(a.cpu(), ao) <= 1e-10
    assert _rel(w.cpu(), wo) <= 1e-10


# ------------------------------------------------------------------ solver edge cases

@pytest.mark.parametrize("kind,s,H", [
    ("dense", 1, 1),    # Grams computed ahead: diagonal blocks inverted ahead
    ("dense", 4, 1),    # ragged step: the solve inverts its own blocks
    ("dense", 4, 9),    # full steps ahead, then a ragged one
    ("csr", 1, 1),
    ("csr", 4, 1),
])
def test_not_positive_definite_block_is_reported(gpu_lib, kind, s, H):
    """Every feature row is the same +-1 vector, so any block of b = 2 holds two
    identical rows: Gamma = [[1, 1], [1, 1]] + lambda I with lambda = 1e-300,
    which rounds to the singular [[1, 1], [1, 1]] (all sums exact).  The
    oracle's Cholesky meets a zero pivot; the GPU must report
    CABCD_ENOTSPD (not the non-finite values that follow)."""
    _say("not SPD", kind, s, H)
    d, n, lam = 6, 64, 1e-300
    rng = np.random.default_rng(3)
    row = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    X = np.tile(row, (d, 1))
    y = rng.standard_normal(n)
    with pytest.raises(bcd.NotSPDError):
        bcd.primal_bcd(X, y, lam, 2, s, H, 1)
    A = (gpu_lib.CSR.from_scipy(_csr(X), DEV) if kind == "csr"
         else torch.tensor(X, device=DEV))
    with pytest.raises(gpu_lib.CabcdError) as e:
        gpu_lib.primal_bcd(A, torch.tensor(y, device=DEV), lam, 2, s, H, 1)
    assert e.value.status == gpu_lib.ENOTSPD


@pytest.mark.parametrize("b,s", [(4, 8), (8, 4), (16, 2)])
def test_ill_conditioned_blocks(gpu_lib, b, s):
    """Rows v + eps z_i (eps = 2e-3): every b x b diagonal block has
    kappa ~ 1e6.  A solve with such a block moves its result by at most about
    kappa u relative to the exact one, in either implementation, and block
    coordinate descent does not amplify such perturbations from step to step
    (each block step is an exact minimisation), so the iterates of H steps
    agree to within H * 10 * kappa_max * u."""
    d, n, lam, H, seed = 32, 1024, 1e-10, 64, 8
    _say("ill-conditioned", b, s)
    rng = np.random.default_rng(11)
    v = rng.standard_normal(n)
    X = v[None, :] + 2e-3 * rng.standard_normal((d, n))
    y = X.T @ rng.standard_normal(d) + 0.1 * rng.standard_normal(n)
    # kappa of the blocks this run factors (the oracle's Gram)
    from oracle import sampler
    blocks = sampler.sample_blocks(seed, 0, H, b, d)
    kap = max(np.linalg.cond(bcd.gram(X, blk, 1.0 / n, lam)[0]) for blk in blocks)
    _say(f"  max kappa(Gamma_j) = {kap:.2e}")
    assert 1e5 <= kap <= 1e8
    w, r = gpu_lib.primal_bcd(torch.tensor(X, device=DEV), torch.tensor(y, device=DEV), lam, b,
                              s, H, seed)
    wo, zo = bcd.primal_bcd(X, y, lam, b, s, H, seed)
    tol = H * 10.0 * kap * U64
    e_w, e_r = _rel(w.cpu(), wo), _rel(r.cpu(), zo - y)
    _say(f"  rel err w {e_w:.2e}, r {e_r:.2e}, bound {tol:.2e}")
    assert e_w <= tol and e_r <= tol


def test_fp8_nan_codes_read_as_nan(gpu_lib):
    """E4M3 has no infinities; 0x7F / 0xFF are NaN.  The FP64 streaming pass
    must read them as NaN (as the matrix instructions do), never as a finite
    value."""
    _say("fp8 nan codes")
    codes = torch.full((3, 40), 0x38, dtype=torch.uint8)   # 1.0
    codes[1, 7] = 0x7F
    codes[2, 9] = 0xFF
    Q = gpu_lib.Quantized(codes.to(DEV), torch.ones(3, dtype=torch.float32, device=DEV),
                          gpu_lib.FP8_E4M3)
    w = torch.tensor([1.0, 1.0, 0.5], dtype=torch.float64, device=DEV)
    y = torch.zeros(40, dtype=torch.float64, device=DEV)
    f, r = gpu_lib.primal_objective(Q, y, 1.0, w)
    rn = r.cpu().numpy()
    assert np.isnan(rn[7]) and np.isnan(rn[9])
    assert np.all(rn[[k for k in range(40) if k not in (7, 9)]] == 2.5)
    assert np.isnan(f.item())


# ------------------------------------------------------------------ s b in (256, 512]

@pytest.mark.parametrize("m,cols", [(257, 1000), (300, 4098), (384, 20000), (385, 777),
                                    (512, 32768), (512, 65), (511, 5001)])
def test_big_gram_matches_oracle(gpu_lib, m, cols):
    """Gram of 257..512 gathered rows (assembled from 256-row Grams), with
    repeated indices, against the oracle's definition."""
    _say("big gram", m, cols)
    rows = m + 40
    g = torch.Generator().manual_seed(m * 7 + cols)
    A = torch.randn(rows, cols, generator=g, dtype=torch.float64)
    u = torch.randn(cols, generator=g, dtype=torch.float64)
    idx = torch.randint(0, rows, (m,), generator=g, dtype=torch.int32)
    scale, shift = 1.0 / cols, 0.37
    G, Yu = gpu_lib.gram(A.to(DEV), idx.to(DEV), scale, shift, u.to(DEV))
    Go, Yo = bcd.gram(A.numpy(), idx.numpy(), scale, shift, u.numpy())
    Y = np.abs(A.numpy()[idx.numpy()])
    assert np.all(np.abs(G.cpu().numpy() - Go) <= 1e-12 * scale * (Y @ Y.T) + 1e-300)
    assert torch.equal(G, G.t())
    assert np.all(np.abs(Yu.cpu().numpy() - Yo) <= 1e-12 * (Y @ np.abs(u.numpy())) + 1e-300)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
@pytest.mark.parametrize("m,cols", [(300, 4096), (512, 20000), (400, 4099)])
def test_big_lowp_gram_matches_oracle(gpu_lib, dtype, m, cols):
    _say("big lowp gram", dtype, m, cols)
    rows = m + 9
    rng = np.random.default_rng(m + cols)
    X = rng.standard_normal((rows, cols)) * np.exp(rng.standard_normal(rows))[:, None]
    code = gpu_lib.BF16 if dtype == "bf16" else gpu_lib.FP8_E4M3
    Q = gpu_lib.quantize(torch.tensor(X, device=DEV), code)
    Xh = Q.dequantize().cpu().numpy()
    idx = rng.integers(0, rows, size=m).astype(np.int32)
    u = rng.standard_normal(cols)
    scale, shift = 1.0 / cols, 0.5
    G, Yu = gpu_lib.gram(Q, torch.tensor(idx, device=DEV), scale, shift,
                         torch.tensor(u, device=DEV))
    Go, Yo = bcd.gram(Xh, idx, scale, shift, u)
    Y = np.abs(Xh[idx])
    # FP32 accumulation bound of the mixed-precision Gram (as for 256 rows)
    rel_bound = cols * 2.0 ** -24 + (0.0 if dtype == "bf16" else 2.0 ** -12)
    assert np.all(np.abs(G.cpu().numpy() - Go) <= rel_bound * scale * (Y @ Y.T) + 1e-300)
    assert np.all(np.abs(Yu.cpu().numpy() - Yo) <= 1e-12 * (Y @ np.abs(u)) + 1e-300)


@pytest.mark.parametrize("d,n,b,s,H", [
    (1024, 8192, 16, 32, 2 * 32 + 7),   # s b = 512: b = 16, s = 32
    (700, 3001, 8, 64, 150),            # s b = 512 with b = 8 (odd n: unaligned rows)
    (600, 4000, 12, 40, 90),            # s b = 480, b not a power of two
    (300, 2048, 16, 20, 50),            # s b = 320: half of the cross blocks
])
def test_primal_big_sb_matches_oracle(gpu_lib, d, n, b, s, H):
    _say("primal big sb", d, n, b, s, H)
    X, y, _ = synth.gaussian_ridge(d, n, 500 + d)
    t = gpu_lib.new_timing()
    w, r = gpu_lib.primal_bcd(X.to(DEV), y.to(DEV), 1e-3, b, s, H, 21, timing=t)
    steps = -(-H // s)
    _assert_per_step(gpu_lib, t, steps)
    wo, zo = bcd.primal_bcd(X.numpy(), y.numpy(), 1e-3, b, s, H, 21)
    assert _rel(w.cpu(), wo) <= 1e-10
    assert _rel(r.cpu(), zo - y.numpy()) <= 1e-10


def test_dual_big_sb_matches_oracle(gpu_lib):
    d, n, b, s, H = 3000, 2048, 16, 32, 70
    _say("dual big sb", d, n, b, s, H)
    X, y, _ = synth.gaussian_ridge(d, n, 808)
    a, w = gpu_lib.dual_bcd(X.t().contiguous().to(DEV), y.to(DEV), 1e-2, b, s, H, 22)
    ao, wo = bcd.dual_bcd(X.numpy(), y.numpy(), 1e-2, b, s, H, 22)
    assert _rel(a.cpu(), ao) <= 1e-10
    assert _rel(w.cpu(), wo) <= 1e-10


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_mixed_primal_big_sb_reaches_1e6(gpu_lib, dtype):
    d, n, b, s, lam = 512, 16384, 16, 32, 1e-4
    H = 40 * s
    _say("mixed big sb", dtype, d, n, b, s, H)
    X, y, _, _ = synth.colscaled_ridge(d, n, 19)
    code = gpu_lib.BF16 if dtype == "bf16" else gpu_lib.FP8_E4M3
    Q = gpu_lib.quantize(X.to(DEV), code)
    Xh = Q.dequantize().cpu().numpy()
    yn = y.numpy()
    fstar = bcd.primal_objective(Xh, yn, lam, bcd.ridge_closed_form(Xh, yn, lam))
    w, r = gpu_lib.primal_bcd(Q, y.to(DEV), lam, b, s, H, 4, resid_every=4)
    wn = w.cpu().numpy()
    rel_obj = (bcd.primal_objective(Xh, yn, lam, wn) - fstar) / fstar
    _say(f"  rel obj error {rel_obj:.2e}")
    assert rel_obj <= 1e-6


@pytest.mark.parametrize("b,s,n", [(8, 1, 300000), (1, 8, 300000), (4, 4, 300000),
                                   (8, 4, 20000)])
def test_graph_captured_call_equals_direct_call(gpu_lib, b, s, n):
    """A one-problem call captured into a HIP graph (caller workspace, no
    synchronisation inside the call) and replayed gives bitwise the iterates of
    the same call issued directly, on every replay from the same state.  n =
    300000: one Gram per step (gathered rows above 8 MiB); n = 20000: Grams of
    future steps computed ahead."""
    _say("graph capture", b, s, n)
    d = 64
    X, y, _ = synth.gaussian_ridge(d, n, 90, device=DEV)
    lam, H, seed = 1e-3, 6 * s, 12
    ws = torch.empty(gpu_lib.workspace_bytes(X, b, s), dtype=torch.uint8, device=DEV)
    w = torch.zeros(d, dtype=torch.float64, device=DEV)
    r = torch.empty(n, dtype=torch.float64, device=DEV)
    gpu_lib.primal_bcd(X, y, lam, b, s, H, seed, w=w, r=r, workspace=ws)
    w0, r0 = w.clone(), r.clone()
    flags = gpu_lib.FLAG_STATE_VALID | gpu_lib.FLAG_ASYNC
    gpu_lib.primal_bcd(X, y, lam, b, s, H, seed, w=w, r=r, h0=H, flags=flags, workspace=ws)
    torch.cuda.synchronize()
    w1, r1 = w.clone(), r.clone()
    wo, ro = bcd.primal_bcd(X.cpu().numpy(), y.cpu().numpy(), lam, b, s, 2 * H, seed)
    assert _rel(w1.cpu().numpy(), wo) <= 1e-10
    w.copy_(w0)
    r.copy_(r0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu_lib.primal_bcd(X, y, lam, b, s, H, seed, w=w, r=r, h0=H, flags=flags, workspace=ws)
    for rep in range(3):
        w.copy_(w0)
        r.copy_(r0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(w, w1) and torch.equal(r, r1), f"replay {rep}"
