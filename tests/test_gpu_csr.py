"""CSR path vs the CPU oracle through the C-ABI.

Tolerances as for the dense FP64 path: Gram entries within 1e-12 of
scale * |Y||Y|^T, iterates within 1e-10 relative.  Outer steps whose Grams come
from the split launch (s b >= 256) update the companion vector with one writer
per column; the other steps scatter with FP64 atomic adds, which makes their
result reproducible only up to the order of those additions, so every
comparison with the oracle has a tolerance.
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


def _random_csr(rows, cols, density, seed, long_rows=(), empty_rows=()):
    rng = np.random.default_rng(seed)
    S = scipy.sparse.random(rows, cols, density=density, format="lil", random_state=rng,
                            data_rvs=rng.standard_normal)
    for r in long_rows:
        c = rng.choice(cols, size=min(cols, 5000), replace=False)
        S[r, c] = rng.standard_normal(len(c))
    for r in empty_rows:
        S[r, :] = 0
    S = S.tocsr()
    S.eliminate_zeros()
    S.sort_indices()
    return S


@pytest.mark.parametrize("m,seed", [(1, 0), (16, 1), (100, 2), (257, 3), (512, 4), (1024, 5)])
def test_csr_gram_matches_oracle(gpu_lib, m, seed):
    _say("csr gram", m, seed)
    rows, cols = 1500, 9000
    S = _random_csr(rows, cols, 0.01, seed, long_rows=(7, 11), empty_rows=(3,))
    rng = np.random.default_rng(seed + 100)
    idx = rng.integers(0, rows, size=m).astype(np.int32)
    idx[: min(m, 3)] = [7, 3, 11][: min(m, 3)]      # long rows and an empty row
    u = rng.standard_normal(cols)
    A = gpu_lib.CSR.from_scipy(S, DEV)
    G, Yu = gpu_lib.gram(A, torch.tensor(idx, device=DEV), 0.5, 0.25,
                         torch.tensor(u, device=DEV))
    Go, Yo = bcd.gram(S, idx, 0.5, 0.25, u)
    Y = np.abs(np.asarray(S[idx].todense()))
    assert np.all(np.abs(G.cpu().numpy() - Go) <= 1e-12 * 0.5 * (Y @ Y.T) + 1e-300)
    assert np.all(np.abs(Yu.cpu().numpy() - Yo) <= 1e-12 * (Y @ np.abs(u)) + 1e-300)


@pytest.fixture(scope="module")
def zipf_small():
    rowptr, colidx, vals, y, _ = synth.zipf_csr_ridge(2000, 1 << 14, 31, 1002)
    A = scipy.sparse.csr_matrix((vals, colidx, rowptr), shape=(2000, 1 << 14))
    return A, y


def test_csr_long_rows_tile_chunks(gpu_lib):
    """Rows of 600 entries: the three rows of a Gram tile exceed one hash-table
    fill, so their entries are taken in chunks whose sums are added."""
    _say("csr long rows")
    rowptr, colidx, vals, y, _ = synth.zipf_csr_ridge(300, 1 << 14, 600, 1009)
    A = scipy.sparse.csr_matrix((vals, colidx, rowptr), shape=(300, 1 << 14))
    XT = gpu_lib.CSR.from_scipy(A, DEV)
    lam, b, s, H, seed = 1e-3, 16, 4, 48, 5
    a, w = gpu_lib.dual_bcd(XT, torch.tensor(y, device=DEV), lam, b, s, H, seed)
    ao, wo = bcd.dual_bcd(A.T.tocsc(), y, lam, b, s, H, seed)
    assert _rel(a.cpu(), ao) <= 1e-10
    assert _rel(w.cpu(), wo) <= 1e-10


def test_csr_split_gram_power_law_columns(gpu_lib):
    """The split path on power-law column popularity (the text-classification
    structure): a few hundred columns in most rows go to the dense panel, the
    long tail to the column lists; 256 and 512 gathered rows an outer step."""
    rows, cols = 3000, 20000
    rowptr, colidx, vals, y, _ = synth.zipf_csr_ridge(rows, cols, 60, 77)
    S = scipy.sparse.csr_matrix((vals, colidx, rowptr), shape=(rows, cols))
    XT = gpu_lib.CSR.from_scipy(S, DEV)
    for s in (16, 32):
        _say("csr split gram power law", s)
        H = 6 * s + 5
        a, w = gpu_lib.dual_bcd(XT, torch.tensor(y, device=DEV), 1e-3, 16, s, H, 21)
        ao, wo = bcd.dual_bcd(S.T.tocsc(), y, 1e-3, 16, s, H, 21)
        assert _rel(a.cpu(), ao) <= 1e-10
        assert _rel(w.cpu(), wo) <= 1e-10


@pytest.mark.parametrize("s", [1, 8, 32])
def test_csr_dual_matches_oracle(gpu_lib, zipf_small, s):
    _say("csr dual", s)
    A, y = zipf_small
    lam, b, H, seed = 1e-3, 16, 96, 2002
    XT = gpu_lib.CSR.from_scipy(A, DEV)
    a, w = gpu_lib.dual_bcd(XT, torch.tensor(y, device=DEV), lam, b, s, H, seed)
    ao, wo = bcd.dual_bcd(A.T.tocsc(), y, lam, b, s, H, seed)
    assert _rel(a.cpu(), ao) <= 1e-10
    assert _rel(w.cpu(), wo) <= 1e-10


def test_csr_dual_link_and_objective(gpu_lib, zipf_small):
    _say("csr dual link")
    A, y = zipf_small
    lam = 1e-3
    XT = gpu_lib.CSR.from_scipy(A, DEV)
    yd = torch.tensor(y, device=DEV)
    trace = torch.zeros(4, dtype=torch.float64, device=DEV)
    a, w = gpu_lib.dual_bcd(XT, yd, lam, 16, 8, 256, 7, monitor_every=8, trace=trace)
    wl = gpu_lib.dual_to_primal(XT, a, lam)
    assert _rel(w.cpu(), wl.cpu()) <= 1e-10
    X = A.T.tocsr()
    f, _ = gpu_lib.primal_objective_t(XT, yd, lam, w)
    fo = bcd.primal_objective(X, y, lam, w.cpu().numpy())
    assert abs(f.item() - fo) <= 1e-12 * fo
    assert abs(trace[3].item() - fo) <= 1e-12 * fo


def test_csr_primal_matches_oracle(gpu_lib):
    _say("csr primal")
    S = _random_csr(300, 4000, 0.02, 9, long_rows=(5,), empty_rows=(17,))
    rng = np.random.default_rng(3)
    y = rng.standard_normal(4000)
    X = gpu_lib.CSR.from_scipy(S, DEV)
    w, r = gpu_lib.primal_bcd(X, torch.tensor(y, device=DEV), 1e-2, 8, 6, 70, 5)
    wo, zo = bcd.primal_bcd(S, y, 1e-2, 8, 6, 70, 5)
    assert _rel(w.cpu(), wo) <= 1e-10
    assert _rel(r.cpu(), zo - y) <= 1e-10
    f, _ = gpu_lib.primal_objective(X, torch.tensor(y, device=DEV), 1e-2, w)
    assert abs(f.item() - bcd.primal_objective(S, y, 1e-2, w.cpu().numpy())) <= 1e-12 * f.item()


def test_csr_repeated_indices_row_per_thread(gpu_lib):
    # s b = 450 rows over 50 samples (dual) or 40 features (primal): every
    # index repeats about ten times, and s * 4 lanes exceed one 512-thread
    # workgroup, so the solve takes one row per thread
    _say("csr repeated indices")
    rng = np.random.default_rng(12)
    S = _random_csr(50, 2000, 0.05, 12, long_rows=(3,), empty_rows=(7,))
    y = rng.standard_normal(50)
    XT = gpu_lib.CSR.from_scipy(S, DEV)
    a, w = gpu_lib.dual_bcd(XT, torch.tensor(y, device=DEV), 1e-2, 3, 150, 300, 11)
    ao, wo = bcd.dual_bcd(S.T.tocsc(), y, 1e-2, 3, 150, 300, 11)
    assert _rel(a.cpu(), ao) <= 1e-10
    assert _rel(w.cpu(), wo) <= 1e-10
    P = _random_csr(40, 3000, 0.05, 13)
    yp = rng.standard_normal(3000)
    X = gpu_lib.CSR.from_scipy(P, DEV)
    wp, rp = gpu_lib.primal_bcd(X, torch.tensor(yp, device=DEV), 1e-2, 3, 150, 300, 12)
    wpo, zpo = bcd.primal_bcd(P, yp, 1e-2, 3, 150, 300, 12)
    assert _rel(wp.cpu(), wpo) <= 1e-10
    assert _rel(rp.cpu(), zpo - yp) <= 1e-10


def test_csr_malformed_is_rejected(gpu_lib):
    _say("csr malformed")
    S = _random_csr(50, 200, 0.05, 1)
    good = gpu_lib.CSR.from_scipy(S, DEV)
    y = torch.zeros(50, dtype=torch.float64, device=DEV)
    bad_cols = good.colidx.clone()
    bad_cols[0] = 200                      # column out of range
    bad = gpu_lib.CSR(good.rowptr, bad_cols, good.vals, (50, 200))
    with pytest.raises(gpu_lib.CabcdError) as e:
        gpu_lib.dual_bcd(bad, y, 0.1, 2, 2, 4, 0)
    assert e.value.status == gpu_lib.EINVAL
    unsorted = good.colidx.clone()
    r0, r1 = int(good.rowptr[4]), int(good.rowptr[5])
    if r1 - r0 >= 2:
        unsorted[r0], unsorted[r0 + 1] = good.colidx[r0 + 1], good.colidx[r0]
        with pytest.raises(gpu_lib.CabcdError):
            gpu_lib.dual_bcd(gpu_lib.CSR(good.rowptr, unsorted, good.vals, (50, 200)), y,
                             0.1, 2, 2, 4, 0)
    # the good matrix still works afterwards
    gpu_lib.dual_bcd(good, y, 0.1, 2, 2, 4, 0)


def test_csr_steps_cross_index_chunks(gpu_lib):
    """More outer steps than one index chunk (4096): the Grams computed ahead
    stop at the chunk boundary, and a ragged last step falls back to the
    one-step Gram."""
    _say("csr many steps")
    S = _random_csr(60, 300, 0.05, 21, long_rows=(3,), empty_rows=(9,))
    rng = np.random.default_rng(4)
    y = rng.standard_normal(60)
    XT = gpu_lib.CSR.from_scipy(S, DEV)
    H = 2 * 4096 + 2 * 50 + 1         # s = 2: 4146 full outer steps, then a ragged one
    a, w = gpu_lib.dual_bcd(XT, torch.tensor(y, device=DEV), 1e-2, 2, 2, H, 13)
    ao, wo = bcd.dual_bcd(S.T.tocsc(), y, 1e-2, 2, 2, H, 13)
    assert _rel(a.cpu(), ao) <= 1e-10
    assert _rel(w.cpu(), wo) <= 1e-10


def test_csr_split_steps_are_reproducible(gpu_lib):
    """Outer steps whose Grams come from the split launch update the companion
    vector with one writer per column and fixed summation orders: two runs
    give bitwise the same alpha and w (and the oracle's to 1e-10), and so does
    the same run split into two calls (3 + 2 outer steps, resumed with h0 and
    the state passed on), whose Grams are computed in other batches."""
    rows, cols = 3000, 20000
    rowptr, colidx, vals, y, _ = synth.zipf_csr_ridge(rows, cols, 60, 78)
    S = scipy.sparse.csr_matrix((vals, colidx, rowptr), shape=(rows, cols))
    XT = gpu_lib.CSR.from_scipy(S, DEV)
    s, b = 32, 16
    H = 5 * s                  # five full outer steps of 512 gathered rows
    yd = torch.tensor(y, device=DEV)
    runs = [gpu_lib.dual_bcd(XT, yd, 1e-3, b, s, H, 23) for _ in range(2)]
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])
    a2, w2 = gpu_lib.dual_bcd(XT, yd, 1e-3, b, s, 3 * s, 23)
    gpu_lib.dual_bcd(XT, yd, 1e-3, b, s, 2 * s, 23, alpha=a2, w=w2, h0=3 * s,
                     flags=gpu_lib.FLAG_STATE_VALID)
    assert torch.equal(a2, runs[0][0]) and torch.equal(w2, runs[0][1])
    ao, wo = bcd.dual_bcd(S.T.tocsc(), y, 1e-3, b, s, H, 23)
    assert _rel(runs[0][0].cpu(), ao) <= 1e-10
    assert _rel(runs[0][1].cpu(), wo) <= 1e-10


@pytest.mark.parametrize("density,s", [(0.01, 32), (0.2, 32), (0.05, 40), (0.05, 64)])
def test_csr_split_gram_without_and_with_heavy_columns(gpu_lib, density, s):
    """Grams computed ahead by the split path: a uniform sparse matrix whose
    columns all stay below the heavy threshold (light lists only), and a denser
    one where the 512 most frequent columns go to the dense panel."""
    _say("csr split gram", density, s)
    S = _random_csr(2000, 4000, density, 31, long_rows=(5,), empty_rows=(9,))
    rng = np.random.default_rng(5)
    y = rng.standard_normal(2000)
    XT = gpu_lib.CSR.from_scipy(S, DEV)
    lam, b, H, seed = 1e-2, 8, 10 * s + 3, 14
    a, w = gpu_lib.dual_bcd(XT, torch.tensor(y, device=DEV), lam, b, s, H, seed)
    ao, wo = bcd.dual_bcd(S.T.tocsc(), y, lam, b, s, H, seed)
    assert _rel(a.cpu(), ao) <= 1e-10
    assert _rel(w.cpu(), wo) <= 1e-10


@pytest.fixture(scope="module")
def zipf_bench():
    rowptr, colidx, vals, y, _ = synth.zipf_csr_ridge(20000, 1 << 20, 315, 1002)
    return scipy.sparse.csr_matrix((vals, colidx, rowptr), shape=(20000, 1 << 20)), y


@pytest.mark.parametrize("s,H", [(1, 64), (8, 8 * 20 + 3), (32, 17 * 32 + 5)])
def test_csr_dual_bench_size(gpu_lib, zipf_bench, s, H):
    """The sparse dual workload at its full size and in the benchmark's launch
    configuration: A = X^T in CSR, 20000 rows x 2^20 columns, 315 Zipf(1.1)
    features per row (the benchmark's generator and seed), lambda = 1e-5,
    b = 16, s = 1, 8, 32.  At s = 32 the Grams come from the split launches of
    16 outer steps each: 17 full steps cross a launch boundary, then a ragged
    step.  alpha and w against the oracle's run of the same steps."""
    _say("csr dual bench size", s, H)
    S, y = zipf_bench
    XT = gpu_lib.CSR.from_scipy(S, DEV)
    lam, b, seed = 1e-5, 16, 2002
    t = gpu_lib.new_timing()
    a, w = gpu_lib.dual_bcd(XT, torch.tensor(y, device=DEV), lam, b, s, H, seed, timing=t)
    n = {k: v["launches"] for k, v in gpu_lib.timing_dict(t).items()}
    _say("  launches", n)
    steps = -(-H // s)
    assert n["solve"] >= steps and n["gram"] < steps   # Grams computed ahead
    ao, wo = bcd.dual_bcd(S.T.tocsc(), y, lam, b, s, H, seed)
    e_a, e_w = _rel(a.cpu(), ao), _rel(w.cpu(), wo)
    _say(f"  rel err alpha {e_a:.2e}, w {e_w:.2e}")
    assert e_a <= 1e-10 and e_w <= 1e-10
