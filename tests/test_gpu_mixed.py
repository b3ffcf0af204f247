"""Mixed-precision path (BF16 / FP8-E4M3 storage) vs the CPU oracle.

* Quantisation: bit-exact against the oracle's encoders (codes and FP32 scales).
* Gram of stored codes: FP32 accumulation on the matrix cores, so the bound is
  Higham's worst case for a K-term FP32 dot product, K * 2^-24 * |Y^||Y^|^T,
  against the FP64 Gram of the dequantised rows X^; Y u is FP64 (1e-12).
* End to end: the problem solved is (X^, y, lambda); the run must reach a
  relative objective error of 1e-6 against the closed-form optimum on X^, and
  an exact residual recomputation must reproduce X^T w - y to 1e-12.  The
  iterates are not expected to equal the FP64 oracle's (the Gram differs at
  the FP32 level); their distance is reported, not pinned.
"""

import numpy as np
import pytest
import torch

from oracle import bcd, quant
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _layouts(gpu_lib, Q):
    """The binding's storage (rows padded to 16-byte boundaries) and, when the
    padding is not empty, a contiguous copy whose rows start at any byte (the
    kernels' unaligned paths)."""
    out = [("padded", Q)]
    if Q.codes.stride(0) != Q.codes.shape[1]:
        out.append(("contiguous", gpu_lib.Quantized(Q.codes.contiguous(), Q.scales, Q.dtype)))
    return out


def _matrix(rows, cols, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((rows, cols)) * np.exp(2.0 * rng.standard_normal(rows))[:, None]
    X[1] = 0.0                                   # an all-zero row
    X[2, :5] = [448.0, -1e6, 3e-12, 0.0, 1.0 + 2.0 ** -8 + 2.0 ** -40]
    return X


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_quantize_bit_exact(gpu_lib, dtype):
    _say("quantize", dtype)
    X = _matrix(37, 1001, 1)
    code = gpu_lib.BF16 if dtype == "bf16" else gpu_lib.FP8_E4M3
    Q = gpu_lib.quantize(torch.tensor(X, device=DEV), code)
    want, s, _ = quant.quantize_rows(X, dtype)
    got = Q.codes.cpu().numpy()
    if dtype == "bf16":
        assert np.array_equal(got.view(np.uint16), want)
        assert Q.scales is None
    else:
        assert np.array_equal(got, want)
        assert np.array_equal(Q.scales.cpu().numpy().view(np.uint32), s.view(np.uint32))


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
@pytest.mark.parametrize("m,cols", [(5, 77), (16, 4096), (100, 10001), (256, 20000),
                                    # sb in (128, 256]: the LDS-DMA kernel on aligned rows
                                    # (several tiles per slab, a partial last tile), and the
                                    # register-fed kernel on unaligned rows
                                    (129, 1024), (200, 4112), (256, 70000), (200, 4099)])
def test_lowp_gram_against_fp64_gram_of_dequantised(gpu_lib, dtype, m, cols):
    _say("lowp gram", dtype, m, cols)
    rows = m + 7
    X = _matrix(rows, cols, m + cols)
    code = gpu_lib.BF16 if dtype == "bf16" else gpu_lib.FP8_E4M3
    Q = gpu_lib.quantize(torch.tensor(X, device=DEV), code)
    Xh = Q.dequantize().cpu().numpy()
    _, _, Xo = quant.quantize_rows(X, dtype)
    assert np.array_equal(Xh, Xo)                    # the torch decode agrees with the oracle
    rng = np.random.default_rng(m)
    idx = rng.integers(0, rows, size=m).astype(np.int32)
    u = rng.standard_normal(cols)
    scale, shift = 1.0 / cols, 0.5
    Go, Yo = bcd.gram(Xh, idx, scale, shift, u)
    Y = np.abs(Xh[idx])
    # BF16: Higham's bound for a K-term FP32 dot product.  FP8: the E4M3 matrix
    # instruction sums its 32 products with a coarser internal accumulation
    # than sequential IEEE FP32 (measured about 1e-5 relative at K = 77), so
    # its bound carries an extra 2^-12 relative term.
    rel_bound = cols * 2.0 ** -24 + (0.0 if dtype == "bf16" else 2.0 ** -12)
    bound = rel_bound * scale * (Y @ Y.T) + 1e-300
    for name, Qv in _layouts(gpu_lib, Q):
        G, Yu = gpu_lib.gram(Qv, torch.tensor(idx, device=DEV), scale, shift,
                             torch.tensor(u, device=DEV))
        err = np.abs(G.cpu().numpy() - Go)
        assert np.all(err <= bound), name
        rel = (err / np.maximum(scale * (Y @ Y.T), 1e-300)).max()
        _say(f"  {name}: max |dG| / (scale |Y||Y|^T) = {rel:.2e}")
        assert np.all(np.abs(Yu.cpu().numpy() - Yo) <= 1e-12 * (Y @ np.abs(u)) + 1e-300), name


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_lowp_gram_bench_size(gpu_lib, dtype):
    """The time-to-1e-6 workload at its full size: d = 4096, n = 2^20,
    column-scaled, generated as the benchmark generates it and stored by the
    binding's quantiser; one Gram of 256 distinct gathered rows (the kernel and
    launch of the benchmark's outer step, sb = 256) with a random u.  The
    expected values come from the oracle alone: its encoder applied to the
    gathered FP64 rows (row-local, so equal to the rows of the whole stored
    matrix) and its Gram of the dequantised rows; every entry within the
    bound of the small-size test."""
    d, n, m = 4096, 1 << 20, 256
    _say("lowp gram bench size", dtype, d, n, m)
    X, _, _, _ = synth.colscaled_ridge(d, n, 1003, device=DEV)
    code = gpu_lib.BF16 if dtype == "bf16" else gpu_lib.FP8_E4M3
    Q = gpu_lib.quantize(X, code)
    rng = np.random.default_rng(4096)
    idx = rng.permutation(d)[:m].astype(np.int32)
    rows = X[torch.tensor(idx, device=DEV, dtype=torch.int64)].cpu().numpy()
    del X
    torch.cuda.empty_cache()
    u = rng.standard_normal(n)
    scale, shift = 1.0 / n, 1e-4
    G, Yu = gpu_lib.gram(Q, torch.tensor(idx, device=DEV), scale, shift,
                         torch.tensor(u, device=DEV))
    G, Yu = G.cpu().numpy(), Yu.cpu().numpy()
    del Q
    torch.cuda.empty_cache()
    _, _, Yh = quant.quantize_rows(rows, dtype)
    del rows
    Go, Yo = bcd.gram(Yh, np.arange(m), scale, shift, u)
    Ya = np.abs(Yh)
    rel_bound = n * 2.0 ** -24 + (0.0 if dtype == "bf16" else 2.0 ** -12)
    mag = scale * (Ya @ Ya.T)
    err = np.abs(G - Go)
    _say(f"  max |dG| / (scale |Y||Y|^T) = {(err / np.maximum(mag, 1e-300)).max():.2e}")
    assert np.all(err <= rel_bound * mag + 1e-300)
    assert np.all(np.abs(Yu - Yo) <= 1e-12 * (Ya @ np.abs(u)) + 1e-300)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
@pytest.mark.parametrize("d,n", [(37, 70001), (3, 4097), (130, 2 * 4096 + 19)])
def test_lowp_companion_pass_entrywise(gpu_lib, dtype, d, n):
    # r = X^T w - y over all rows of the stored codes (the exact recomputation
    # pass): odd row counts split into unequal row ranges, fewer rows than are
    # kept in flight, and a last column chunk that is partly past the end
    _say("lowp companion pass", dtype, d, n)
    X = _matrix(d, n, 40 + d) if d > 2 else np.random.default_rng(d).standard_normal((d, n))
    rng = np.random.default_rng(n)
    y = rng.standard_normal(n)
    w = rng.standard_normal(d)
    code = gpu_lib.BF16 if dtype == "bf16" else gpu_lib.FP8_E4M3
    Q = gpu_lib.quantize(torch.tensor(X, device=DEV), code)
    Xh = Q.dequantize().cpu().numpy()
    ro = Xh.T @ w - y
    bound = np.abs(Xh).T @ np.abs(w) + np.abs(y)
    for name, Qv in _layouts(gpu_lib, Q):
        _, r = gpu_lib.primal_bcd(Qv, torch.tensor(y, device=DEV), 1e-3, 1, 1, 0, 1,
                                  w=torch.tensor(w, device=DEV))
        assert np.all(np.abs(r.cpu().numpy() - ro) <= 1e-12 * bound), name


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_mixed_primal_reaches_1e6_on_dequantised_problem(gpu_lib, dtype):
    _say("mixed primal", dtype)
    X, y, _, _ = synth.colscaled_ridge(128, 8192, 7)
    lam, b, s, H, seed = 1e-4, 16, 8, 8 * 24, 3
    code = gpu_lib.BF16 if dtype == "bf16" else gpu_lib.FP8_E4M3
    Q = gpu_lib.quantize(X.to(DEV), code)
    Xh = Q.dequantize().cpu().numpy()
    yn = y.numpy()
    wstar = bcd.ridge_closed_form(Xh, yn, lam)
    fstar = bcd.primal_objective(Xh, yn, lam, wstar)
    trace = torch.zeros(6, dtype=torch.float64, device=DEV)
    w, r = gpu_lib.primal_bcd(Q, y.to(DEV), lam, b, s, H, seed, resid_every=4,
                              monitor_every=4, trace=trace)
    wn = w.cpu().numpy()
    rel_obj = (bcd.primal_objective(Xh, yn, lam, wn) - fstar) / fstar
    _say(f"  rel obj error {rel_obj:.2e}; trace {trace.cpu().numpy()}")
    assert rel_obj <= 1e-6
    t = (trace.cpu().numpy() - fstar) / fstar
    assert abs(t[-1] - rel_obj) <= 1e-9
    # the last outer step was an exact recomputation (24 outer steps, every 4th)
    assert np.linalg.norm(r.cpu().numpy() - (Xh.T @ wn - yn)) <= 1e-12 * np.linalg.norm(yn)
    wo, _ = bcd.primal_bcd(Xh, yn, lam, b, s, H, seed)
    _say(f"  ||w_mixed - w_fp64 oracle|| / ||w_fp64|| = "
         f"{np.linalg.norm(wn - wo) / np.linalg.norm(wo):.2e} (reported, not pinned)")


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
@pytest.mark.parametrize("d", [512, 500])   # 500: rows of the stored X^T not 16-byte aligned
def test_mixed_dual_reaches_1e6_on_dequantised_problem(gpu_lib, dtype, d):
    """Dual CA-BDCD on BF16 / FP8 storage of X^T: the instance is (X^, y, lambda)
    with X^ the dequantised stored matrix.  D(alpha) reaches 1e-6 relative error
    against D(alpha*) on X^, the maintained w keeps the primal-dual link with
    X^, and the dual-layout helpers (primal objective, dual-to-primal map, dual
    residual) read the codes like the oracle reads X^."""
    _say("mixed dual", dtype, d)
    n, lam, b, s, H, seed = 200, 1e-2, 16, 8, 800, 5
    X, y, _ = synth.gaussian_ridge(d, n, 17)
    code = gpu_lib.BF16 if dtype == "bf16" else gpu_lib.FP8_E4M3
    Q = gpu_lib.quantize(X.t().contiguous().to(DEV), code)
    if d % 16:   # rows of the stored X^T starting at any byte
        Q = gpu_lib.Quantized(Q.codes.contiguous(), Q.scales, Q.dtype)
    Xh = Q.dequantize().cpu().numpy().T            # d x n
    yn = y.numpy()
    ws = bcd.ridge_closed_form(Xh, yn, lam)
    astar = Xh.T @ ws - yn
    Dstar = bcd.dual_objective(Xh, yn, lam, astar)
    a, w = gpu_lib.dual_bcd(Q, y.to(DEV), lam, b, s, H, seed)
    an, wn = a.cpu().numpy(), w.cpu().numpy()
    rel = (bcd.dual_objective(Xh, yn, lam, an) - Dstar) / abs(Dstar)
    _say(f"  rel dual objective error {rel:.2e}")
    assert rel <= 1e-6
    wl = -(Xh @ an) / (lam * n)
    assert np.linalg.norm(wn - wl) <= 1e-10 * np.linalg.norm(wl)
    w2 = gpu_lib.dual_to_primal(Q, a, lam)
    assert np.linalg.norm(w2.cpu().numpy() - wl) <= 1e-12 * np.linalg.norm(wl)
    f, _ = gpu_lib.primal_objective_t(Q, y.to(DEV), lam, w)
    fo = bcd.primal_objective(Xh, yn, lam, wn)
    assert abs(f.item() - fo) <= 1e-12 * fo
    nrm, rho = gpu_lib.dual_residual(Q, y.to(DEV), a, w)
    ro = bcd.dual_residual(Xh, yn, an, wn)
    bound = np.abs(Xh.T) @ np.abs(wn) + np.abs(an) + np.abs(yn)
    assert np.all(np.abs(rho.cpu().numpy() - ro) <= 1e-12 * bound)
    ao, _ = bcd.dual_bcd(Xh, yn, lam, b, s, H, seed)
    _say(f"  ||a_mixed - a_fp64 oracle|| / ||a_fp64|| = "
         f"{np.linalg.norm(an - ao) / np.linalg.norm(ao):.2e} (reported, not pinned)")


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_every_code_decodes_exactly(gpu_lib, dtype):
    """Every finite storage code, through the Gram's FP64 Y u and through the
    FP64 streaming pass of the exact residual, against the oracle's decoder."""
    _say("decode all codes", dtype)
    if dtype == "fp8":
        codes = np.array([c for c in range(256) if c & 0x7F != 0x7F], dtype=np.uint8)
        want = quant.e4m3_decode(codes)
        ct = torch.tensor(codes, dtype=torch.uint8)
        code, scales = gpu_lib.FP8_E4M3, torch.ones(len(codes), dtype=torch.float32, device=DEV)
    else:
        bits = np.arange(65536, dtype=np.uint32)
        finite = ((bits >> 7) & 0xFF) != 0xFF
        codes = bits[finite].astype(np.uint16)
        want = quant.bf16_decode(codes)
        ct = torch.tensor(codes.view(np.int16), dtype=torch.int16)
        code, scales = gpu_lib.BF16, None
    m, cols = len(codes), 40
    Qc = torch.zeros((m, cols), dtype=ct.dtype)
    Qc[:, 0] = ct
    Q = gpu_lib.Quantized(Qc.to(DEV), scales, code)
    u = torch.zeros(cols, dtype=torch.float64, device=DEV)
    u[0] = 1.0
    for r0 in range(0, m, 256):
        r1 = min(m, r0 + 256)
        idx = torch.arange(r0, r1, dtype=torch.int32, device=DEV)
        _, Yu = gpu_lib.gram(Q, idx, 1.0, 0.0, u)
        assert np.array_equal(Yu.cpu().numpy(), want[r0:r1])
    # streaming pass: r = X^T w - y with w picking one code per column sum
    rng = np.random.default_rng(5)
    w = rng.integers(-4, 5, size=m).astype(np.float64)
    w[(np.abs(want) > 1e20) | ((np.abs(want) < 1e-20) & (want != 0))] = 0.0   # keep the sum finite
    y = torch.zeros(cols, dtype=torch.float64, device=DEV)
    _, r = gpu_lib.primal_objective(Q, y, 1.0, torch.tensor(w, device=DEV))
    ref = float(np.sum(w * want))
    got = r.cpu().numpy()
    assert abs(got[0] - ref) <= 1e-13 * np.sum(np.abs(w * want))
    assert np.all(got[1:] == 0.0)
