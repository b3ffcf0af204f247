"""cabcd_gram_noalloc (the Gram for callers that cannot allocate) against
cabcd_gram through the C-ABI: two calls in a row, the second with a smaller
input, for FP64 and the low-precision storage types; an index out of range is
reported through the device status word; after a warm-up call nothing is
allocated on the device.

Bars: FP64 entries within 1e-12 * scale * |Y||Y|^T of cabcd_gram's (the two
calls sum the same products in different slab orders); low-precision entries
within the FP32 accumulation bound of the mixed-precision Gram; Y u to 1e-12.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _codes(gpu_lib, A, dtype):
    if dtype == "f64":
        return A, A.cpu().numpy()
    code = gpu_lib.BF16 if dtype == "bf16" else gpu_lib.FP8_E4M3
    Q = gpu_lib.quantize(A, code)
    return Q, Q.dequantize().cpu().numpy()


def _bound(dtype, cols, scale, Y):
    rel = {"f64": 1e-12, "bf16": 2 * cols * 2.0 ** -24,
           "fp8": 2 * (cols * 2.0 ** -24 + 2.0 ** -12)}[dtype]
    return rel * scale * (Y @ Y.T) + 1e-300


@pytest.mark.parametrize("dtype", ["f64", "bf16", "fp8"])
def test_noalloc_gram_matches_gram_two_calls(gpu_lib, dtype):
    # (rows, cols, m): the first call's partials do not fit the fixed scratch
    # with cabcd_gram's slab plan at FP64 (256 x 2^18), so its slabs are
    # widened; the second call is smaller, with a ragged block row
    shapes = [(300, 1 << 18, 256), (90, 5001, 70)] if dtype == "f64" else \
             [(300, 1 << 18, 256), (90, 5008, 70)]
    g = torch.Generator().manual_seed(11)
    for rows, cols, m in shapes:
        _say("noalloc gram", dtype, rows, cols, m)
        A = torch.randn(rows, cols, generator=g, dtype=torch.float64).to(DEV)
        Astore, Ah = _codes(gpu_lib, A, dtype)
        idx = torch.randint(0, rows, (m,), generator=g, dtype=torch.int32).to(DEV)
        u = torch.randn(cols, generator=g, dtype=torch.float64).to(DEV)
        scale, shift = 1.0 / cols, 0.25
        G1, Yu1, st = gpu_lib.gram_noalloc(Astore, idx, scale, shift, u)
        G0, Yu0 = gpu_lib.gram(Astore, idx, scale, shift, u)
        torch.cuda.synchronize()
        assert int(st.item()) == gpu_lib.OK
        Y = np.abs(Ah[idx.cpu().numpy()])
        err = np.abs(G1.cpu().numpy() - G0.cpu().numpy())
        assert np.all(err <= _bound(dtype, cols, scale, Y))
        assert torch.equal(G1, G1.t())
        ub = 1e-12 * (Y @ np.abs(u.cpu().numpy())) + 1e-300
        assert np.all(np.abs(Yu1.cpu().numpy() - Yu0.cpu().numpy()) <= ub)
        # without u: G alone, the same values
        G2, Yu2, st2 = gpu_lib.gram_noalloc(Astore, idx, scale, shift)
        torch.cuda.synchronize()
        assert Yu2 is None and int(st2.item()) == gpu_lib.OK
        assert np.all(np.abs(G2.cpu().numpy() - G0.cpu().numpy()) <= _bound(dtype, cols, scale, Y))
        del A, Astore


def test_noalloc_reports_bad_index_and_allocates_nothing(gpu_lib):
    _say("noalloc status and memory")
    g = torch.Generator().manual_seed(12)
    A = torch.randn(40, 3000, generator=g, dtype=torch.float64).to(DEV)
    good = torch.tensor([0, 5, 39, 7], dtype=torch.int32, device=DEV)
    bad = torch.tensor([0, 5, 40, 7], dtype=torch.int32, device=DEV)
    neg = torch.tensor([-1, 3], dtype=torch.int32, device=DEV)
    G = torch.empty((4, 4), dtype=torch.float64, device=DEV)
    G2 = torch.empty((2, 2), dtype=torch.float64, device=DEV)
    st = torch.empty(1, dtype=torch.int32, device=DEV)
    # warm-up: every kernel of these calls has been loaded once
    gpu_lib.gram_noalloc(A, good, 1.0, 0.0, G=G, status=st)
    gpu_lib.gram_noalloc(A, neg, 1.0, 0.0, G=G2, status=st)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    gpu_lib.gram_noalloc(A, bad, 1.0, 0.0, G=G, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == gpu_lib.EINVAL
    gpu_lib.gram_noalloc(A, good, 1.0, 0.0, G=G, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == gpu_lib.OK
    gpu_lib.gram_noalloc(A, neg, 1.0, 0.0, G=G2, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == gpu_lib.EINVAL
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    Gr, _ = gpu_lib.gram(A, good, 1.0, 0.0)
    Y = np.abs(A.cpu().numpy()[good.cpu().numpy()])
    assert np.all(np.abs(G.cpu().numpy() - Gr.cpu().numpy()) <= 1e-12 * (Y @ Y.T))


def test_noalloc_argument_errors(gpu_lib):
    import ctypes
    lib = gpu_lib.load()
    A = torch.zeros((300, 64), dtype=torch.float64, device=DEV)
    M = gpu_lib.describe(A)
    idx = torch.zeros(257, dtype=torch.int32, device=DEV)
    G = torch.empty((257, 257), dtype=torch.float64, device=DEV)
    st = lib.cabcd_gram_noalloc(ctypes.byref(M), ctypes.c_void_p(idx.data_ptr()), 257, 1.0, 0.0,
                                None, ctypes.c_void_p(G.data_ptr()), None, None, None)
    assert st == gpu_lib.EUNSUPPORTED and b"256" in lib.cabcd_last_error()
    st = lib.cabcd_gram_noalloc(ctypes.byref(M), ctypes.c_void_p(idx.data_ptr()), 0, 1.0, 0.0,
                                None, ctypes.c_void_p(G.data_ptr()), None, None, None)
    assert st == gpu_lib.EINVAL
