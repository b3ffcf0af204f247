"""The C-ABI library: it loads, exports every entry point include/cabcd.h
declares, and rejects invalid arguments before touching the GPU."""

import ctypes
import os
import re

import pytest

import paper_1612_04003_amd as cabcd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cabcd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cabcd_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared() == sorted(cabcd.exported_symbols())


def test_library_exports_every_declared_symbol():
    lib = cabcd.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.cabcd_version().decode().startswith("cabcd")


def test_struct_layout_matches_header():
    # Field order and sizes of the two structs as the header declares them.
    assert ctypes.sizeof(cabcd.Matrix) == 4 + 4 + 8 * 9
    assert ctypes.sizeof(cabcd.Opts) == (8 + 4 + 4 + 4 + 4 + 8 + 8 + 8 + 8 + 8 + 8
                                         + 8 + 4 + 4 + 8 + 8)


def _fake_matrix(rows, cols, kind=cabcd.DENSE, dtype=cabcd.F64):
    m = cabcd.Matrix()
    m.kind, m.dtype, m.rows, m.cols = kind, dtype, rows, cols
    m.data = 0x1000          # never dereferenced: validation fails first
    m.ld = cols
    return m


@pytest.mark.parametrize("kw,status", [
    (dict(lam=0.0), cabcd.EINVAL),
    (dict(lam=-1.0), cabcd.EINVAL),
    (dict(lam=float("nan")), cabcd.EINVAL),
    (dict(b=0), cabcd.EINVAL),
    (dict(b=65), cabcd.EINVAL),        # b > d
    (dict(s=0), cabcd.EINVAL),
    (dict(H=-1), cabcd.EINVAL),
    (dict(b=33), cabcd.EUNSUPPORTED),
    (dict(b=16, s=33), cabcd.EUNSUPPORTED),   # s b = 528 > 512 dense
])
def test_primal_argument_errors(kw, status):
    lib = cabcd.load()
    args = dict(lam=1e-3, b=4, s=8, H=10)
    args.update(kw)
    M = _fake_matrix(64, 1024)
    st = lib.cabcd_primal_bcd(ctypes.byref(M), ctypes.c_void_p(0x2000), args["lam"],
                              args["b"], args["s"], args["H"], 1, ctypes.c_void_p(0x3000),
                              ctypes.c_void_p(0x4000), None, None)
    assert st == status
    assert lib.cabcd_last_error().decode() != ""


def test_csr_large_blocks_limit():
    # blocks of b > 16 take the 32-lane solves, which hold at most 512 rows
    lib = cabcd.load()
    M = _fake_matrix(20000, 1 << 20, kind=cabcd.CSR_KIND)
    M.rowptr, M.colidx, M.vals, M.nnz = 0x1000, 0x2000, 0x3000, 10
    for fn in (lib.cabcd_primal_bcd, lib.cabcd_dual_bcd):
        st = fn(ctypes.byref(M), ctypes.c_void_p(0x2000), 1e-3, 32, 17, 10, 1,
                ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), None, None)
        assert st == cabcd.EUNSUPPORTED
        assert "512" in lib.cabcd_last_error().decode()


def test_matrix_errors():
    lib = cabcd.load()
    st = lib.cabcd_primal_bcd(None, None, 1.0, 1, 1, 1, 0, None, None, None, None)
    assert st == cabcd.EINVAL
    M = _fake_matrix(64, 1024)
    M.ld = 100
    assert lib.cabcd_dual_bcd(ctypes.byref(M), ctypes.c_void_p(8), 1.0, 1, 1, 1, 0,
                              ctypes.c_void_p(8), ctypes.c_void_p(8), None, None) == cabcd.EINVAL
    M = _fake_matrix(64, 1024, dtype=7)
    assert lib.cabcd_gram(ctypes.byref(M), ctypes.c_void_p(8), 4, 1.0, 0.0, None,
                          ctypes.c_void_p(8), None, None) == cabcd.EINVAL
    assert lib.cabcd_sample(1, 0, 4, 5, 4, ctypes.c_void_p(8), None) == cabcd.EINVAL
    assert lib.cabcd_sample(1, -1, 4, 1, 4, ctypes.c_void_p(8), None) == cabcd.EINVAL


def test_workspace_bytes_grows_with_problem():
    lib = cabcd.load()
    a = lib.cabcd_workspace_bytes(ctypes.byref(_fake_matrix(64, 1024)), 4, 8)
    b = lib.cabcd_workspace_bytes(ctypes.byref(_fake_matrix(2048, 262144)), 8, 32)
    assert 0 < a < b
    assert lib.cabcd_workspace_bytes(ctypes.byref(_fake_matrix(64, 1024)), 16, 33) == 0
    # s b in (256, 512]: the four-part dense Gram needs more partials than s b = 256
    c = lib.cabcd_workspace_bytes(ctypes.byref(_fake_matrix(2048, 262144)), 16, 32)
    assert c > b


def test_batch_struct_layout_matches_header():
    assert ctypes.sizeof(cabcd.Problem) == ctypes.sizeof(cabcd.Matrix) + 8 * 8
    assert ctypes.sizeof(cabcd.BatchOpts) == 4 * 4
    assert ctypes.sizeof(cabcd.BatchInfo) == 4 * 4 + 8 * 3 + 8 + 4 + 4


def _fake_problem(**kw):
    q = cabcd.Problem()
    q.X = _fake_matrix(kw.pop("d", 64), kw.pop("n", 1024))
    q.y, q.w, q.r = 0x2000, 0x3000, 0x4000
    q.lam, q.b, q.s, q.seed, q.H = 1e-3, 4, 8, 1, 10
    for k, v in kw.items():
        setattr(q, k, v)
    return q


@pytest.mark.parametrize("kw,status", [
    (dict(lam=0.0), cabcd.EINVAL),
    (dict(lam=float("inf")), cabcd.EINVAL),
    (dict(b=-1), cabcd.EINVAL),
    (dict(b=17), cabcd.EINVAL),           # above the batched block limit
    (dict(b=65, d=64), cabcd.EINVAL),     # b > d
    (dict(b=16, s=33), cabcd.EINVAL),     # s*b > 512
    (dict(b=9, s=40), cabcd.EUNSUPPORTED),  # s*b = 360, but s*16 > 512 solve lanes
    (dict(s=-2), cabcd.EINVAL),
    (dict(y=0), cabcd.EINVAL),
    (dict(w=0), cabcd.EINVAL),
    (dict(n=0), cabcd.EINVAL),
])
def test_batch_argument_errors(kw, status):
    lib = cabcd.load()
    probs = (cabcd.Problem * 3)(_fake_problem(), _fake_problem(**kw), _fake_problem())
    h = ctypes.c_void_p(0x1)
    st = lib.cabcd_batch_create(probs, 3, None, None, ctypes.byref(h))
    assert st == status
    assert h.value is None
    msg = lib.cabcd_last_error().decode()
    assert "problem 1" in msg
    assert lib.cabcd_primal_bcd_batched(probs, 3, 10, None, None) == status


def test_batch_plan_errors():
    lib = cabcd.load()
    h = ctypes.c_void_p()
    assert lib.cabcd_batch_create(None, 1, None, None, ctypes.byref(h)) == cabcd.EINVAL
    probs = (cabcd.Problem * 1)(_fake_problem())
    assert lib.cabcd_batch_create(probs, 0, None, None, ctypes.byref(h)) == cabcd.EINVAL
    o = cabcd.BatchOpts()
    o.monitor_every = -1
    assert lib.cabcd_batch_create(probs, 1, ctypes.byref(o), None,
                                  ctypes.byref(h)) == cabcd.EINVAL
    assert lib.cabcd_batch_run(None, 1, None, None) == cabcd.EINVAL
    assert lib.cabcd_batch_query(None, 0, None, None) == cabcd.EINVAL
    assert lib.cabcd_batch_destroy(None) == cabcd.OK
    probs[0].X.kind = cabcd.CSR_KIND
    assert lib.cabcd_batch_create(probs, 1, None, None, ctypes.byref(h)) == cabcd.EUNSUPPORTED
    probs[0].X.kind, probs[0].X.dtype = cabcd.DENSE, cabcd.FP8_E4M3
    assert lib.cabcd_batch_create(probs, 1, None, None, ctypes.byref(h)) == cabcd.EINVAL
    assert "row scales" in lib.cabcd_last_error().decode()
    probs[0].X.dtype = 9
    assert lib.cabcd_batch_create(probs, 1, None, None, ctypes.byref(h)) == cabcd.EINVAL
    two = (cabcd.Problem * 2)(_fake_problem(), _fake_problem())
    two[1].X.dtype = cabcd.BF16
    assert lib.cabcd_batch_create(two, 2, None, None, ctypes.byref(h)) == cabcd.EINVAL
    assert "same storage type" in lib.cabcd_last_error().decode()


@pytest.mark.parametrize("kw", [
    dict(tol=-1.0, check_every=1),
    dict(tol=float("nan"), check_every=1),
    dict(tol=float("inf"), check_every=1),
    dict(tol=1e-3, check_every=0),           # a tolerance needs checks
    dict(tol=0.0, check_every=-2),
    dict(tol=1e-3, check_every=2, flags=cabcd.FLAG_ASYNC),   # checks read the norm on the host
])
def test_residual_check_option_errors(kw):
    lib = cabcd.load()
    o = cabcd._opts(**kw)
    M = _fake_matrix(64, 1024)
    for fn in (lib.cabcd_primal_bcd, lib.cabcd_dual_bcd):
        st = fn(ctypes.byref(M), ctypes.c_void_p(0x2000), 1e-3, 4, 8, 10, 1,
                ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), ctypes.byref(o), None)
        assert st == cabcd.EINVAL
        assert "check" in lib.cabcd_last_error().decode()


def test_residual_entry_point_errors():
    lib = cabcd.load()
    M = _fake_matrix(64, 1024)
    p = ctypes.c_void_p(0x2000)
    assert lib.cabcd_primal_residual(None, 1e-3, p, p, p, p, None) == cabcd.EINVAL
    assert lib.cabcd_primal_residual(ctypes.byref(M), 1e-3, None, p, p, p, None) == cabcd.EINVAL
    assert lib.cabcd_primal_residual(ctypes.byref(M), 1e-3, p, None, p, p, None) == cabcd.EINVAL
    assert lib.cabcd_primal_residual(ctypes.byref(M), -1.0, p, p, p, p, None) == cabcd.EINVAL
    assert lib.cabcd_primal_residual(ctypes.byref(M), 1e-3, p, p, None, None,
                                     None) == cabcd.EINVAL
    assert lib.cabcd_dual_residual(ctypes.byref(M), None, p, p, p, p, None) == cabcd.EINVAL
    assert lib.cabcd_dual_residual(ctypes.byref(M), p, p, p, None, None, None) == cabcd.EINVAL
    M.dtype = 9                           # no such storage type
    assert lib.cabcd_dual_residual(ctypes.byref(M), p, p, p, p, p, None) == cabcd.EINVAL


@pytest.mark.parametrize("dtype,es", [(cabcd.F64, 8), (cabcd.BF16, 2), (cabcd.FP8_E4M3, 1)])
def test_leading_dimension(dtype, es):
    """cabcd_leading_dim (host only): at least cols, rows on 256-byte
    boundaries, never a multiple of 64 KiB, at most 511 bytes of padding."""
    for cols in (1, 7, 127, 128, 4096, 8192, 32768, 65536, 100000, 1 << 18, 1 << 20,
                 (1 << 20) + 3):
        ld = cabcd.leading_dim(cols, dtype)
        assert ld >= cols
        assert (ld * es) % 256 == 0 and (ld * es) % 65536 != 0
        assert ld * es - cols * es < 512
    assert cabcd.leading_dim(1 << 20, dtype) * es == (1 << 20) * es + 256
    for bad in ((0, dtype), (-5, dtype), (10, 7)):
        with pytest.raises(cabcd.CabcdError) as e:
            cabcd.leading_dim(*bad)
        assert e.value.status == cabcd.EINVAL
