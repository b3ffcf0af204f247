"""Python binding of libcabcd (CA-BCD / CA-BDCD on MI355X).

Argument marshalling only: every step of the method runs in the HIP kernels of
libcabcd.so.  Device memory and streams come from PyTorch tensors.  The
functions mirror the C entry points of include/cabcd.h without the `cabcd_`
prefix.  Loading fails loudly when the built library is missing; there is no
CPU fallback.
"""

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcabcd.so")

OK, EINVAL, ENOTSPD, EHIP, ENOMEM, EUNSUPPORTED, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
DENSE, CSR_KIND = 0, 1
F64, BF16, FP8_E4M3 = 0, 1, 2
FLAG_STATE_VALID, FLAG_ASYNC, FLAG_MONITOR_MAINTAINED, FLAG_FOLD_UPDATE = 1, 2, 4, 8

_STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOTSPD: "ENOTSPD", EHIP: "EHIP",
                 ENOMEM: "ENOMEM", EUNSUPPORTED: "EUNSUPPORTED", ENONFINITE: "ENONFINITE"}


class CabcdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Matrix(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("data", ctypes.c_void_p), ("ld", ctypes.c_int64),
                ("row_scale", ctypes.c_void_p),
                ("rowptr", ctypes.c_void_p), ("colidx", ctypes.c_void_p),
                ("vals", ctypes.c_void_p), ("nnz", ctypes.c_int64)]


class Opts(ctypes.Structure):
    _fields_ = [("h0", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("resid_every", ctypes.c_int32), ("monitor_every", ctypes.c_int32),
                ("timing_mask", ctypes.c_uint32),
                ("explicit_idx", ctypes.c_void_p),
                ("trace", ctypes.c_void_p), ("trace_len", ctypes.c_int64),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("timing", ctypes.POINTER(ctypes.c_double)),
                ("tol", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("reserved1", ctypes.c_int32),
                ("iters_done", ctypes.POINTER(ctypes.c_int64)),
                ("resid_norm", ctypes.POINTER(ctypes.c_double))]


class Problem(ctypes.Structure):
    _fields_ = [("X", Matrix), ("y", ctypes.c_void_p), ("lam", ctypes.c_double),
                ("b", ctypes.c_int32), ("s", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("H", ctypes.c_int64), ("f_target", ctypes.c_double),
                ("w", ctypes.c_void_p), ("r", ctypes.c_void_p)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("monitor_every", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("cheap_monitors", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("b", ctypes.c_int32), ("s", ctypes.c_int32), ("nslab", ctypes.c_int32),
                ("active", ctypes.c_int32), ("chunk", ctypes.c_int64), ("h", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("objective", ctypes.c_double),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


BATCH_NO_GRAPH = 1

NPHASES = 9
PHASES = ["sample", "gram", "reduce", "solve", "update", "recompute", "monitor", "check", "yu"]


_lib = None


def load():
    """Load libcabcd.so (built by build.py).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1612_04003_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64, D, U32 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                ctypes.c_uint64, ctypes.c_double, ctypes.c_uint32)
    MP = ctypes.POINTER(Matrix)
    OP = ctypes.POINTER(Opts)
    sigs = {
        "cabcd_opts_init": (None, [OP]),
        "cabcd_sample": (I32, [U64, I64, I64, I32, I64, P, P]),
        "cabcd_gram": (I32, [MP, P, I32, D, D, P, P, P, P]),
        "cabcd_gram_noalloc": (I32, [MP, P, I32, D, D, P, P, P, P, P]),
        "cabcd_primal_bcd": (I32, [MP, P, D, I32, I32, I64, U64, P, P, OP, P]),
        "cabcd_dual_bcd": (I32, [MP, P, D, I32, I32, I64, U64, P, P, OP, P]),
        "cabcd_primal_objective": (I32, [MP, P, D, P, P, P, P]),
        "cabcd_primal_objective_t": (I32, [MP, P, D, P, P, P, P]),
        "cabcd_dual_to_primal": (I32, [MP, P, D, P, P]),
        "cabcd_primal_residual": (I32, [MP, D, P, P, P, P, P]),
        "cabcd_dual_residual": (I32, [MP, P, P, P, P, P, P]),
        "cabcd_workspace_bytes": (ctypes.c_size_t, [MP, I32, I32]),
        "cabcd_quantize": (I32, [P, I64, I64, I64, I32, P, I64, P, P]),
        "cabcd_leading_dim": (I64, [I64, I32]),
        "cabcd_batch_create": (I32, [ctypes.POINTER(Problem), I32, ctypes.POINTER(BatchOpts), P,
                                     ctypes.POINTER(P)]),
        "cabcd_batch_run": (I32, [P, I64, P, ctypes.POINTER(I32)]),
        "cabcd_batch_query": (I32, [P, I32, ctypes.POINTER(BatchInfo), P]),
        "cabcd_batch_destroy": (I32, [P]),
        "cabcd_primal_bcd_batched": (I32, [ctypes.POINTER(Problem), I32, I64,
                                           ctypes.POINTER(BatchOpts), P]),
        "cabcd_last_error": (ctypes.c_char_p, []),
        "cabcd_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names of the C entry points this binding expects the library to export."""
    return ["cabcd_opts_init", "cabcd_sample", "cabcd_gram", "cabcd_gram_noalloc",
            "cabcd_primal_bcd",
            "cabcd_dual_bcd", "cabcd_primal_objective", "cabcd_primal_objective_t",
            "cabcd_dual_to_primal", "cabcd_primal_residual", "cabcd_dual_residual",
            "cabcd_workspace_bytes", "cabcd_last_error",
            "cabcd_version", "cabcd_quantize", "cabcd_leading_dim", "cabcd_batch_create",
            "cabcd_batch_run",
            "cabcd_batch_query", "cabcd_batch_destroy", "cabcd_primal_bcd_batched"]


def _check(status):
    if status != OK:
        msg = load().cabcd_last_error()
        raise CabcdError(status, msg.decode() if msg else "")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, name, numel=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


def dense(A):
    """Describe a row-major 2-D FP64 CUDA tensor (rows = samplable coordinates)."""
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("dense matrix must be 2-D with unit column stride")
    if not A.is_cuda:
        raise TypeError("matrix must live on the GPU")
    if A.dtype != torch.float64:
        raise TypeError("dense matrix must be float64")
    m = Matrix()
    m.kind, m.dtype = DENSE, F64
    m.rows, m.cols = A.shape
    m.data = A.data_ptr()
    m.ld = A.stride(0)
    m.row_scale = None
    m._keep = A
    return m


def new_timing():
    """Host array for per-phase timing (milliseconds, then launch counts)."""
    return (ctypes.c_double * (2 * NPHASES))()


def timing_dict(t):
    return {name: {"ms": t[i], "launches": int(t[NPHASES + i])} for i, name in enumerate(PHASES)}


class CSR:
    """A CSR matrix on the GPU: rowptr (int64, rows+1), colidx (int32, nnz,
    strictly increasing within a row), vals (float64, nnz), shape (rows, cols)."""

    def __init__(self, rowptr, colidx, vals, shape):
        _need(rowptr, torch.int64, "rowptr", shape[0] + 1)
        _need(colidx, torch.int32, "colidx")
        _need(vals, torch.float64, "vals", colidx.numel())
        self.rowptr, self.colidx, self.vals = rowptr, colidx, vals
        self.shape = (int(shape[0]), int(shape[1]))
        self.device = vals.device

    @classmethod
    def from_scipy(cls, S, device="cuda"):
        S = S.tocsr()
        S.sort_indices()
        return cls(torch.as_tensor(S.indptr.astype("int64")).to(device),
                   torch.as_tensor(S.indices.astype("int32")).to(device),
                   torch.as_tensor(S.data.astype("float64")).to(device), S.shape)


class Quantized:
    """Dense low-precision storage: codes (uint16 BF16 or uint8 E4M3 as int16 /
    uint8 tensors, rows x cols), FP32 row scales (or None), dtype BF16 / FP8_E4M3."""

    def __init__(self, codes, scales, dtype):
        self.codes, self.scales, self.dtype = codes, scales, dtype
        self.shape = tuple(codes.shape)
        self.device = codes.device

    def dequantize(self):
        """X^ in FP64 (exact), computed with torch for tests and baselines; its
        rows are leading_dim(cols, F64) apart."""
        rows, cols = self.shape
        out = empty_dense(rows, cols, self.device)
        view = torch.bfloat16 if self.dtype == BF16 else torch.float8_e4m3fn
        for r0 in range(0, rows, 1024):   # row blocks keep the FP64 temporaries small
            r1 = min(rows, r0 + 1024)
            x = self.codes[r0:r1].view(view).to(torch.float64)
            if self.scales is not None:
                x = x * self.scales[r0:r1].to(torch.float64)[:, None]
            out[r0:r1] = x
        return out


def leading_dim(cols, dtype):
    """cabcd_leading_dim: the leading dimension (elements) to allocate a dense
    matrix of `cols` columns with (F64, BF16 or FP8_E4M3)."""
    ld = load().cabcd_leading_dim(int(cols), int(dtype))
    if ld < 0:
        msg = load().cabcd_last_error()
        raise CabcdError(EINVAL, msg.decode() if msg else "")
    return ld


def empty_dense(rows, cols, device="cuda"):
    """An uninitialised rows x cols float64 matrix whose rows are
    leading_dim(cols, F64) apart (the view of a padded buffer)."""
    ld = leading_dim(cols, F64)
    return torch.empty((rows, ld), dtype=torch.float64, device=device)[:, :cols]


def quantize(A, dtype):
    """Store the FP64 matrix A (rows x cols) as BF16 or FP8-E4M3 codes.  The
    codes' rows start on 16-byte boundaries (leading dimension from
    leading_dim, padded with zero codes), which is what the 16-byte loads and
    the LDS-DMA paths of the kernels need; `codes` is the rows x cols view."""
    if not isinstance(A, torch.Tensor) or not A.is_cuda or A.dtype != torch.float64:
        raise TypeError("A must be a float64 CUDA (HIP) tensor")
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be 2-D with unit column stride")
    rows, cols = A.shape
    if dtype not in (BF16, FP8_E4M3):
        raise ValueError("dtype must be BF16 or FP8_E4M3")
    ldq = leading_dim(cols, dtype)
    if dtype == BF16:
        buf = torch.zeros((rows, ldq), dtype=torch.int16, device=A.device)
        scales = None
    else:
        buf = torch.zeros((rows, ldq), dtype=torch.uint8, device=A.device)
        scales = torch.empty(rows, dtype=torch.float32, device=A.device)
    _check(load().cabcd_quantize(_ptr(A), rows, cols, A.stride(0), dtype, _ptr(buf), ldq,
                                 _ptr(scales), _stream()))
    return Quantized(buf[:, :cols], scales, dtype)


def describe(A):
    """cabcd_matrix for a dense float64 CUDA tensor, a Quantized or a CSR object."""
    if isinstance(A, Quantized):
        m = Matrix()
        m.kind, m.dtype = DENSE, A.dtype
        m.rows, m.cols = A.shape
        m.data = A.codes.data_ptr()
        m.ld = A.codes.stride(0)
        m.row_scale = None if A.scales is None else A.scales.data_ptr()
        m._keep = A
        return m
    if isinstance(A, CSR):
        m = Matrix()
        m.kind, m.dtype = CSR_KIND, F64
        m.rows, m.cols = A.shape
        m.rowptr, m.colidx, m.vals = (A.rowptr.data_ptr(), A.colidx.data_ptr(),
                                      A.vals.data_ptr())
        m.nnz = A.colidx.numel()
        m._keep = A
        return m
    return dense(A)


def _opts(h0=0, flags=0, resid_every=0, monitor_every=0, explicit_idx=None, trace=None,
          workspace=None, timing=None, timing_mask=0, tol=0.0, check_every=0, stats=None):
    """cabcd_opts from keywords.  `stats`, a dict, receives "h" (inner
    iterations performed) and "resid_norm" (norm at the last residual check)
    after the call."""
    o = Opts()
    load().cabcd_opts_init(ctypes.byref(o))
    o.h0, o.flags = h0, flags
    o.resid_every, o.monitor_every = resid_every, monitor_every
    o.tol, o.check_every = float(tol), int(check_every)
    o._h, o._norm, o._stats = ctypes.c_int64(0), ctypes.c_double(0.0), stats
    o.iters_done = ctypes.pointer(o._h)
    o.resid_norm = ctypes.pointer(o._norm)
    if explicit_idx is not None:
        _need(explicit_idx, torch.int32, "explicit_idx")
        o.explicit_idx = explicit_idx.data_ptr()
    if trace is not None:
        _need(trace, torch.float64, "trace")
        o.trace, o.trace_len = trace.data_ptr(), trace.numel()
    if workspace is not None:
        _need(workspace, torch.uint8, "workspace")
        o.workspace, o.workspace_bytes = workspace.data_ptr(), workspace.numel()
    if timing is not None:
        o.timing = ctypes.cast(timing, ctypes.POINTER(ctypes.c_double))
        o.timing_mask = timing_mask
    return o


def _report(o):
    if o._stats is not None:
        o._stats["h"] = int(o._h.value)
        o._stats["resid_norm"] = float(o._norm.value)


def _check_explicit(opt, H, b):
    e = opt.get("explicit_idx")
    if e is not None and e.numel() < H * b:
        raise ValueError(f"explicit_idx holds {e.numel()} indices, need H*b = {H * b}")


def sample(seed, h0, count, b, rng, out=None):
    """Blocks of iterations h0 .. h0+count-1 as an int32 (count, b) tensor."""
    if out is None:
        out = torch.empty((count, b), dtype=torch.int32, device="cuda")
    _need(out, torch.int32, "out", count * b)
    _check(load().cabcd_sample(seed, h0, count, b, rng, _ptr(out), _stream()))
    return out


def gram(A, idx, scale, shift, u=None):
    """(scale * Y Y^T + shift I, Y u) for the rows idx of A (dense or CSR)."""
    M = describe(A)
    _need(idx, torch.int32, "idx")
    m = idx.numel()
    G = torch.empty((m, m), dtype=torch.float64, device=A.device)
    Yu = None
    if u is not None:
        _need(u, torch.float64, "u", A.shape[1])
        Yu = torch.empty(m, dtype=torch.float64, device=A.device)
    _check(load().cabcd_gram(ctypes.byref(M), _ptr(idx), m, scale, shift, _ptr(u), _ptr(G),
                             _ptr(Yu), _stream()))
    return G, Yu


def gram_noalloc(A, idx, scale, shift, u=None, G=None, Yu=None, status=None):
    """cabcd_gram_noalloc: the Gram of gram() for a dense A without any device
    allocation inside the library.  G (m x m float64), Yu (m float64, with u)
    and status (1-element int32) may be passed in; missing ones are created
    here, outside the call.  Returns (G, Yu, status); status holds the device
    check of the indices (OK or EINVAL) once the stream reaches it."""
    M = describe(A)
    _need(idx, torch.int32, "idx")
    m = idx.numel()
    if G is None:
        G = torch.empty((m, m), dtype=torch.float64, device=A.device)
    _need(G, torch.float64, "G", m * m)
    if u is not None:
        _need(u, torch.float64, "u", A.shape[1])
        if Yu is None:
            Yu = torch.empty(m, dtype=torch.float64, device=A.device)
        _need(Yu, torch.float64, "Yu", m)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=A.device)
    _need(status, torch.int32, "status", 1)
    _check(load().cabcd_gram_noalloc(ctypes.byref(M), _ptr(idx), m, scale, shift, _ptr(u),
                                     _ptr(G), _ptr(Yu if u is not None else None), _ptr(status),
                                     _stream()))
    return G, Yu, status


def primal_bcd(X, y, lam, b, s, H, seed, w=None, r=None, **opt):
    """Primal CA-BCD on A = X (d x n, dense or CSR).  Returns (w_H, r_H = z_H - y)."""
    M = describe(X)
    d, n = X.shape
    _need(y, torch.float64, "y", n)
    if w is None:
        w = torch.zeros(d, dtype=torch.float64, device=X.device)
    _need(w, torch.float64, "w", d)
    if r is None:
        r = torch.empty(n, dtype=torch.float64, device=X.device)
    _need(r, torch.float64, "r", n)
    _check_explicit(opt, H, b)
    o = _opts(**opt)
    _check(load().cabcd_primal_bcd(ctypes.byref(M), _ptr(y), lam, b, s, H, seed, _ptr(w),
                                   _ptr(r), ctypes.byref(o), _stream()))
    _report(o)
    return w, r


def dual_bcd(XT, y, lam, b, s, H, seed, alpha=None, w=None, **opt):
    """Dual CA-BDCD on A = X^T (n x d, dense or CSR).  Returns (alpha_H, w_H)."""
    M = describe(XT)
    n, d = XT.shape
    _need(y, torch.float64, "y", n)
    if alpha is None:
        alpha = torch.zeros(n, dtype=torch.float64, device=XT.device)
    _need(alpha, torch.float64, "alpha", n)
    if w is None:
        w = torch.empty(d, dtype=torch.float64, device=XT.device)
    _need(w, torch.float64, "w", d)
    _check_explicit(opt, H, b)
    o = _opts(**opt)
    _check(load().cabcd_dual_bcd(ctypes.byref(M), _ptr(y), lam, b, s, H, seed, _ptr(alpha),
                                 _ptr(w), ctypes.byref(o), _stream()))
    _report(o)
    return alpha, w


def primal_objective(X, y, lam, w, r=None):
    """(f(w), r = X^T w - y) from A = X."""
    M = describe(X)
    f = torch.empty(1, dtype=torch.float64, device=X.device)
    if r is None:
        r = torch.empty(X.shape[1], dtype=torch.float64, device=X.device)
    _check(load().cabcd_primal_objective(ctypes.byref(M), _ptr(y), lam, _ptr(w), _ptr(r),
                                         _ptr(f), _stream()))
    return f, r


def primal_objective_t(XT, y, lam, w, r=None):
    """(f(w), r = X^T w - y) from A = X^T."""
    M = describe(XT)
    f = torch.empty(1, dtype=torch.float64, device=XT.device)
    if r is None:
        r = torch.empty(XT.shape[0], dtype=torch.float64, device=XT.device)
    _check(load().cabcd_primal_objective_t(ctypes.byref(M), _ptr(y), lam, _ptr(w), _ptr(r),
                                           _ptr(f), _stream()))
    return f, r


def primal_residual(X, lam, w, r, rho=None):
    """(||rho||_2 as a 1-element tensor, rho) with rho = -lam w - 1/n X r, the
    full primal residual of the stopping test, from A = X."""
    M = describe(X)
    norm = torch.empty(1, dtype=torch.float64, device=X.device)
    if rho is None:
        rho = torch.empty(X.shape[0], dtype=torch.float64, device=X.device)
    _need(rho, torch.float64, "rho", X.shape[0])
    _check(load().cabcd_primal_residual(ctypes.byref(M), lam, _ptr(w), _ptr(r), _ptr(rho),
                                        _ptr(norm), _stream()))
    return norm, rho


def dual_residual(XT, y, alpha, w, rho=None):
    """(||rho||_2 as a 1-element tensor, rho) with rho = -X^T w + alpha + y, the
    full dual residual of the stopping test, from A = X^T."""
    M = describe(XT)
    norm = torch.empty(1, dtype=torch.float64, device=XT.device)
    if rho is None:
        rho = torch.empty(XT.shape[0], dtype=torch.float64, device=XT.device)
    _need(rho, torch.float64, "rho", XT.shape[0])
    _check(load().cabcd_dual_residual(ctypes.byref(M), _ptr(y), _ptr(alpha), _ptr(w), _ptr(rho),
                                      _ptr(norm), _stream()))
    return norm, rho


def dual_to_primal(XT, alpha, lam, w=None):
    """w = -X alpha / (lambda n) from A = X^T."""
    M = describe(XT)
    if w is None:
        w = torch.empty(XT.shape[1], dtype=torch.float64, device=XT.device)
    _check(load().cabcd_dual_to_primal(ctypes.byref(M), _ptr(alpha), lam, _ptr(w), _stream()))
    return w


def workspace_bytes(A, b, s):
    M = describe(A)
    return int(load().cabcd_workspace_bytes(ctypes.byref(M), b, s))


# ------------------------------------------------------------------ batched


def _problems(problems):
    """ctypes array of cabcd_problem from dicts with keys X, y, lam and optional
    b, s (0: autotuned), seed, H (<= 0: unlimited), f_target (<= 0: none), w, r."""
    arr = (Problem * len(problems))()
    keep = []
    for i, q in enumerate(problems):
        X, y = q["X"], q["y"]
        d, n = X.shape
        _need(y, torch.float64, f"problems[{i}].y", n)
        w = q.get("w")
        if w is None:
            w = torch.zeros(d, dtype=torch.float64, device=X.device)
            q["w"] = w
        _need(w, torch.float64, f"problems[{i}].w", d)
        r = q.get("r")
        if r is None:
            r = torch.empty(n, dtype=torch.float64, device=X.device)
            q["r"] = r
        _need(r, torch.float64, f"problems[{i}].r", n)
        M = describe(X)
        arr[i].X = M
        arr[i].y, arr[i].lam = y.data_ptr(), float(q["lam"])
        arr[i].b, arr[i].s = int(q.get("b", 0)), int(q.get("s", 0))
        arr[i].seed, arr[i].H = int(q.get("seed", 0)), int(q.get("H", 0))
        arr[i].f_target = float(q.get("f_target", 0.0))
        arr[i].w, arr[i].r = w.data_ptr(), r.data_ptr()
        keep.append((M, X, y, w, r))
    return arr, keep


class Batch:
    """A plan of many primal ridge problems solved by batched CA-BCD: one
    persistent launch per round for the whole batch, captured in a hipGraph.
    `problems` is a list of dicts (see _problems); w and r are created when
    absent and written in place (q["w"], q["r"])."""

    def __init__(self, problems, monitor_every=4, graph=True, cheap_monitors=0):
        self.problems = problems
        arr, self._keep = _problems(problems)
        o = BatchOpts()
        o.monitor_every, o.flags = monitor_every, 0 if graph else BATCH_NO_GRAPH
        o.cheap_monitors = cheap_monitors
        h = ctypes.c_void_p()
        _check(load().cabcd_batch_create(arr, len(problems), ctypes.byref(o), _stream(),
                                         ctypes.byref(h)))
        self._h = h

    def run(self, rounds, sync=True):
        """Run `rounds` rounds; with sync, return the number of active problems."""
        act = ctypes.c_int32(-1)
        _check(load().cabcd_batch_run(self._h, rounds, _stream(),
                                      ctypes.byref(act) if sync else None))
        return act.value if sync else None

    def info(self, p):
        i = BatchInfo()
        _check(load().cabcd_batch_query(self._h, p, ctypes.byref(i), _stream()))
        return {"b": i.b, "s": i.s, "nslab": i.nslab, "active": bool(i.active),
                "chunk": i.chunk, "h": i.h, "steps": i.steps, "objective": i.objective,
                "status": i.status}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value is not None:
            load().cabcd_batch_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def primal_bcd_batched(problems, max_rounds, monitor_every=4, graph=True, cheap_monitors=0):
    """One-shot batched solve (plan, run until no problem is active or
    max_rounds, release).  Results are written to each problem's w and r."""
    arr, keep = _problems(problems)
    o = BatchOpts()
    o.monitor_every, o.flags = monitor_every, 0 if graph else BATCH_NO_GRAPH
    o.cheap_monitors = cheap_monitors
    _check(load().cabcd_primal_bcd_batched(arr, len(problems), max_rounds, ctypes.byref(o),
                                           _stream()))
    del keep
    return problems
