"""Python binding of librqrcp: truncated randomized QR with column pivoting on MI355X.

Thin ctypes marshalling over the C ABI declared in ``include/rqrcp.h``: torch
tensors supply device memory and the current HIP stream; every step of the
factorization runs in the library's HIP kernels.  Importing works without a
GPU; calling anything that computes requires the built ``librqrcp.so`` and a
gfx950 device, and raises otherwise (there is no fallback path).

Matrices are column-major: an m x n matrix is a tensor of shape (m, n) with
strides (1, ld), e.g. ``torch.empty(n, m).t()``.  ``colmajor(x)`` converts.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librqrcp.so")

F64 = 0
F32 = 1
BF16 = 2
F8E4M3 = 3
SKETCH_TYPES = {"f64": F64, "bf16": BF16, "fp8": F8E4M3}
FROZEN_PIVOTS = 1
USER_SKETCH = 2
HOUSEHOLDER_PANEL = 4
TOURNAMENT = 8
TOURNAMENT_GROUP = 256
TOURNAMENT_FANOUT = 4
SRQR_EXACT = 1

STATUS = {
    1001: "HIP runtime error", 1002: "workspace too small",
    1003: "unsupported data type combination", 1004: "device is not gfx950",
    1005: "size beyond the kernels' limits", 1006: "grid barrier timed out",
    1007: "non-finite value in the sketch", 1008: "jpvt is not a permutation of 0..n-1",
    1009: "sizes need more than the static scratch of rqrcp_factor_noalloc",
}
NOALLOC_MAX_BYTES = 64 << 20

# Every symbol declared in include/rqrcp.h.
EXPORTS = (
    "rqrcp_create", "rqrcp_destroy", "rqrcp_set_stream", "rqrcp_workspace_size",
    "rqrcp_limits", "rqrcp_gaussian", "rqrcp_sketch", "rqrcp_factor", "rqrcp_form_q",
    "rqrcp_check", "rqrcp_status_string", "rqrcp_set_timing", "rqrcp_read_timing",
    "srqr_workspace_size", "srqr_swap", "rqrcp_backward_workspace_size", "rqrcp_backward",
    "rqrcp_batched_limits", "rqrcp_batched_workspace_size", "rqrcp_factor_batched",
    "rqrcp_autotune_batched", "rqrcp_qrcp_workspace_size", "rqrcp_qrcp", "rqrcp_factor_tol",
    "rqrcp_cx_workspace_size", "rqrcp_cx", "rqrcp_cur_workspace_size", "rqrcp_cur",
    "rqrcp_compress_workspace_size", "rqrcp_compress", "rqrcp_factor_noalloc",
)
PHASES = ("sketch", "qrcp", "swap", "panel", "trail", "bupdate", "other", "final")


class Params(ctypes.Structure):
    _fields_ = [("b", ctypes.c_int), ("p", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("a_type", ctypes.c_int), ("sketch_type", ctypes.c_int),
                ("flags", ctypes.c_uint)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librqrcp.so (no GPU needed).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"librqrcp.so not built ({path}); run paper_1804_05138_amd/build.py")
    # torch first: the library must bind to the HIP runtime torch loads (its
    # streams and allocations are passed straight through), not pull in a
    # second copy that torch would then pick up in place of its own
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i, u64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t
    i64 = ctypes.c_int64
    P = ctypes.POINTER
    sig = {
        "rqrcp_create": (i, [P(vp), vp]),
        "rqrcp_destroy": (i, [vp]),
        "rqrcp_set_stream": (i, [vp, vp]),
        "rqrcp_workspace_size": (i, [i, i, i, P(Params), P(sz)]),
        "rqrcp_limits": (i, [i, P(i), P(i), P(i)]),
        "rqrcp_gaussian": (i, [vp, i, i, u64, u64, vp, i]),
        "rqrcp_sketch": (i, [vp, i, i, i, u64, i, vp, i, i, vp, i, vp, i, vp, sz]),
        "rqrcp_factor": (i, [vp, i, i, i, P(Params), vp, i, vp, vp, vp, i, vp, vp, sz]),
        "rqrcp_factor_noalloc": (i, [vp, i, i, i, P(Params), vp, i, vp, vp, vp, i, vp]),
        "rqrcp_form_q": (i, [vp, i, i, i, i, vp, i, vp, vp, i, vp, sz]),
        "rqrcp_check": (i, [vp, vp]),
        "srqr_workspace_size": (i, [i, i, i, P(Params), i, ctypes.c_uint, P(sz)]),
        "rqrcp_backward_workspace_size": (i, [i, i, i, i, i, P(sz)]),
        "rqrcp_batched_limits": (i, [P(i), P(i), P(i), P(i)]),
        "rqrcp_batched_workspace_size": (i, [P(sz)]),
        "rqrcp_factor_batched": (i, [vp, i, vp, P(Params), vp, i64, vp, i64, vp, i64, vp, i64,
                                     vp, vp, sz]),
        "rqrcp_autotune_batched": (i, [vp, i, vp, P(Params), vp, i64, vp, i64, vp, i64, vp, i64,
                                       vp, vp, sz, vp, P(i), P(ctypes.c_float)]),
        "rqrcp_backward": (i, [vp, i, i, i, i, i, vp, i, vp, i, vp, vp, vp, i, vp, i, vp, i,
                               vp, sz]),
        "srqr_swap": (i, [vp, i, i, i, P(Params), ctypes.c_double, i, i, ctypes.c_uint,
                          vp, i, vp, i, vp, vp, vp, i, vp, vp, vp, vp, sz]),
        "rqrcp_qrcp_workspace_size": (i, [i, i, i, i, P(sz)]),
        "rqrcp_cx_workspace_size": (i, [i, i, i, P(sz)]),
        "rqrcp_cx": (i, [vp, i, i, i, vp, i, vp, vp, i, vp, sz]),
        "rqrcp_cur_workspace_size": (i, [i, i, i, i, P(sz)]),
        "rqrcp_cur": (i, [vp, i, i, i, i, vp, i, vp, vp, i, vp, vp, i, vp, sz]),
        "rqrcp_compress_workspace_size": (i, [i, i, i, i, i, P(sz)]),
        "rqrcp_compress": (i, [vp, i, i, i, i, i, vp, i, vp, vp, vp, i, vp, i, vp, vp, sz]),
        "rqrcp_factor_tol": (i, [vp, i, i, i, ctypes.c_double, P(Params), vp, i, vp, vp, vp, i,
                                 vp, P(i), P(ctypes.c_double), vp, sz]),
        "rqrcp_qrcp": (i, [vp, i, i, i, i, vp, i, vp, vp, vp, sz]),
        "rqrcp_status_string": (ctypes.c_char_p, [i]),
        "rqrcp_set_timing": (i, [vp, i]),
        "rqrcp_read_timing": (i, [vp, P(ctypes.c_double), P(i), P(ctypes.c_double),
                                  P(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        msg = STATUS.get(status, "invalid argument %d" % -status if status < 0 else "error")
        raise RuntimeError(f"{what}: librqrcp status {status} ({msg})")


# ---------------------------------------------------------------------------
# handles and tensors
# ---------------------------------------------------------------------------

_handles = {}


def _torch():
    import torch
    return torch


def handle():
    """The library handle bound to the current device and its current stream."""
    torch = _torch()
    lib = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("librqrcp needs a GPU (torch.cuda is not available)")
    stream = torch.cuda.current_stream().cuda_stream
    key = (torch.cuda.current_device(), stream)
    h = _handles.get(key)
    if h is None:
        h = ctypes.c_void_p()
        _check(lib.rqrcp_create(ctypes.byref(h), ctypes.c_void_p(stream)), "rqrcp_create")
        _handles[key] = h
    return h


def colmajor(x, dtype=None):
    """Column-major copy (strides (1, rows)) of a 2-D tensor, unless it already is one."""
    torch = _torch()
    if dtype is not None and x.dtype != dtype:
        x = x.to(dtype)
    if x.dim() != 2:
        raise ValueError("expected a matrix")
    if x.stride(0) == 1 and x.stride(1) >= max(1, x.shape[0]):
        return x
    return x.t().contiguous().t()


def empty_colmajor(m, n, dtype, device):
    torch = _torch()
    return torch.empty((n, m), dtype=dtype, device=device).t()


def _ld(x):
    return max(1, x.stride(1)) if x.shape[1] > 1 else max(1, x.shape[0])


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else ctypes.c_void_p(0)


def _a_type(dtype):
    torch = _torch()
    if dtype == torch.float64:
        return F64
    if dtype == torch.float32:
        return F32
    raise ValueError(f"unsupported matrix dtype {dtype} (float64 or float32)")


def _sketch_type(st):
    if isinstance(st, int):
        return st
    try:
        return SKETCH_TYPES[st]
    except KeyError:
        raise ValueError(f"sketch type {st!r}: one of {sorted(SKETCH_TYPES)}") from None


def workspace_bytes(m, n, k, b, p, flags=0, a_type=F64, sketch_type=F64):
    lib = load_library()
    out = ctypes.c_size_t()
    prm = Params(b, p, 0, a_type, _sketch_type(sketch_type), flags)
    _check(lib.rqrcp_workspace_size(m, n, k, ctypes.byref(prm), ctypes.byref(out)),
           "rqrcp_workspace_size")
    return out.value


def workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(1, nbytes), dtype=torch.uint8, device=device)


def limits(l):
    lib = load_library()
    mb, ml, mn = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib.rqrcp_limits(l, ctypes.byref(mb), ctypes.byref(ml), ctypes.byref(mn))
    return mb.value, ml.value, mn.value


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------

def gaussian(rows, cols, seed, stream=0, device="cuda"):
    """Omega (rows x cols) from Philox4x64-10 key (seed, stream)."""
    torch = _torch()
    h = handle()
    out = empty_colmajor(rows, cols, torch.float64, device)
    _check(load_library().rqrcp_gaussian(h, rows, cols, seed, stream, _ptr(out),
                                          max(1, rows)), "rqrcp_gaussian")
    return out


def sketch(a, l, seed=0, omega=None, ws=None, sketch_type="f64"):
    """B = Omega A (l x n, FP64) for a column-major FP64 or FP32 A."""
    torch = _torch()
    if a.dtype not in (torch.float64, torch.float32):
        a = a.to(torch.float64)
    a = colmajor(a)
    m, n = a.shape
    at = _a_type(a.dtype)
    st = _sketch_type(sketch_type)
    h = handle()
    b = empty_colmajor(l, n, torch.float64, a.device)
    if omega is not None:
        omega = colmajor(omega, torch.float64)
    nbytes = workspace_bytes(m, n, 1, l, 0, 0, at, st)
    ws = workspace(nbytes, a.device) if ws is None else ws
    _check(load_library().rqrcp_sketch(h, m, n, l, seed, at, _ptr(a), _ld(a), st, _ptr(omega),
                                        _ld(omega) if omega is not None else 0, _ptr(b), l,
                                        _ptr(ws), ws.numel()), "rqrcp_sketch")
    return b


@dataclass
class Factorization:
    a: object       # m x n column-major: R, V, R22 (LAPACK storage)
    jpvt: object    # int32 (n,)
    tau: object     # float64 (k,)
    b: object       # sketch ((b+p) x n) or None
    info: object    # int32 (1,)
    k: int
    block: int


def factor(a, k, b, p, seed=0, *, jpvt=None, sketch_b=None, ws=None, inplace=False,
           check=True, sketch_type="f64", householder_panel=False, tournament=False):
    """Truncated RQRCP (Alg. 2) of the FP64 or FP32 matrix ``a`` to rank ``k``.

    jpvt: frozen pivots (the columns A(:, jpvt) are factored without pivoting).
    sketch_b: a precomputed sketch Omega A ((b+p) x n), e.g. with a custom Omega.
    sketch_type: "f64", "bf16" or "fp8" (the arithmetic of B = Omega A).
    An FP32 ``a`` is the mixed-precision form (FP32 trailing update and storage,
    FP64 reflectors, sketch and sample update).
    householder_panel: every panel one reflector at a time instead of by
    Cholesky-QR2 (RQRCP_HOUSEHOLDER_PANEL).
    tournament: pivots by QR with tournament pivoting on the sketch
    (RQRCP_TOURNAMENT; groups of 256 columns, four-way merges).
    Returns a Factorization with device tensors.
    """
    torch = _torch()
    if a.dtype not in (torch.float64, torch.float32):
        a = a.to(torch.float64)
    if inplace:
        if a.stride(0) != 1:
            raise ValueError("inplace needs a column-major tensor")
        af = a
    else:
        af = colmajor(a).clone(memory_format=torch.preserve_format)
        if af.stride(0) != 1:
            af = colmajor(af)
    m, n = af.shape
    dev = af.device
    flags = (HOUSEHOLDER_PANEL if householder_panel else 0) | (TOURNAMENT if tournament else 0)
    jp = torch.empty(n, dtype=torch.int32, device=dev)
    if jpvt is not None:
        flags |= FROZEN_PIVOTS
        jp.copy_(torch.as_tensor(jpvt, dtype=torch.int32, device=dev))
        bs = None
    elif sketch_b is not None:
        flags |= USER_SKETCH
        bs = colmajor(sketch_b, torch.float64).clone()
        if bs.stride(0) != 1:
            bs = colmajor(bs)
    else:
        bs = empty_colmajor(b + p, n, torch.float64, dev)
    tau = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    at, st = _a_type(af.dtype), _sketch_type(sketch_type)
    nbytes = workspace_bytes(m, n, k, b, p, flags, at, st)
    if ws is None or ws.numel() < nbytes:
        ws = workspace(nbytes, dev)
    prm = Params(b, p, seed, at, st, flags)
    lib = load_library()
    h = handle()
    _check(lib.rqrcp_factor(h, m, n, k, ctypes.byref(prm), _ptr(af), _ld(af), _ptr(jp),
                            _ptr(tau), _ptr(bs), (_ld(bs) if bs is not None else b + p),
                            _ptr(info), _ptr(ws), ws.numel()), "rqrcp_factor")
    if check:
        _check(lib.rqrcp_check(h, _ptr(ws)), "rqrcp_check")
    return Factorization(af, jp, tau, bs, info, k, b)


def factor_tol(a, tol, kmax, b, p, seed=0, *, sketch_b=None, ws=None, sketch_type="f64"):
    """Tolerance-driven RQRCP (rqrcp_factor_tol): blocks of Alg. 2 until the
    sketch estimate of ||R22||_F / ||A||_F is <= tol (at most kmax columns).
    Returns (Factorization with k = the rank reached, estimate ratio)."""
    torch = _torch()
    if a.dtype not in (torch.float64, torch.float32):
        a = a.to(torch.float64)
    af = colmajor(a).clone(memory_format=torch.preserve_format)
    if af.stride(0) != 1:
        af = colmajor(af)
    m, n = af.shape
    dev = af.device
    flags = 0
    if sketch_b is not None:
        flags |= USER_SKETCH
        bs = colmajor(sketch_b, torch.float64).clone()
        if bs.stride(0) != 1:
            bs = colmajor(bs)
    else:
        bs = empty_colmajor(b + p, n, torch.float64, dev)
    jp = torch.empty(n, dtype=torch.int32, device=dev)
    tau = torch.zeros(kmax, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    at, st = _a_type(af.dtype), _sketch_type(sketch_type)
    nbytes = workspace_bytes(m, n, kmax, b, p, flags, at, st)
    if ws is None or ws.numel() < nbytes:
        ws = workspace(nbytes, dev)
    prm = Params(b, p, seed, at, st, flags)
    kout = ctypes.c_int()
    est = ctypes.c_double()
    lib = load_library()
    _check(lib.rqrcp_factor_tol(handle(), m, n, kmax, float(tol), ctypes.byref(prm), _ptr(af),
                                _ld(af), _ptr(jp), _ptr(tau), _ptr(bs), _ld(bs), _ptr(info),
                                ctypes.byref(kout), ctypes.byref(est), _ptr(ws), ws.numel()),
           "rqrcp_factor_tol")
    _check(lib.rqrcp_check(handle(), _ptr(ws)), "rqrcp_check")
    k = kout.value
    return Factorization(af, jp, tau[:k], bs, info, k, b), est.value


def qrcp(a, k, nb=64, ws=None):
    """QR with column pivoting of the whole FP64 matrix ``a`` (Alg. 1, the
    comparator; rqrcp_qrcp): returns a Factorization (b = None)."""
    torch = _torch()
    af = colmajor(a, torch.float64).clone(memory_format=torch.preserve_format)
    if af.stride(0) != 1:
        af = colmajor(af)
    m, n = af.shape
    dev = af.device
    jp = torch.empty(n, dtype=torch.int32, device=dev)
    tau = torch.empty(k, dtype=torch.float64, device=dev)
    lib = load_library()
    nbytes = ctypes.c_size_t()
    _check(lib.rqrcp_qrcp_workspace_size(m, n, k, nb, ctypes.byref(nbytes)),
           "rqrcp_qrcp_workspace_size")
    if ws is None or ws.numel() < nbytes.value:
        ws = workspace(nbytes.value, dev)
    _check(lib.rqrcp_qrcp(handle(), m, n, k, nb, _ptr(af), _ld(af), _ptr(jp), _ptr(tau),
                          _ptr(ws), ws.numel()), "rqrcp_qrcp")
    return Factorization(af, jp, tau, None, None, k, nb)


def qrcp_into(a, k, nb, jpvt, tau, ws):
    """rqrcp_qrcp on caller-owned device buffers (no allocation, no sync)."""
    m, n = a.shape
    _check(load_library().rqrcp_qrcp(handle(), m, n, k, nb, _ptr(a), _ld(a), _ptr(jpvt),
                                      _ptr(tau), _ptr(ws), ws.numel()), "rqrcp_qrcp")


def qrcp_workspace_bytes(m, n, k, nb=64):
    out = ctypes.c_size_t()
    _check(load_library().rqrcp_qrcp_workspace_size(m, n, k, nb, ctypes.byref(out)),
           "rqrcp_qrcp_workspace_size")
    return out.value


def factor_into(a, k, b, p, seed, jpvt, tau, bsk, info, ws, flags=0, sketch_type="f64"):
    """rqrcp_factor on caller-owned device buffers (no allocation, no sync).

    a: column-major float64 or float32 (m x n), overwritten; jpvt int32 (n);
    tau float64 (k); bsk column-major float64 ((b+p) x n) or None with
    FROZEN_PIVOTS; info int32 (1); ws uint8 workspace of at least
    workspace_bytes(m, n, k, b, p, flags, a_type, sketch_type).
    """
    m, n = a.shape
    prm = Params(b, p, seed, _a_type(a.dtype), _sketch_type(sketch_type), flags)
    _check(load_library().rqrcp_factor(handle(), m, n, k, ctypes.byref(prm), _ptr(a), _ld(a),
                                        _ptr(jpvt), _ptr(tau), _ptr(bsk),
                                        (_ld(bsk) if bsk is not None else b + p), _ptr(info),
                                        _ptr(ws), ws.numel()), "rqrcp_factor")


def factor_noalloc_into(a, k, b, p, seed, jpvt, tau, bsk, info, flags=0, sketch_type="f64"):
    """rqrcp_factor_noalloc on caller-owned buffers: no workspace argument, the
    library's static device scratch instead (the call allocates nothing)."""
    m, n = a.shape
    prm = Params(b, p, seed, _a_type(a.dtype), _sketch_type(sketch_type), flags)
    _check(load_library().rqrcp_factor_noalloc(handle(), m, n, k, ctypes.byref(prm), _ptr(a),
                                                _ld(a), _ptr(jpvt), _ptr(tau), _ptr(bsk),
                                                (_ld(bsk) if bsk is not None else b + p),
                                                _ptr(info)), "rqrcp_factor_noalloc")


def form_q(fact_a, tau, k=None, b=64, ws=None):
    """Explicit Q1 (m x k) of a factorization in LAPACK storage (FP64 or FP32)."""
    torch = _torch()
    k = tau.numel() if k is None else k
    m = fact_a.shape[0]
    at = _a_type(fact_a.dtype)
    q = empty_colmajor(m, k, fact_a.dtype, fact_a.device)
    nbytes = workspace_bytes(m, k, k, b, 0, 0, at)
    ws = workspace(nbytes, fact_a.device) if ws is None or ws.numel() < nbytes else ws
    _check(load_library().rqrcp_form_q(handle(), m, k, b, at, _ptr(fact_a), _ld(fact_a),
                                        _ptr(tau), _ptr(q), max(1, m), _ptr(ws), ws.numel()),
           "rqrcp_form_q")
    return q


@dataclass
class SRQR:
    a: object       # m x n: the (l+1)-step factorization (LAPACK storage)
    jpvt: object    # int32 (n,)
    tau: object     # float64 (l+1,)
    g2: object      # float64 (1,): last g2 value
    nswaps: object  # int32 (1,)
    info: object    # int32 (1,): 0, or -max_swaps if the cap was reached


def srqr_into(a0, fact, g, seed=0, *, d=16, exact=False, max_swaps=-1, ws=None):
    """srqr_swap on an existing l-step factorization ``fact`` of ``a0`` (in place:
    fact.a, fact.jpvt; returns (tau of length l+1, g2, nswaps, info) tensors)."""
    torch = _torch()
    m, n = a0.shape
    l, b = fact.k, fact.block
    p = fact.b.shape[0] - b
    dev = a0.device
    tau = torch.zeros(l + 1, dtype=torch.float64, device=dev)
    tau[:l].copy_(fact.tau[:l])
    g2 = torch.zeros(1, dtype=torch.float64, device=dev)
    ns = torch.zeros(1, dtype=torch.int32, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    flags = SRQR_EXACT if exact else 0
    prm = Params(b, p, seed, F64, F64, 0)
    lib = load_library()
    nb = ctypes.c_size_t()
    _check(lib.srqr_workspace_size(m, n, l, ctypes.byref(prm), d, flags, ctypes.byref(nb)),
           "srqr_workspace_size")
    if ws is None or ws.numel() < nb.value:
        ws = workspace(nb.value, dev)
    _check(lib.srqr_swap(handle(), m, n, l, ctypes.byref(prm), float(g), d, max_swaps, flags,
                         _ptr(a0), _ld(a0), _ptr(fact.a), _ld(fact.a), _ptr(fact.jpvt),
                         _ptr(tau), _ptr(fact.b), _ld(fact.b), _ptr(g2), _ptr(ns), _ptr(info),
                         _ptr(ws), ws.numel()), "srqr_swap")
    return tau, g2, ns, info


def srqr(a0, l, b, p, g, seed=0, *, d=16, exact=False, max_swaps=-1, sketch_b=None):
    """Alg. 3: the l-step RQRCP of ``a0`` followed by spectrum-revealing swaps.

    sketch_b: a precomputed sketch (e.g. Omega = I) for the RQRCP start.
    Returns an SRQR with device tensors (synchronizes once per g2 evaluation).
    """
    torch = _torch()
    a0 = colmajor(a0, torch.float64)
    m, n = a0.shape
    dev = a0.device
    f = factor(a0, l, b, p, seed, sketch_b=sketch_b)
    tau = torch.zeros(l + 1, dtype=torch.float64, device=dev)
    tau[:l].copy_(f.tau)
    g2 = torch.zeros(1, dtype=torch.float64, device=dev)
    ns = torch.zeros(1, dtype=torch.int32, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    flags = SRQR_EXACT if exact else 0
    prm = Params(b, p, seed, F64, F64, 0)
    lib = load_library()
    nb = ctypes.c_size_t()
    _check(lib.srqr_workspace_size(m, n, l, ctypes.byref(prm), d, flags, ctypes.byref(nb)),
           "srqr_workspace_size")
    ws = workspace(nb.value, dev)
    _check(lib.srqr_swap(handle(), m, n, l, ctypes.byref(prm), float(g), d, max_swaps, flags,
                         _ptr(a0), _ld(a0), _ptr(f.a), _ld(f.a), _ptr(f.jpvt), _ptr(tau),
                         _ptr(f.b), _ld(f.b), _ptr(g2), _ptr(ns), _ptr(info), _ptr(ws),
                         ws.numel()), "srqr_swap")
    _check(lib.rqrcp_check(handle(), _ptr(ws)), "rqrcp_check")
    return SRQR(f.a, f.jpvt, tau, g2, ns, info)


def backward(a, fact, dq1=None, dr=None, check=True):
    """dL/dA of the frozen-pivot factorization ``fact`` of ``a`` (rqrcp_backward).

    dq1: m x k cotangent of Q1, dr: k x n cotangent of [R11 R12] (pivot order);
    either may be None (zero).  Returns dA (m x n, original column order).
    check: synchronize and raise if fact.jpvt was not a permutation.
    """
    torch = _torch()
    a = colmajor(a, fact.a.dtype)
    m, n = a.shape
    k, b = fact.k, fact.block
    at = _a_type(a.dtype)
    dq1 = colmajor(dq1, a.dtype) if dq1 is not None else None
    dr = colmajor(dr, a.dtype) if dr is not None else None
    da = empty_colmajor(m, n, a.dtype, a.device)
    lib = load_library()
    nb = ctypes.c_size_t()
    _check(lib.rqrcp_backward_workspace_size(m, n, k, b, at, ctypes.byref(nb)),
           "rqrcp_backward_workspace_size")
    ws = workspace(nb.value, a.device)
    _check(lib.rqrcp_backward(handle(), m, n, k, b, at, _ptr(a), _ld(a), _ptr(fact.a),
                              _ld(fact.a), _ptr(fact.tau), _ptr(fact.jpvt), _ptr(dq1),
                              _ld(dq1) if dq1 is not None else m, _ptr(dr),
                              _ld(dr) if dr is not None else k, _ptr(da), _ld(da), _ptr(ws),
                              ws.numel()), "rqrcp_backward")
    if check:
        _check(lib.rqrcp_check(handle(), _ptr(ws)), "rqrcp_check")
    return da


# ---------------------------------------------------------------------------
# uses of a factorization: CX, CUR, SVD compression
# ---------------------------------------------------------------------------

def cx_from(fact, k=None):
    """X = C^+ A (k x n) for C = A(:, jpvt[0:k]) from a factorization (rqrcp_cx)."""
    torch = _torch()
    k = fact.k if k is None else k
    m, n = fact.a.shape
    x = empty_colmajor(k, n, torch.float64, fact.a.device)
    lib = load_library()
    nb = ctypes.c_size_t()
    _check(lib.rqrcp_cx_workspace_size(m, n, k, ctypes.byref(nb)), "rqrcp_cx_workspace_size")
    ws = workspace(nb.value, fact.a.device)
    _check(lib.rqrcp_cx(handle(), m, n, k, _ptr(fact.a), _ld(fact.a), _ptr(fact.jpvt), _ptr(x),
                        k, _ptr(ws), ws.numel()), "rqrcp_cx")
    return x


def cur_from(fc, fr, k=None):
    """U = C^+ A R^+ (k x k) from the column factorization ``fc`` of A and the
    row factorization ``fr`` of A^T (rqrcp_cur); C = A(:, fc.jpvt[:k]),
    R = A(fr.jpvt[:k], :)."""
    torch = _torch()
    k = fc.k if k is None else k
    m, n = fc.a.shape
    u = empty_colmajor(k, k, torch.float64, fc.a.device)
    lib = load_library()
    nb = ctypes.c_size_t()
    _check(lib.rqrcp_cur_workspace_size(m, n, k, fr.block, ctypes.byref(nb)),
           "rqrcp_cur_workspace_size")
    ws = workspace(nb.value, fc.a.device)
    _check(lib.rqrcp_cur(handle(), m, n, k, fr.block, _ptr(fc.a), _ld(fc.a), _ptr(fc.jpvt),
                         _ptr(fr.a), _ld(fr.a), _ptr(fr.tau), _ptr(u), k, _ptr(ws), ws.numel()),
           "rqrcp_cur")
    return u


def compress(fact, l, k):
    """Rank-k SVD compression of the l-step factorization ``fact``
    (rqrcp_compress): returns (X m x k, Y k x n, sigma) with A ~ X Y."""
    torch = _torch()
    m, n = fact.a.shape
    dev = fact.a.device
    x = empty_colmajor(m, k, torch.float64, dev)
    y = empty_colmajor(k, n, torch.float64, dev)
    sig = torch.empty(k, dtype=torch.float64, device=dev)
    lib = load_library()
    nb = ctypes.c_size_t()
    _check(lib.rqrcp_compress_workspace_size(m, n, l, k, fact.block, ctypes.byref(nb)),
           "rqrcp_compress_workspace_size")
    ws = workspace(nb.value, dev)
    _check(lib.rqrcp_compress(handle(), m, n, l, k, fact.block, _ptr(fact.a), _ld(fact.a),
                              _ptr(fact.tau), _ptr(fact.jpvt), _ptr(x), m, _ptr(y), k, _ptr(sig),
                              _ptr(ws), ws.numel()), "rqrcp_compress")
    return x, y, sig


_FN = None


def _function():
    """torch.autograd.Function over rqrcp_factor / rqrcp_form_q / rqrcp_backward."""
    global _FN
    if _FN is not None:
        return _FN
    torch = _torch()

    class RQRCPFunction(torch.autograd.Function):
        @staticmethod
        def forward(ctx, a, k, b, p, seed, jpvt, sketch_type):
            f = factor(a.detach(), k, b, p, seed, jpvt=jpvt, sketch_type=sketch_type)
            q1 = form_q(f.a, f.tau, k, b)
            r = colmajor(torch.triu(f.a[:k]))
            ctx.save_for_backward(a.detach(), f.a, f.tau, f.jpvt)
            ctx.k, ctx.b = k, b
            jp = f.jpvt.clone()
            ctx.mark_non_differentiable(jp)
            return q1, r, jp

        @staticmethod
        def backward(ctx, dq1, dr, _djp):
            a, af, tau, jp = ctx.saved_tensors
            fact = Factorization(af, jp, tau, None, None, ctx.k, ctx.b)
            da = backward(a, fact, dq1, dr)
            return da.to(a.dtype), None, None, None, None, None, None

    _FN = RQRCPFunction
    return _FN


def rqrcp(a, k, b, p, seed=0, *, jpvt=None, sketch_type="f64"):
    """Differentiable truncated RQRCP: returns (Q1, R~, jpvt) with A Pi ~ Q1 R~.

    R~ = [R11 R12] is k x n in pivot order; the gradient treats the pivots as
    fixed (they are piecewise constant in A).  Runs in the dtype of ``a``
    (float64, or float32 for the mixed-precision form).
    """
    return _function().apply(a, k, b, p, seed, jpvt, sketch_type)


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------

# numpy layout of rqrcp_problem (include/rqrcp.h)
PROBLEM_FIELDS = [("a_off", "<i8"), ("b_off", "<i8"), ("jpvt_off", "<i8"), ("tau_off", "<i8"),
                  ("m", "<i4"), ("n", "<i4"), ("k", "<i4"), ("lda", "<i4")]


@dataclass
class Batch:
    """Device pools and descriptors of a batch of column-major FP32 problems."""
    desc: object     # uint8 device tensor holding rqrcp_problem[batch]
    a: object        # float32 pool (problems back to back, lda = m)
    jpvt: object     # int32 pool
    tau: object      # float64 pool
    b: object        # float64 pool (final sketches, ld = b + p)
    info: object     # int32 (batch,)
    ws: object       # uint8 workspace
    shapes: list     # (m, n, k) per problem
    offsets: object  # numpy structured array of the descriptors
    l: int


def make_batch(shapes, l, device="cuda"):
    """Pools and descriptors for problems of the given (m, n, k) shapes."""
    import numpy as np
    torch = _torch()
    recs = np.zeros(len(shapes), dtype=np.dtype(PROBLEM_FIELDS))
    ao = bo = jo = to = 0
    for j, (m, n, k) in enumerate(shapes):
        recs[j] = (ao, bo, jo, to, m, n, k, m)
        ao += m * n
        bo += l * n
        jo += n
        to += k
    desc = torch.from_numpy(recs.view(np.uint8).copy()).to(device)
    nb = ctypes.c_size_t()
    _check(load_library().rqrcp_batched_workspace_size(ctypes.byref(nb)),
           "rqrcp_batched_workspace_size")
    return Batch(desc, torch.zeros(max(ao, 1), dtype=torch.float32, device=device),
                 torch.zeros(max(jo, 1), dtype=torch.int32, device=device),
                 torch.zeros(max(to, 1), dtype=torch.float64, device=device),
                 torch.zeros(max(bo, 1), dtype=torch.float64, device=device),
                 torch.zeros(len(shapes), dtype=torch.int32, device=device),
                 workspace(nb.value, device), list(shapes), recs, l)


def factor_batched(batch: Batch, b, p, seed=0):
    """rqrcp_factor_batched on the pools of ``batch`` (in place; no sync, no
    allocation, so it can be captured in a graph)."""
    prm = Params(b, p, seed, F32, F64, 0)
    _check(load_library().rqrcp_factor_batched(
        handle(), len(batch.shapes), _ptr(batch.desc), ctypes.byref(prm), _ptr(batch.a),
        batch.a.numel(), _ptr(batch.jpvt), batch.jpvt.numel(), _ptr(batch.tau),
        batch.tau.numel(), _ptr(batch.b), batch.b.numel(), _ptr(batch.info), _ptr(batch.ws),
        batch.ws.numel()), "rqrcp_factor_batched")


def autotune_batched(batch: Batch, a_orig, b, p, seed=0):
    """rqrcp_autotune_batched: (best variant, ms per variant); outputs are left
    holding the best variant's factorization of ``a_orig``."""
    prm = Params(b, p, seed, F32, F64, 0)
    best = ctypes.c_int()
    ms = (ctypes.c_float * 8)()
    _check(load_library().rqrcp_autotune_batched(
        handle(), len(batch.shapes), _ptr(batch.desc), ctypes.byref(prm), _ptr(batch.a),
        batch.a.numel(), _ptr(batch.jpvt), batch.jpvt.numel(), _ptr(batch.tau),
        batch.tau.numel(), _ptr(batch.b), batch.b.numel(), _ptr(batch.info), _ptr(batch.ws),
        batch.ws.numel(), _ptr(a_orig), ctypes.byref(best), ms), "rqrcp_autotune_batched")
    return best.value, [x for x in ms if x > 0.0]


def batched_limits():
    lib = load_library()
    mm, ml, mb, mx = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib.rqrcp_batched_limits(ctypes.byref(mm), ctypes.byref(ml), ctypes.byref(mb),
                             ctypes.byref(mx))
    return mm.value, ml.value, mb.value, mx.value


def set_timing(enable: bool):
    _check(load_library().rqrcp_set_timing(handle(), 1 if enable else 0), "rqrcp_set_timing")


def read_timing():
    """Per-phase totals since the last read: {phase: (ms, launches, flops, bytes)}."""
    n = len(PHASES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int * n)()
    fl = (ctypes.c_double * n)()
    by = (ctypes.c_double * n)()
    _check(load_library().rqrcp_read_timing(handle(), ms, cnt, fl, by), "rqrcp_read_timing")
    return {PHASES[i]: (ms[i], cnt[i], fl[i], by[i]) for i in range(n)}


def check(ws=None):
    _check(load_library().rqrcp_check(handle(), _ptr(ws)), "rqrcp_check")
