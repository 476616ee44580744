"""libimpconv: implicitly dealiased convolutions on AMD MI355X (gfx950).

Thin Python binding over the C ABI declared in ``include/impconv.h``: every
function here only checks shapes, allocates the caller-side output and
workspace with torch (device memory), and calls the library on torch's
current HIP stream.  All arithmetic happens in the library's HIP kernels.
There is no CPU fallback: if ``libimpconv.so`` is missing or a tensor is not
on a GPU, the call raises.

Operations (Bowman & Roberts, "Efficient dealiased convolutions without
padding"):
  conv1d_complex    Sec. 2.1   h_k = sum_{p<=k} f_p g_{k-p}, k < m
  conv1d_hermitian  Sec. 2.3   centered Hermitian (2/3 rule), k = 0..m-1
  conv1d_ternary    Sec. 4     centered Hermitian ternary, k = 0..m-1
  conv2d / conv3d   Sec. 3     complex or centered Hermitian, multi-D
  RaggedPlan        uneven-length batches of complex 1D convolutions
  conv1d_complex_ad / ragged_conv_ad  differentiable wrappers (autograd)
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "lib", "available", "ImpconvError", "conv1d_complex", "conv1d_hermitian", "conv1d_ternary",
    "conv2d", "conv3d", "conv2d_noalloc", "noalloc_capacity", "RaggedPlan", "conv1d_complex_ad", "ragged_conv_ad", "workspace_bytes",
    "timing_enable", "timing_report", "schedule_cache_export", "schedule_cache_import", "schedule_cache_clear",
    "schedule_cache_save", "schedule_cache_load",
    "EXPLICIT_PADDED", "REV_F", "CONJ_G", "REV_OUT", "NO_SYMMETRIZE", "ONE_STREAM",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libimpconv.so")

EXPLICIT_PADDED, REV_F, CONJ_G, REV_OUT, NO_SYMMETRIZE, HERMITIAN_ADJOINT, EXPLICIT_PRUNED = 1, 2, 4, 8, 16, 32, 64
COMPENSATED = 128  # complex64: compensated twiddle products (complex convolutions)
ONE_STREAM = 256  # ragged batches and 3D: every launch in order on the caller's stream
COMPLEX, HERMITIAN, TERNARY = 0, 1, 2
C64, C128 = 0, 1

_lib = None
_i64 = ctypes.c_int64
_p = ctypes.c_void_p
_u32 = ctypes.c_uint32
_sz = ctypes.c_size_t


class ImpconvError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = ""
        if _lib is not None:
            msg = _lib.impconv_last_error().decode()
            kind = _lib.impconv_status_string(status).decode()
        else:
            kind = str(status)
        super().__init__(f"{where}: {kind} ({status}): {msg}")
        self.status = status


class Desc(ctypes.Structure):
    """impconv_desc of the C ABI."""
    _fields_ = [("kind", ctypes.c_int), ("dtype", ctypes.c_int), ("ndim", ctypes.c_int),
                ("m", ctypes.c_int64 * 3), ("n", ctypes.c_int64 * 3), ("batch", ctypes.c_int64),
                ("M", ctypes.c_int64), ("flags", ctypes.c_uint32)]


def lib():
    """The loaded C library (ctypes).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1008_1366_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int
        sig = {
            "impconv_version": ([], ctypes.c_int),
            "impconv_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "impconv_last_error": ([], ctypes.c_char_p),
            "impconv_init": ([], st),
            "impconv_conv1d_workspace": ([ctypes.c_int, ctypes.c_int, _i64, _i64, _i64, _u32,
                                          ctypes.POINTER(_sz)], st),
            "impconv_conv1d_complex": ([ctypes.c_int, _i64, _i64, _i64, _p, _p, _p, _p, _sz, _u32, _p], st),
            "impconv_conv1d_complex_pq": ([ctypes.c_int, _i64, _i64, _i64, _i64, _p, _p, _p, _p, _sz, _u32, _p],
                                          st),
            "impconv_conv1d_complex_pq_workspace": ([ctypes.c_int, _i64, _i64, _i64, _i64, ctypes.POINTER(_sz)],
                                                    st),
            "impconv_conv1d_complex_rule": ([ctypes.c_int, _i64, ctypes.POINTER(_i64),
                                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], st),
            "impconv_conv1d_hermitian": ([ctypes.c_int, _i64, _i64, _i64, _p, _p, _p, _p, _sz, _u32, _p], st),
            "impconv_conv1d_ternary": ([ctypes.c_int, _i64, _i64, _p, _p, _p, _p, _p, _sz, _u32, _p], st),
            "impconv_convnd_workspace": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, _p, _p, _i64, _i64,
                                          _u32, ctypes.POINTER(_sz)], st),
            "impconv_conv2d": ([ctypes.c_int, ctypes.c_int, _i64, _i64, _p, _p, _p, _p, _p, _p, _sz,
                                _u32, _p], st),
            "impconv_conv3d": ([ctypes.c_int, ctypes.c_int, _i64, _i64, _p, _p, _p, _p, _p, _p, _sz,
                                _u32, _p], st),
            "impconv_conv2d_noalloc": ([ctypes.c_int, ctypes.c_int, _i64, _i64, _p, _p, _p, _p, _p, _u32, _p],
                                       st),
            "impconv_noalloc_capacity": ([], _sz),
            "impconv_ragged_plan_create": ([ctypes.c_int, _i64, _p, _p, ctypes.POINTER(_p)], st),
            "impconv_ragged_workspace": ([_p, ctypes.POINTER(_sz)], st),
            "impconv_ragged_execute": ([_p, _p, _p, _p, _p, _sz, _u32, _p], st),
            "impconv_ragged_plan_destroy": ([_p], st),
            "impconv_ragged_plan_autotune": ([_p, _p], st),
            "impconv_plan_create": ([ctypes.POINTER(_p), ctypes.POINTER(Desc)], st),
            "impconv_conv2d_ternary": ([ctypes.c_int, _i64, _p, _p, _p, _p, _p, _p, _p, _sz, _u32, _p], st),
            "impconv_workspace_bytes": ([_p, ctypes.POINTER(_sz)], st),
            "impconv_execute": ([_p, _p, _p, _p, _p, _p, _sz, _p], st),
            "impconv_plan_destroy": ([_p], st),
            "impconv_conv1d_complex_ragged_workspace": ([ctypes.c_int, _i64, _p, _p, ctypes.POINTER(_sz)], st),
            "impconv_conv1d_complex_ragged": ([ctypes.c_int, _i64, _p, _p, _p, _p, _p, _p, _sz, _u32, _p], st),
            "impconv_ragged_plan_schedule": ([_p, ctypes.c_char_p, _sz, ctypes.POINTER(_sz)], st),
            "impconv_ragged_plan_set_fused": ([_p, ctypes.c_int, ctypes.c_int], st),
            "impconv_schedule_cache_export": ([ctypes.c_char_p, _sz, ctypes.POINTER(_sz)], st),
            "impconv_schedule_cache_import": ([ctypes.c_char_p], st),
            "impconv_schedule_cache_clear": ([], st),
            "impconv_timing_enable": ([ctypes.c_int], None),
            "impconv_timing_report": ([ctypes.c_char_p, _sz], _sz),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def available() -> bool:
    return os.path.exists(LIB_PATH) and torch.cuda.is_available()


def _check(status: int, where: str):
    if status != 0:
        raise ImpconvError(status, where)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.complex64:
        return C64
    if t.dtype == torch.complex128:
        return C128
    raise TypeError(f"expected complex64 or complex128, got {t.dtype}")


def _dev(*ts: torch.Tensor):
    d = ts[0].device
    for t in ts:
        if t.device.type != "cuda":
            raise RuntimeError("libimpconv runs on the GPU only: move the tensors to a cuda device")
        if t.device != d:
            raise RuntimeError("all tensors must be on the same device")
        if not t.is_contiguous():
            raise RuntimeError("tensors must be contiguous")
    return d


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _work(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 16), dtype=torch.uint8, device=device)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _as_bmm(f: torch.Tensor):
    """(m,) -> (1,1,m); (B,m) -> (B,1,m); (B,M,m) stays."""
    if f.dim() == 1:
        return f.view(1, 1, -1)
    if f.dim() == 2:
        return f.view(f.shape[0], 1, f.shape[1])
    if f.dim() == 3:
        return f
    raise ValueError("1D inputs must have shape (m,), (B, m) or (B, M, m)")


def workspace_bytes(kind: int, dtype: int, batch: int, M: int, m: int, flags: int = 0) -> int:
    out = _sz()
    _check(lib().impconv_conv1d_workspace(kind, dtype, batch, M, m, flags, ctypes.byref(out)),
           "impconv_conv1d_workspace")
    return out.value


def _conv1d(kind: int, f, g, method: str, flags: int):
    if f.shape != g.shape or f.dtype != g.dtype:
        raise ValueError("f and g must have the same shape and dtype")
    dev = _dev(f, g)
    F, G = _as_bmm(f), _as_bmm(g)
    B, M, m = F.shape
    dt = _dtype_code(f)
    if method == "explicit":
        flags |= EXPLICIT_PADDED
    elif method == "pruned" and kind == COMPLEX:
        flags |= EXPLICIT_PADDED | EXPLICIT_PRUNED
    elif method != "implicit":
        raise ValueError("method must be 'implicit' or 'explicit' (complex also 'pruned')")
    h = torch.empty((B, m), dtype=f.dtype, device=dev)
    wb = workspace_bytes(kind, dt, B, M, m, flags)
    w = _work(wb, dev)
    fn = lib().impconv_conv1d_complex if kind == COMPLEX else lib().impconv_conv1d_hermitian
    _check(fn(dt, B, M, m, _ptr(F), _ptr(G), _ptr(h), _ptr(w), wb, flags, ctypes.c_void_p(_stream(dev))),
           "conv1d")
    if f.dim() == 1:
        return h.view(m)
    return h


def conv1d_complex(f, g, method: str = "implicit", flags: int = 0):
    """Complex 1D dealiased convolution (Sec. 2.1) of (m,), (B, m) or (B, M, m)
    inputs (M = dot-product width); returns (m,) or (B, m).  method="explicit"
    runs the explicitly zero-padded comparator, "pruned" its form with the
    padding fused into the loads."""
    return _conv1d(COMPLEX, f, g, method, flags)


def conv1d_complex_pq(f, g, np: int, flags: int = 0):
    """Complex 1D convolution with the general p/q padding of Sec. 2.4 at
    block size np (a power of two): P = ceil(m / np) blocks, q =
    ceil((2m - 1) / np) residues of size-np transforms; np >= m is the 1/2
    rule at size np (np = 2^ceil(log2 m) above 8192: the multi-pass 1/2
    rule), np = 0 the library's automatic choice."""
    if f.shape != g.shape or f.dtype != g.dtype:
        raise ValueError("f and g must have the same shape and dtype")
    dev = _dev(f, g)
    F, G = _as_bmm(f), _as_bmm(g)
    B, M, m = F.shape
    dt = _dtype_code(f)
    h = torch.empty((B, m), dtype=f.dtype, device=dev)
    wb = _sz()
    _check(lib().impconv_conv1d_complex_pq_workspace(dt, B, M, m, int(np), ctypes.byref(wb)),
           "conv1d_complex_pq_workspace")
    w = _work(wb.value, dev)
    _check(lib().impconv_conv1d_complex_pq(dt, B, M, m, int(np), _ptr(F), _ptr(G), _ptr(h), _ptr(w), wb.value,
                                           flags, ctypes.c_void_p(_stream(dev))), "conv1d_complex_pq")
    return h.view(m) if f.dim() == 1 else h


def complex_rule(m: int, dtype=torch.complex64):
    """(np, p, q) of the rule conv1d_complex uses for length m: np = 0 is the
    1/2 rule at the power-of-two size (p = 1, q = 2)."""
    np_, p, q = _i64(), ctypes.c_int(), ctypes.c_int()
    dt = C128 if dtype == torch.complex128 else C64
    _check(lib().impconv_conv1d_complex_rule(dt, int(m), ctypes.byref(np_), ctypes.byref(p), ctypes.byref(q)),
           "conv1d_complex_rule")
    return np_.value, p.value, q.value


def conv1d_hermitian(f, g, method: str = "implicit", flags: int = 0):
    """Centered Hermitian 1D convolution (Sec. 2.3) of non-negative-wavenumber
    halves; Im f[0] and Im g[0] are ignored."""
    return _conv1d(HERMITIAN, f, g, method, flags)


def conv1d_ternary(f, g, e, method: str = "implicit"):
    """Centered Hermitian ternary convolution (Sec. 4) of (m,) or (B, m) halves;
    method="explicit" runs the explicitly zero-padded comparator."""
    flags = {"implicit": 0, "explicit": EXPLICIT_PADDED}[method]
    if not (f.shape == g.shape == e.shape) or not (f.dtype == g.dtype == e.dtype):
        raise ValueError("f, g, e must share shape and dtype")
    dev = _dev(f, g, e)
    F, G, Ev = (x.view(1, -1) if x.dim() == 1 else x for x in (f, g, e))
    B, m = F.shape
    dt = _dtype_code(f)
    h = torch.empty((B, m), dtype=f.dtype, device=dev)
    wb = workspace_bytes(TERNARY, dt, B, 1, m, flags)
    w = _work(wb, dev)
    _check(lib().impconv_conv1d_ternary(dt, B, m, _ptr(F), _ptr(G), _ptr(Ev), _ptr(h), _ptr(w), wb, flags,
                                        ctypes.c_void_p(_stream(dev))), "conv1d_ternary")
    return h.view(m) if f.dim() == 1 else h


def _convnd(nd: int, f, g, kind: str, m, flags: int):
    """nD convolution of (*n), (B, *n) or (B, M, *n) inputs."""
    if f.shape != g.shape or f.dtype != g.dtype:
        raise ValueError("f and g must have the same shape and dtype")
    dev = _dev(f, g)
    k = {"complex": COMPLEX, "hermitian": HERMITIAN}[kind]
    n = tuple(f.shape[-nd:])
    lead = f.shape[:-nd]
    if len(lead) == 0:
        B, M = 1, 1
    elif len(lead) == 1:
        B, M = lead[0], 1
    elif len(lead) == 2:
        B, M = lead
    else:
        raise ValueError("inputs must be (*n), (B, *n) or (B, M, *n)")
    if m is None:
        if k == COMPLEX:
            m = n
        else:
            raise ValueError("Hermitian nD convolutions need the logical sizes m")
    m = tuple(int(x) for x in m)
    dt = _dtype_code(f)
    marr = (ctypes.c_int64 * nd)(*m)
    narr = (ctypes.c_int64 * nd)(*n)
    out = _sz()
    _check(lib().impconv_convnd_workspace(k, dt, nd, marr, narr, B, M, flags, ctypes.byref(out)),
           "impconv_convnd_workspace")
    w = _work(out.value, dev)
    h = torch.empty((B, *n), dtype=f.dtype, device=dev)
    fn = lib().impconv_conv2d if nd == 2 else lib().impconv_conv3d
    _check(fn(k, dt, B, M, marr, narr, _ptr(f), _ptr(g), _ptr(h), _ptr(w), out.value, flags,
              ctypes.c_void_p(_stream(dev))), f"conv{nd}d")
    return h.view(*n) if len(lead) == 0 else h


def conv2d(f, g, kind: str = "complex", m=None, symmetrize: bool = True, method: str = "implicit",
           flags: int = 0):
    """2D convolution (Secs. 3.1 / 3.2); inputs (n0, n1), (B, n0, n1) or
    (B, M, n0, n1); Hermitian needs m = (m0, m1).  method="explicit" runs the
    explicitly zero-padded comparator, "pruned" its pruned form (complex
    only); flags adds ABI flags (e.g. COMPENSATED)."""
    flags |= 0 if symmetrize else NO_SYMMETRIZE
    flags |= {"implicit": 0, "explicit": EXPLICIT_PADDED, "pruned": EXPLICIT_PADDED | EXPLICIT_PRUNED}[method]
    return _convnd(2, f, g, kind, m, flags)


def conv2d_noalloc(f, g, kind: str = "complex", m=None, symmetrize: bool = True, out=None, flags: int = 0):
    """impconv_conv2d_noalloc: conv2d (implicit method) whose work arrays are
    the library's fixed per-device region instead of memory allocated here.
    Pass `out` (shape (B, n0, n1), or (n0, n1) for unbatched inputs) to
    allocate nothing at all.  impconv_init runs first on the current device."""
    flags |= 0 if symmetrize else NO_SYMMETRIZE
    k = {"complex": COMPLEX, "hermitian": HERMITIAN}[kind]
    if f.shape != g.shape or f.dtype != g.dtype:
        raise ValueError("f and g must share shape and dtype")
    dev = _dev(f, g)
    if f.dim() not in (2, 3, 4):
        raise ValueError("inputs must be (n0, n1), (B, n0, n1) or (B, M, n0, n1)")
    n = tuple(f.shape[-2:])
    B = 1 if f.dim() == 2 else f.shape[0]
    M = f.shape[1] if f.dim() == 4 else 1
    if m is None:
        if k != COMPLEX:
            raise ValueError("Hermitian 2D convolutions need the logical sizes m")
        m = n
    m = tuple(int(x) for x in m)
    h = torch.empty((B, *n), dtype=f.dtype, device=dev) if out is None else out
    if h.shape != (B, *n) and not (f.dim() == 2 and h.shape == n):
        raise ValueError(f"out must have shape {(B, *n)}")
    if h.dtype != f.dtype or h.device != dev or not h.is_contiguous():
        raise ValueError("out must be a contiguous tensor of the inputs' dtype on their device")
    with torch.cuda.device(dev):
        _check(lib().impconv_init(), "impconv_init")
        _check(lib().impconv_conv2d_noalloc(k, _dtype_code(f), B, M, (ctypes.c_int64 * 2)(*m),
                                            (ctypes.c_int64 * 2)(*n), _ptr(f), _ptr(g), _ptr(h), flags,
                                            ctypes.c_void_p(_stream(dev))), "conv2d_noalloc")
    return h.view(*n) if f.dim() == 2 and out is None else h


def noalloc_capacity() -> int:
    """Bytes of work memory impconv_conv2d_noalloc has on each device."""
    return int(lib().impconv_noalloc_capacity())


def conv2d_ternary(f, g, e, m, symmetrize: bool = True, method: str = "implicit"):
    """2D centered Hermitian ternary convolution (Sec. 4, tconv2) of inputs
    (n0, n1) or (B, n0, n1) in the 2D Hermitian storage; m = (m0, m1).
    method="explicit" runs the explicitly zero-padded comparator, "pruned"
    its form without transforms of all-zero columns."""
    if not (f.shape == g.shape == e.shape) or not (f.dtype == g.dtype == e.dtype):
        raise ValueError("f, g, e must share shape and dtype")
    dev = _dev(f, g, e)
    n = tuple(f.shape[-2:])
    B = 1 if f.dim() == 2 else f.shape[0]
    m = tuple(int(x) for x in m)
    dt = _dtype_code(f)
    flags = (0 if symmetrize else NO_SYMMETRIZE) | {"implicit": 0, "explicit": EXPLICIT_PADDED,
                                                    "pruned": EXPLICIT_PADDED | EXPLICIT_PRUNED}[method]
    marr = (ctypes.c_int64 * 2)(*m)
    narr = (ctypes.c_int64 * 2)(*n)
    out = _sz()
    _check(lib().impconv_convnd_workspace(TERNARY, dt, 2, marr, narr, B, 1, flags, ctypes.byref(out)),
           "impconv_convnd_workspace")
    w = _work(out.value, dev)
    h = torch.empty((B, *n), dtype=f.dtype, device=dev)
    _check(lib().impconv_conv2d_ternary(dt, B, marr, narr, _ptr(f), _ptr(g), _ptr(e), _ptr(h), _ptr(w), out.value,
                                        flags, ctypes.c_void_p(_stream(dev))), "conv2d_ternary")
    return h.view(*n) if f.dim() == 2 else h


def conv3d(f, g, kind: str = "complex", m=None, symmetrize: bool = True, flags: int = 0,
           method: str = "implicit"):
    """3D convolution (Sec. 3.4); inputs (n0, n1, n2), (B, ...) or (B, M, ...);
    method="explicit" runs the explicitly zero-padded comparator (centered
    Hermitian), "pruned" its form without transforms of all-zero columns."""
    flags |= {"implicit": 0, "explicit": EXPLICIT_PADDED, "pruned": EXPLICIT_PADDED | EXPLICIT_PRUNED}[method]
    return _convnd(3, f, g, kind, m, flags | (0 if symmetrize else NO_SYMMETRIZE))


def timing_enable(on: bool = True) -> None:
    """Bracket every library kernel launch with hipEvents (profiling mode)."""
    lib().impconv_timing_enable(1 if on else 0)


def timing_report() -> list:
    """Per-kernel aggregates since the last report (waits for the events)."""
    import json
    cap = 1 << 20
    buf = ctypes.create_string_buffer(cap)
    n = lib().impconv_timing_report(buf, cap)
    if n >= cap:
        raise RuntimeError("timing report truncated")
    return json.loads(buf.value.decode() or "[]")


# Ragged plans whose destruction was requested (by the garbage collector)
# while the current stream was being captured: destroying a plan waits on
# the host for its executions, which a capture must not see, so they are
# destroyed at the next plan creation or destruction outside a capture.
_deferred_plans: list = []


def _capturing() -> bool:
    try:
        return torch.cuda.is_available() and torch.cuda.is_current_stream_capturing()
    except Exception:
        return False


def _destroy_deferred() -> None:
    while _deferred_plans and not _capturing():
        _lib.impconv_ragged_plan_destroy(_deferred_plans.pop())


def schedule_cache_export() -> list:
    """Entries of the process-wide schedule cache: {"arch", "variant"
    ("fused": values per thread; "fourstep": column length N2), "dtype",
    "N", "choice", "ms"}."""
    import json
    n = _sz()
    _check(lib().impconv_schedule_cache_export(None, 0, ctypes.byref(n)), "schedule_cache_export")
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(lib().impconv_schedule_cache_export(buf, n.value + 1, ctypes.byref(n)), "schedule_cache_export")
    return json.loads(buf.value.decode())


def schedule_cache_import(entries) -> None:
    """Merges entries (the list schedule_cache_export returns, or its JSON
    text) into the process-wide schedule cache."""
    import json
    text = entries if isinstance(entries, str) else json.dumps(entries)
    _check(lib().impconv_schedule_cache_import(text.encode()), "schedule_cache_import")


def schedule_cache_clear() -> None:
    _check(lib().impconv_schedule_cache_clear(), "schedule_cache_clear")


def schedule_cache_save(path: str) -> None:
    """Writes the schedule cache to a JSON file."""
    import json
    with open(path, "w") as fh:
        json.dump(schedule_cache_export(), fh, indent=1)


def schedule_cache_load(path: str) -> None:
    """Merges a JSON file written by schedule_cache_save."""
    with open(path) as fh:
        schedule_cache_import(fh.read())


class RaggedPlan:
    """Uneven-length batch of complex 1D convolutions packed in one array:
    pair j uses elements offsets[j] .. offsets[j] + ms[j] - 1.  With
    `one_stream` set, every execution (the autograd adjoints included) runs
    the size classes one after another on the current stream (ONE_STREAM)."""

    one_stream = False

    def __init__(self, ms, offsets, dtype=torch.complex64, device=None, autotune: bool = False):
        import numpy as np
        self.ms = np.ascontiguousarray(np.asarray(ms, dtype=np.int64))
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.dtype = dtype
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.extent = int((self.ms + self.offsets).max()) if len(self.ms) else 0
        # pairs tile [0, extent) exactly: every output element is written
        order = np.argsort(self.offsets, kind="stable")
        ends = (self.offsets + self.ms)[order]
        self.dense = bool(len(self.ms) and self.offsets[order][0] == 0 and np.all(self.offsets[order][1:] == ends[:-1]))
        dt = C64 if dtype == torch.complex64 else C128
        self._h = ctypes.c_void_p()
        lib()
        _destroy_deferred()
        with torch.cuda.device(self.device):
            _check(lib().impconv_ragged_plan_create(dt, len(self.ms), self.ms.ctypes.data_as(_p),
                                                    self.offsets.ctypes.data_as(_p), ctypes.byref(self._h)),
                   "impconv_ragged_plan_create")
        out = _sz()
        _check(lib().impconv_ragged_workspace(self._h, ctypes.byref(out)), "impconv_ragged_workspace")
        self.work_bytes = out.value
        self._work = _work(self.work_bytes, self.device)
        if autotune:
            self.autotune()

    def autotune(self):
        """Time the candidate schedules on this device and keep the fastest
        (synchronous; not under capture): every supported four-step split of
        the long size classes, both values-per-thread of every class in the
        work queue, and the queue against one launch per fused class.  Class
        choices found in the process-wide schedule cache are taken from it."""
        with torch.cuda.device(self.device):
            _check(lib().impconv_ragged_plan_autotune(self._h, ctypes.c_void_p(_stream(self.device))),
                   "impconv_ragged_plan_autotune")

    def set_fused(self, queue: bool, elems: int = 0):
        """Fix how the fused size classes run: one work-queue launch (queue =
        True) or one launch per class, with `elems` values per thread in the
        queue for every class that supports it (0: the row kernels' choice).
        Synchronous; not under capture."""
        with torch.cuda.device(self.device):
            _check(lib().impconv_ragged_plan_set_fused(self._h, int(bool(queue)), int(elems)),
                   "impconv_ragged_plan_set_fused")

    def schedule_info(self) -> dict:
        """The plan's schedule: how the fused classes launch ("queue": one
        persistent work-queue launch, or "per-class"), the queue's grid, the
        autotuner's times of both, and per size class N, pair count, method
        ("queue", "fused" or "four-step"), stream, values per thread E or
        split N1 x N2, where the choice came from ("default", "timed",
        "cache") and the autotuner's times per candidate."""
        import json
        n = _sz()
        _check(lib().impconv_ragged_plan_schedule(self._h, None, 0, ctypes.byref(n)), "schedule")
        buf = ctypes.create_string_buffer(n.value + 1)
        _check(lib().impconv_ragged_plan_schedule(self._h, buf, n.value + 1, ctypes.byref(n)), "schedule")
        return json.loads(buf.value.decode())

    def schedule(self) -> list:
        """Per size class entries of schedule_info()."""
        return self.schedule_info()["classes"]

    def execute(self, f, g, flags: int = 0, out=None, work=None):
        _dev(f, g)
        if f.dtype != self.dtype or g.dtype != self.dtype:
            raise TypeError("dtype differs from the plan's")
        if f.numel() < self.extent or g.numel() < self.extent:
            raise ValueError("packed inputs shorter than the plan's extent")
        if out is not None:
            h = out
        elif self.dense:
            h = torch.empty_like(f)
            if f.numel() > self.extent:
                h.view(-1)[self.extent:].zero_()
        else:
            h = torch.zeros_like(f)
        w = self._work if work is None else work
        if self.one_stream:
            flags |= ONE_STREAM
        _check(lib().impconv_ragged_execute(self._h, _ptr(f), _ptr(g), _ptr(h), _ptr(w), self.work_bytes,
                                            flags, ctypes.c_void_p(_stream(f.device))), "ragged_execute")
        return h

    def __del__(self):
        try:
            if self._h and _lib is not None:
                if _capturing():
                    _deferred_plans.append(self._h)
                else:
                    _lib.impconv_ragged_plan_destroy(self._h)
                    _destroy_deferred()
        except Exception:
            pass


class Plan:
    """Descriptor-based plan (impconv_plan_create / impconv_execute): kind in
    {"complex", "hermitian", "ternary"}, logical sizes m per axis, storage
    extents n (2D/3D; default m for complex), batch, dot-product width M."""

    def __init__(self, kind: str, dtype, m, n=None, batch: int = 1, M: int = 1, flags: int = 0, device=None):
        m = tuple(int(x) for x in (m if hasattr(m, "__len__") else (m,)))
        nd = len(m)
        n = tuple(int(x) for x in (n if n is not None else m))
        self.kind = {"complex": COMPLEX, "hermitian": HERMITIAN, "ternary": TERNARY}[kind]
        self.dtype = dtype
        self.m, self.n, self.batch, self.M = m, n, int(batch), int(M)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        d = Desc(self.kind, C64 if dtype == torch.complex64 else C128, nd, (ctypes.c_int64 * 3)(*m),
                 (ctypes.c_int64 * 3)(*n), self.batch, self.M, flags)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().impconv_plan_create(ctypes.byref(self._h), ctypes.byref(d)), "impconv_plan_create")
        out = _sz()
        _check(lib().impconv_workspace_bytes(self._h, ctypes.byref(out)), "impconv_workspace_bytes")
        self.work_bytes = out.value

    def execute(self, f, g, e=None, out=None, work=None):
        _dev(*(x for x in (f, g, e) if x is not None))
        oshape = (self.batch, *self.n) if len(self.m) > 1 else (self.batch, self.m[0])
        h = torch.empty(oshape, dtype=self.dtype, device=f.device) if out is None else out
        w = _work(self.work_bytes, f.device) if work is None else work
        _check(lib().impconv_execute(self._h, _ptr(f), _ptr(g), _ptr(e) if e is not None else None, _ptr(h),
                                     _ptr(w), self.work_bytes, ctypes.c_void_p(_stream(f.device))), "impconv_execute")
        return h

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.impconv_plan_destroy(self._h)
        except Exception:
            pass


def conv1d_complex_ragged(f, g, ms=None, offsets=None, flags: int = 0):
    """One-shot ragged batch (impconv_conv1d_complex_ragged; the library
    caches the plan of each layout).  Packed form: f, g 1D tensors holding
    pair j at offsets[j] .. offsets[j] + ms[j] - 1; returns the packed h.
    List form: f, g equal-length sequences of 1D tensors (pair j = f[j],
    g[j], same length); they are packed end to end and the list of the pairs'
    outputs is returned."""
    import numpy as np
    if isinstance(f, (list, tuple)):
        if not isinstance(g, (list, tuple)) or len(f) != len(g):
            raise ValueError("list form: f and g must be sequences of the same length")
        if ms is not None or offsets is not None:
            raise ValueError("list form: lengths and offsets come from the tensors")
        if len(f) == 0:
            return []
        lens = [int(a.numel()) for a in f]
        if any(int(b.numel()) != n for b, n in zip(g, lens)) or min(lens) < 1:
            raise ValueError("list form: f[j] and g[j] must have the same length >= 1")
        hp = conv1d_complex_ragged(torch.cat([a.reshape(-1) for a in f]), torch.cat([b.reshape(-1) for b in g]),
                                   lens, np.concatenate([[0], np.cumsum(lens)[:-1]]), flags)
        return list(torch.split(hp, lens))
    _dev(f, g)
    ms = np.ascontiguousarray(np.asarray(ms, dtype=np.int64))
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    dt = _dtype_code(f)
    out = _sz()
    _check(lib().impconv_conv1d_complex_ragged_workspace(dt, len(ms), ms.ctypes.data_as(_p), offs.ctypes.data_as(_p),
                                                          ctypes.byref(out)), "ragged workspace")
    w = _work(out.value, f.device)
    h = torch.zeros_like(f)
    _check(lib().impconv_conv1d_complex_ragged(dt, len(ms), ms.ctypes.data_as(_p), offs.ctypes.data_as(_p),
                                               _ptr(f), _ptr(g), _ptr(h), _ptr(w), out.value, flags,
                                               ctypes.c_void_p(_stream(f.device))), "conv1d_complex_ragged")
    return h


# ---------------------------------------------------------------- autograd
# For h = f * g (complex 1D, Sec. 2.1 sum) and a real loss L with
# gh = dL/dRe h + i dL/dIm h (torch's convention), the vector-Jacobian
# products are correlations:
#   grad_f[p] = sum_{k>=p} gh_k conj(g_{k-p}) = REV(conv(REV(gh), conj g))_p
# and symmetrically for g; the library evaluates them with the REV_F,
# CONJ_G and REV_OUT load/store flags.

class _Conv1dComplexFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, g):
        ctx.save_for_backward(f, g)
        return conv1d_complex(f, g)

    @staticmethod
    def backward(ctx, gh):
        f, g = ctx.saved_tensors
        gh = gh.contiguous()
        gf = gg = None
        shape = f.shape
        F, G = _as_bmm(f), _as_bmm(g)
        GH = gh.reshape(F.shape[0], 1, F.shape[2]).expand(-1, F.shape[1], -1).contiguous()
        fl = REV_F | CONJ_G | REV_OUT
        if ctx.needs_input_grad[0]:
            gf = torch.stack([conv1d_complex(GH[:, i].contiguous(), G[:, i].contiguous(), flags=fl)
                              for i in range(F.shape[1])], 1).reshape(shape)
        if ctx.needs_input_grad[1]:
            gg = torch.stack([conv1d_complex(GH[:, i].contiguous(), F[:, i].contiguous(), flags=fl)
                              for i in range(F.shape[1])], 1).reshape(shape)
        return gf, gg


def conv1d_complex_ad(f, g):
    """Differentiable conv1d_complex (hand-written adjoint, no autograd tape
    through the kernels)."""
    return _Conv1dComplexFn.apply(f, g)


def _per_term(fn, gh, F, G, flags):
    """Vector-Jacobian products of an M-term dot product h = sum_i f_i * g_i:
    grad f_i = fn(gh, g_i, flags) for each i (the upstream gradient gh is
    shared by the terms).  F, G: (B, M, ...); returns (B, M, ...)."""
    return torch.stack([fn(gh, G[:, i].contiguous(), flags) for i in range(F.shape[1])], 1)


class _Conv1dHermitianFn(torch.autograd.Function):
    # For the centered Hermitian sum (Sec. 2.3) the stored halves define the
    # full fields through f_{-p} = conj f_p, with Im f_0 ignored.  For a real
    # loss L and gh = dL/dRe h + i dL/dIm h (k = 0..m-1) the gradient with
    # respect to the stored half of f is the Hermitian convolution of gh',
    # the Hermitian extension of gh with gh'_0 = 2 Re gh_0, with g, entry 0
    # halved and real (the HERMITIAN_ADJOINT flag applies both edits in the
    # kernel); symmetrically for g.
    @staticmethod
    def forward(ctx, f, g):
        ctx.save_for_backward(f, g)
        return conv1d_hermitian(f, g)

    @staticmethod
    def backward(ctx, gh):
        f, g = ctx.saved_tensors
        F, G = _as_bmm(f), _as_bmm(g)
        GH = gh.contiguous().reshape(F.shape[0], F.shape[2])
        fn = lambda a, b, fl: conv1d_hermitian(a, b, flags=fl)
        gf = _per_term(fn, GH, F, G, HERMITIAN_ADJOINT).reshape(f.shape) if ctx.needs_input_grad[0] else None
        gg = _per_term(fn, GH, G, F, HERMITIAN_ADJOINT).reshape(g.shape) if ctx.needs_input_grad[1] else None
        return gf, gg


def conv1d_hermitian_ad(f, g):
    """Differentiable conv1d_hermitian (hand-written adjoint)."""
    return _Conv1dHermitianFn.apply(f, g)


class _ConvNdComplexFn(torch.autograd.Function):
    # nD complex sum (Secs. 3.1, 3.4): the vector-Jacobian product is the
    # correlation grad f = REV_OUT(conv(REV_F(gh), CONJ_G(g))) with every
    # reversal applied along all axes, evaluated by the same kernels through
    # their load / store flags.
    @staticmethod
    def forward(ctx, nd, f, g):
        ctx.nd = nd
        ctx.save_for_backward(f, g)
        return _convnd(nd, f, g, "complex", None, 0)

    @staticmethod
    def backward(ctx, gh):
        f, g = ctx.saved_tensors
        nd = ctx.nd
        n = f.shape[-nd:]
        lead = f.shape[:-nd]
        B = lead[0] if len(lead) >= 1 else 1
        M = lead[1] if len(lead) == 2 else 1
        F, G = f.reshape(B, M, *n), g.reshape(B, M, *n)
        GH = gh.contiguous().reshape(B, *n)
        fl = REV_F | CONJ_G | REV_OUT
        fn = lambda a, b, flags: _convnd(nd, a, b, "complex", None, flags)
        gf = _per_term(fn, GH, F, G, fl).reshape(f.shape) if ctx.needs_input_grad[1] else None
        gg = _per_term(fn, GH, G, F, fl).reshape(g.shape) if ctx.needs_input_grad[2] else None
        return None, gf, gg


def conv2d_ad(f, g):
    """Differentiable complex conv2d (hand-written adjoint)."""
    return _ConvNdComplexFn.apply(2, f, g)


def conv3d_ad(f, g):
    """Differentiable complex conv3d (hand-written adjoint)."""
    return _ConvNdComplexFn.apply(3, f, g)


class _ConvNdHermitianFn(torch.autograd.Function):
    # nD centered Hermitian sum (Secs. 3.2, 3.4) with the k_last = 0
    # hyperplane symmetrized on load.  For a real loss and gh = dL/dRe h +
    # i dL/dIm h the gradient with respect to the stored half of f is the
    # Hermitian convolution of Gamma with g, Gamma = gh with gh_k + conj gh_{-k}
    # on the hyperplane, the entries the symmetrization overwrites zero and
    # the origin halved and real (the HERMITIAN_ADJOINT flag applies the
    # load and store edits in the first and last outer passes).
    @staticmethod
    def forward(ctx, nd, m, f, g):
        ctx.nd, ctx.m = nd, m
        ctx.save_for_backward(f, g)
        return _convnd(nd, f, g, "hermitian", m, 0)

    @staticmethod
    def backward(ctx, gh):
        f, g = ctx.saved_tensors
        nd, m = ctx.nd, ctx.m
        n = f.shape[-nd:]
        lead = f.shape[:-nd]
        B = lead[0] if len(lead) >= 1 else 1
        M = lead[1] if len(lead) == 2 else 1
        F, G = f.reshape(B, M, *n), g.reshape(B, M, *n)
        GH = gh.contiguous().reshape(B, *n)
        fn = lambda a, b, flags: _convnd(nd, a, b, "hermitian", m, flags)
        gf = _per_term(fn, GH, F, G, HERMITIAN_ADJOINT).reshape(f.shape) if ctx.needs_input_grad[2] else None
        gg = _per_term(fn, GH, G, F, HERMITIAN_ADJOINT).reshape(g.shape) if ctx.needs_input_grad[3] else None
        return None, None, gf, gg


def conv2d_hermitian_ad(f, g, m):
    """Differentiable centered Hermitian conv2d (hand-written adjoint)."""
    return _ConvNdHermitianFn.apply(2, tuple(int(x) for x in m), f, g)


def conv3d_hermitian_ad(f, g, m):
    """Differentiable centered Hermitian conv3d (hand-written adjoint)."""
    return _ConvNdHermitianFn.apply(3, tuple(int(x) for x in m), f, g)


class _RaggedFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, f, g):
        ctx.plan = plan
        ctx.save_for_backward(f, g)
        return plan.execute(f, g)

    @staticmethod
    def backward(ctx, gh):
        plan = ctx.plan
        f, g = ctx.saved_tensors
        gh = gh.contiguous()
        fl = REV_F | CONJ_G | REV_OUT
        gf = plan.execute(gh, g, flags=fl) if ctx.needs_input_grad[1] else None
        gg = plan.execute(gh, f, flags=fl) if ctx.needs_input_grad[2] else None
        return None, gf, gg


def ragged_conv_ad(plan: RaggedPlan, f, g):
    """Differentiable ragged batch (forward and hand-written adjoint)."""
    return _RaggedFn.apply(plan, f, g)
