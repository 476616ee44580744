"""FP64 CPU oracle for implicitly dealiased convolutions -- TEST INFRASTRUCTURE.

Loads ``liboracle.so`` (plain C direct sums, see ``impconv_oracle.c``) through
ctypes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import this package; the product path never does.

Every function takes and returns numpy complex128 arrays and evaluates the
plain definition of the convolution sum it names (Bowman & Roberts, Secs. 2-4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "impconv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        sig = {
            "orc_num_threads": ([], ctypes.c_int),
            "orc_set_num_threads": ([ctypes.c_int], None),
            "orc_conv1d_complex": ([_i64, _i64, _i64, _p, _p, _p], None),
            "orc_conv1d_complex_ragged": ([_i64, _p, _p, _p, _p, _p], None),
            "orc_grad_conv1d_complex": ([_i64, _p, _p, _p, _p, _p], None),
            "orc_conv1d_centered": ([_i64, _p, _p, _p], None),
            "orc_conv1d_hermitian": ([_i64, _i64, _i64, _p, _p, _p], None),
            "orc_conv1d_ternary": ([_i64, _i64, _p, _p, _p, _p], None),
            "orc_conv1d_ternary_at": ([_i64, _p, _p, _p, _i64, _p, _p], None),
            "orc_convnd_complex": ([ctypes.c_int, _p, _i64, _p, _p, _p], None),
            "orc_convnd_complex_at": ([ctypes.c_int, _p, _i64, _p, _p, _i64, _p, _p], None),
            "orc_convnd_hermitian": ([ctypes.c_int, _p, _p, _i64, ctypes.c_int, _p, _p, _p], None),
            "orc_convnd_hermitian_at": ([ctypes.c_int, _p, _p, _i64, ctypes.c_int, _p, _p, _i64,
                                         _p, _p], None),
            "orc_hermitian_expand": ([ctypes.c_int, _p, _p, ctypes.c_int, _p, _p], None),
            "orc_convnd_ternary": ([ctypes.c_int, _p, _p, ctypes.c_int, _p, _p, _p, _p], ctypes.c_int),
            "orc_convnd_ternary_at": ([ctypes.c_int, _p, _p, ctypes.c_int, _p, _p, _p, _i64, _p, _p],
                                      ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i64arr(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.int64))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    _load().orc_set_num_threads(int(n))


def conv1d_complex(f, g) -> np.ndarray:
    """Sec. 2.1 sum h_k = sum_i sum_{p<=k} f_{i,p} g_{i,k-p}, k < m.

    f, g: (..., M, m) or (m,) arrays; the M axis (dot-product width, Sec. 3.3)
    is the second to last one when f.ndim >= 2.  Returns (..., m)."""
    f, g = _c(f), _c(g)
    if f.shape != g.shape:
        raise ValueError("f and g must have equal shapes")
    if f.ndim == 1:
        f, g = f[None, None], g[None, None]
        squeeze = True
    else:
        squeeze = False
    *lead, M, m = f.shape
    batch = int(np.prod(lead)) if lead else 1
    h = np.empty((batch, m), np.complex128)
    _load().orc_conv1d_complex(m, M, batch, _ptr(f), _ptr(g), _ptr(h))
    return h[0] if squeeze else h.reshape(*lead, m)


def conv1d_complex_ragged(ms, offs, f, g) -> np.ndarray:
    f, g = _c(f), _c(g)
    ms, offs = _i64arr(ms), _i64arr(offs)
    h = np.zeros_like(f)
    _load().orc_conv1d_complex_ragged(len(ms), _ptr(ms), _ptr(offs), _ptr(f), _ptr(g), _ptr(h))
    return h


def grad_conv1d_complex(f, g, gh):
    """Adjoint of conv1d_complex (derived from the Sec. 2.1 definition)."""
    f, g, gh = _c(f), _c(g), _c(gh)
    m = f.shape[-1]
    gf, gg = np.empty_like(f), np.empty_like(f)
    _load().orc_grad_conv1d_complex(m, _ptr(f), _ptr(g), _ptr(gh), _ptr(gf), _ptr(gg))
    return gf, gg


def conv1d_centered(f, g) -> np.ndarray:
    """Sec. 2.2 centered sum over inputs of length 2m-1 (origin m-1)."""
    f, g = _c(f), _c(g)
    n = f.shape[-1]
    m = (n + 1) // 2
    h = np.empty_like(f)
    _load().orc_conv1d_centered(m, _ptr(f), _ptr(g), _ptr(h))
    return h


def conv1d_hermitian(f, g) -> np.ndarray:
    """Sec. 2.3 centered Hermitian sum, k = 0..m-1 (Im f_0 ignored).

    Same shape conventions as conv1d_complex."""
    f, g = _c(f), _c(g)
    if f.ndim == 1:
        f, g = f[None, None], g[None, None]
        squeeze = True
    else:
        squeeze = False
    *lead, M, m = f.shape
    batch = int(np.prod(lead)) if lead else 1
    h = np.empty((batch, m), np.complex128)
    _load().orc_conv1d_hermitian(m, M, batch, _ptr(f), _ptr(g), _ptr(h))
    return h[0] if squeeze else h.reshape(*lead, m)


def conv1d_ternary(f, g, e) -> np.ndarray:
    """Sec. 4 centered Hermitian ternary sum (direct O(m^3)); (..., m) inputs."""
    f, g, e = _c(f), _c(g), _c(e)
    squeeze = f.ndim == 1
    if squeeze:
        f, g, e = f[None], g[None], e[None]
    *lead, m = f.shape
    batch = int(np.prod(lead)) if lead else 1
    h = np.empty((batch, m), np.complex128)
    _load().orc_conv1d_ternary(m, batch, _ptr(f), _ptr(g), _ptr(e), _ptr(h))
    return h[0] if squeeze else h.reshape(*lead, m)


def conv1d_ternary_at(f, g, e, ks) -> np.ndarray:
    """Sec. 4 ternary sum at the output indices ks (O(m^2) per index)."""
    f, g, e = _c(f), _c(g), _c(e)
    ks = _i64arr(ks)
    out = np.empty(len(ks), np.complex128)
    _load().orc_conv1d_ternary_at(f.shape[-1], _ptr(f), _ptr(g), _ptr(e), len(ks), _ptr(ks), _ptr(out))
    return out


def convnd_complex(f, g) -> np.ndarray:
    """Secs. 3.1/3.3 complex nD sum; f, g of shape (M, *m) or (*m) with 1-3 axes."""
    f, g = _c(f), _c(g)
    return _convnd_complex(f, g, f.ndim)


def convnd_complex_M(f, g) -> np.ndarray:
    """As convnd_complex with a leading dot-product axis M (Sec. 3.3)."""
    f, g = _c(f), _c(g)
    return _convnd_complex(f, g, f.ndim - 1)


def _convnd_complex(f, g, ndim):
    m = _i64arr(f.shape[-ndim:])
    M = int(np.prod(f.shape[:-ndim])) if f.ndim > ndim else 1
    h = np.empty(tuple(m), np.complex128)
    _load().orc_convnd_complex(ndim, _ptr(m), M, _ptr(f), _ptr(g), _ptr(h))
    return h


def convnd_complex_at(f, g, pts, ndim=None) -> np.ndarray:
    """Complex nD sum at the output points pts (npts, ndim); f, g may carry a
    leading M axis when ndim is given."""
    f, g = _c(f), _c(g)
    ndim = f.ndim if ndim is None else ndim
    m = _i64arr(f.shape[-ndim:])
    M = int(np.prod(f.shape[:-ndim])) if f.ndim > ndim else 1
    pts = _i64arr(pts).reshape(-1, ndim)
    out = np.empty(len(pts), np.complex128)
    _load().orc_convnd_complex_at(ndim, _ptr(m), M, _ptr(f), _ptr(g), len(pts), _ptr(pts),
                                  _ptr(out))
    return out


def convnd_hermitian(f, g, m, symmetrize=True) -> np.ndarray:
    """Secs. 3.2/3.4 centered Hermitian nD sum in the storage layout.

    f, g: (M, *n) or (*n) storage arrays, n = extents (leading axes 2m-1 or 2m,
    last axis m or m+1); m: logical modes per axis."""
    f, g = _c(f), _c(g)
    ndim = len(m)
    n = _i64arr(f.shape[-ndim:])
    M = int(np.prod(f.shape[:-ndim])) if f.ndim > ndim else 1
    mm = _i64arr(m)
    h = np.empty(tuple(n), np.complex128)
    _load().orc_convnd_hermitian(ndim, _ptr(mm), _ptr(n), M, int(bool(symmetrize)),
                                 _ptr(f), _ptr(g), _ptr(h))
    return h


def convnd_hermitian_at(f, g, m, pts, symmetrize=True) -> np.ndarray:
    """Centered Hermitian nD sum at logical wavenumbers pts (npts, ndim)."""
    f, g = _c(f), _c(g)
    ndim = len(m)
    n = _i64arr(f.shape[-ndim:])
    M = int(np.prod(f.shape[:-ndim])) if f.ndim > ndim else 1
    mm = _i64arr(m)
    pts = _i64arr(pts).reshape(-1, ndim)
    out = np.empty(len(pts), np.complex128)
    _load().orc_convnd_hermitian_at(ndim, _ptr(mm), _ptr(n), M, int(bool(symmetrize)),
                                    _ptr(f), _ptr(g), len(pts), _ptr(pts), _ptr(out))
    return out


def convnd_ternary(f, g, e, m, symmetrize=True) -> np.ndarray:
    """Sec. 4 centered Hermitian ternary sum in nD (tconv2 for 2D), in the
    storage layout of convnd_hermitian: h_k = sum f_p g_q e_{k-p-q} over p,
    q, k-p-q in the box, k in the box with k_last >= 0."""
    f, g, e = _c(f), _c(g), _c(e)
    if not (f.shape == g.shape == e.shape):
        raise ValueError("f, g, e must have equal shapes")
    ndim = len(m)
    n = _i64arr(f.shape)
    mm = _i64arr(m)
    h = np.empty(f.shape, np.complex128)
    if _load().orc_convnd_ternary(ndim, _ptr(mm), _ptr(n), int(bool(symmetrize)), _ptr(f), _ptr(g), _ptr(e),
                                  _ptr(h)):
        raise MemoryError("oracle allocation failed")
    return h


def convnd_ternary_at(f, g, e, m, pts, symmetrize=True) -> np.ndarray:
    """convnd_ternary at logical wavenumbers pts (npts, ndim), k_last >= 0."""
    f, g, e = _c(f), _c(g), _c(e)
    ndim = len(m)
    n = _i64arr(f.shape)
    mm = _i64arr(m)
    pts = _i64arr(pts).reshape(-1, ndim)
    out = np.empty(len(pts), np.complex128)
    if _load().orc_convnd_ternary_at(ndim, _ptr(mm), _ptr(n), int(bool(symmetrize)), _ptr(f), _ptr(g),
                                     _ptr(e), len(pts), _ptr(pts), _ptr(out)):
        raise MemoryError("oracle allocation failed")
    return out


def hermitian_expand(u, m, symmetrize=True) -> np.ndarray:
    """Full centered field over prod(2m_d-1) from a stored Hermitian half."""
    u = _c(u)
    ndim = len(m)
    n = _i64arr(u.shape[-ndim:])
    mm = _i64arr(m)
    full = np.empty(tuple(2 * int(x) - 1 for x in m), np.complex128)
    _load().orc_hermitian_expand(ndim, _ptr(mm), _ptr(n), int(bool(symmetrize)), _ptr(u),
                                 _ptr(full))
    return full


def rel_l2(x, ref) -> float:
    """Normalized L2 error of Sec. 2.1: ||x - ref|| / ||ref||."""
    x = np.asarray(x, np.complex128).ravel()
    ref = np.asarray(ref, np.complex128).ravel()
    den = np.linalg.norm(ref)
    num = np.linalg.norm(x - ref)
    return float(num / den) if den > 0 else float(num)
