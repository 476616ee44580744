"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/impconv.h declares, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "impconv.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(impconv_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_1008_1366_amd as ic
    if not os.path.exists(ic.LIB_PATH):
        pytest.skip("libimpconv.so not built")
    return ic.lib()


def test_header_declares_entry_points():
    names = declared()
    for n in ["impconv_conv1d_complex", "impconv_conv1d_hermitian", "impconv_conv1d_ternary",
              "impconv_conv2d", "impconv_conv3d", "impconv_ragged_execute"]:
        assert n in names


def test_all_declared_symbols_exported(L):
    lib = ctypes.CDLL(L._name)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(L):
    assert L.impconv_status_string(0) == b"ok"
    assert L.impconv_status_string(3) == b"workspace too small"
    assert L.impconv_version() >= 10000


def ws(L, kind, dt, batch, M, m, flags=0):
    out = ctypes.c_size_t(123)
    st = L.impconv_conv1d_workspace(kind, dt, batch, M, m, flags, ctypes.byref(out))
    return st, out.value


def test_workspace_query_and_size_errors(L):
    assert ws(L, 0, 0, 4, 1, 1024) == (0, 0)           # fused: no workspace
    st, b = ws(L, 0, 0, 2, 1, 16384)                   # four-step: 4 residue arrays
    assert st == 0 and b == 4 * 2 * 16384 * 8
    st, b = ws(L, 0, 1, 3, 2, 100, 1)                  # explicit comparator: padded copies
    assert st == 0 and b == 3 * (2 * 2 + 1) * 256 * 16
    assert ws(L, 0, 0, 1, 1, 0)[0] == 2                # m < 1
    assert ws(L, 0, 0, -1, 1, 8)[0] == 2               # batch < 0
    assert ws(L, 0, 0, 1, 0, 8)[0] == 2                # M < 1
    assert ws(L, 0, 7, 1, 1, 8)[0] == 1                # bad dtype
    assert ws(L, 5, 0, 1, 1, 8)[0] == 1                # bad kind
    assert ws(L, 1, 0, 1, 1, 8, 2)[0] == 1             # REV flag on Hermitian
    assert ws(L, 0, 0, 1, 1, 1 << 20)[0] == 5          # beyond the four-step range
    assert ws(L, 0, 0, 1, 1, 1 << 17) == (0, 4 * (1 << 17) * 8)  # its last length
    assert ws(L, 0, 0, 1, 1, (1 << 17) + 1)[0] == 5
    assert ws(L, 1, 0, 1, 1, 16384)[0] == 0
    assert ws(L, 1, 0, 1, 1, 16385)[0] == 5
    # EXPLICIT_PRUNED: complex 1D with EXPLICIT_PADDED only; no workspace
    assert ws(L, 0, 0, 4, 2, 1000, 1 | (1 << 6)) == (0, 0)
    assert ws(L, 0, 0, 4, 2, 1000, 1)[1] > 0
    assert ws(L, 0, 0, 4, 2, 1000, 1 << 6)[0] == 1
    assert ws(L, 1, 0, 4, 2, 1000, 1 | (1 << 6))[0] == 1
    assert ws(L, 0, 0, 1, 1, 4097, 1 | (1 << 6))[0] == 5


def test_call_errors_before_launch(L):
    c = ctypes.c_void_p
    # null pointers are rejected before any device work
    assert L.impconv_conv1d_complex(0, 1, 1, 8, None, None, None, None, 0, 0, None) == 1
    # misaligned pointer
    assert L.impconv_conv1d_complex(0, 1, 1, 8, c(8), c(4099), c(1 << 20), None, 0, 0, None) == 4
    # h overlapping f other than exactly (in place is h == f with the same extent)
    assert L.impconv_conv1d_complex(0, 1, 1, 8, c(1 << 20), c(1 << 24), c((1 << 20) + 16), None, 0, 0, None) == 1
    # h == f but f is [batch][M][m] with M = 2: extents differ, rejected
    assert L.impconv_conv1d_complex(0, 1, 2, 8, c(1 << 20), c(1 << 24), c(1 << 20), None, 0, 0, None) == 1
    assert b"overlaps" in L.impconv_last_error()
    # undersized workspace (explicit comparator needs one)
    assert L.impconv_conv1d_complex(0, 1, 1, 8, c(1 << 20), c(1 << 24), c(1 << 26), c(1 << 28), 8, 1, None) == 3
    assert b"workspace" in L.impconv_last_error()


def test_nd_workspace_and_errors(L):
    m = (ctypes.c_int64 * 2)(2048, 2048)
    out = ctypes.c_size_t()
    assert L.impconv_convnd_workspace(0, 0, 2, m, m, 8, 1, 0, ctypes.byref(out)) == 0
    assert out.value == 2 * 2 * 8 * 2048 * 2048 * 8      # f and g residue arrays
    n = (ctypes.c_int64 * 2)(2048, 2047)
    assert L.impconv_convnd_workspace(0, 0, 2, m, n, 8, 1, 0, ctypes.byref(out)) == 2
    mh = (ctypes.c_int64 * 3)(256, 256, 256)
    nh = (ctypes.c_int64 * 3)(512, 512, 257)
    assert L.impconv_convnd_workspace(1, 0, 3, mh, nh, 1, 3, 0, ctypes.byref(out)) == 0
    nb = (ctypes.c_int64 * 3)(512, 511, 258)
    assert L.impconv_convnd_workspace(1, 0, 3, mh, nb, 1, 3, 0, ctypes.byref(out)) == 2
    assert L.impconv_convnd_workspace(1, 0, 4, mh, nh, 1, 3, 0, ctypes.byref(out)) == 1
    # HERMITIAN_ADJOINT: Hermitian kind only, not with NO_SYMMETRIZE
    assert L.impconv_convnd_workspace(1, 0, 3, mh, nh, 1, 1, 1 << 5, ctypes.byref(out)) == 0
    assert L.impconv_convnd_workspace(0, 0, 2, m, m, 8, 1, 1 << 5, ctypes.byref(out)) == 1
    assert L.impconv_convnd_workspace(1, 0, 3, mh, nh, 1, 1, (1 << 5) | (1 << 4), ctypes.byref(out)) == 1


def test_ragged_plan_validation(L):
    import numpy as np
    p = ctypes.c_void_p()
    ms = np.array([4, 8], np.int64)
    offs = np.array([0, 2], np.int64)  # overlapping spans
    st = L.impconv_ragged_plan_create(0, 2, ms.ctypes.data_as(ctypes.c_void_p),
                                      offs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(p))
    assert st == 1
    ms0 = np.array([0], np.int64)
    st = L.impconv_ragged_plan_create(0, 1, ms0.ctypes.data_as(ctypes.c_void_p),
                                      offs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(p))
    assert st == 2


def test_ragged_autotune_and_schedule_null_arguments(L):
    n = ctypes.c_size_t()
    assert L.impconv_ragged_plan_autotune(None, None) == 1
    assert L.impconv_ragged_plan_schedule(None, None, 0, ctypes.byref(n)) == 1


def test_ragged_set_fused_null_arguments(L):
    assert L.impconv_ragged_plan_set_fused(None, 1, 0) == 1


def test_schedule_cache_roundtrip(L):
    """The autotuner's schedule cache lives in host memory: import merges a
    JSON array, export returns every entry once, a malformed import changes
    nothing, clear empties it."""
    import json

    import paper_1008_1366_amd as ic
    ic.schedule_cache_clear()
    assert ic.schedule_cache_export() == []
    entries = [{"arch": "gfx950", "variant": "fused", "dtype": "c64", "N": 1024, "choice": 8, "ms": 0.0125},
               {"arch": "gfx950", "variant": "fourstep", "dtype": "c128", "N": 65536, "choice": 256, "ms": 1.5}]
    ic.schedule_cache_import(entries)
    got = sorted(ic.schedule_cache_export(), key=lambda e: e["N"])
    assert got == sorted(entries, key=lambda e: e["N"])
    # a later entry of the same key replaces the earlier one
    ic.schedule_cache_import(json.dumps([dict(entries[0], choice=16, ms=0.01)]))
    got = {(e["variant"], e["N"]): e["choice"] for e in ic.schedule_cache_export()}
    assert got == {("fused", 1024): 16, ("fourstep", 65536): 256}
    # malformed: an unknown variant in the second entry -> E_ARG, nothing merged
    bad = json.dumps([dict(entries[0], N=2048), dict(entries[0], variant="other")])
    assert L.impconv_schedule_cache_import(bad.encode()) == 1
    assert b"variant" in L.impconv_last_error()
    assert len(ic.schedule_cache_export()) == 2
    for broken in ('[{"arch": "gfx950", "variant": "fused", "dtype": "c64", "N": 0, "choice": 8}]',
                   '[{"arch": "gfx950", "variant": "fused", "dtype": "c32", "N": 64, "choice": 8}]',
                   '[{"arch": "gfx950", "variant": "fused", "dtype": "c64", "N": 64}]',
                   '[{"arch": "gfx950", "variant": "fused"'):
        assert L.impconv_schedule_cache_import(broken.encode()) == 1
    assert len(ic.schedule_cache_export()) == 2
    ic.schedule_cache_clear()
    assert ic.schedule_cache_export() == []


def test_plan_create_validation(L):
    """The descriptor plan rejects bad descriptors with the one-shot calls'
    codes before touching a device."""
    import paper_1008_1366_amd as ic
    p = ctypes.c_void_p()

    def create(kind=0, dtype=0, ndim=1, m=(16, 0, 0), n=(0, 0, 0), batch=1, M=1, flags=0):
        d = ic.Desc(kind, dtype, ndim, (ctypes.c_int64 * 3)(*m), (ctypes.c_int64 * 3)(*n), batch, M, flags)
        return L.impconv_plan_create(ctypes.byref(p), ctypes.byref(d))

    assert L.impconv_plan_create(ctypes.byref(p), None) == 1
    assert create(ndim=0) == 1 and create(ndim=4) == 1
    assert create(kind=7) == 1
    assert create(dtype=5) == 1
    assert create(m=(0, 0, 0)) == 2
    assert create(M=0) == 2
    assert create(batch=-1) == 2
    assert create(kind=2, ndim=3, m=(4, 4, 4), n=(8, 8, 5)) == 5  # ternary is 1D or 2D
    assert create(kind=2, ndim=2, m=(8192, 4, 0), n=(16384, 5, 0)) == 5  # ternary x axis m <= 4096
    # explicit: m0 <= 4096 in complex64, 2048 in complex128
    assert create(kind=2, dtype=1, ndim=2, m=(4096, 4, 0), n=(8192, 5, 0), flags=1) == 5
    assert create(kind=1, ndim=2, m=(4, 4, 0), n=(9, 5, 0)) == 2  # centered axis needs 2m-1 or 2m
    assert create(kind=0, ndim=2, m=(4, 4, 0), n=(4, 5, 0)) == 2  # complex storage n == m
    assert create(flags=1 << 8) == 1  # ONE_STREAM is for ragged batches only
    assert create(flags=1 << 9) == 1
    assert create(kind=0, ndim=2, m=(4, 4, 0), n=(4, 4, 0), flags=1 << 6) == 1  # PRUNED needs EXPLICIT
    n = ctypes.c_size_t()
    assert L.impconv_workspace_bytes(None, ctypes.byref(n)) == 1
    assert L.impconv_execute(None, None, None, None, None, None, 0, None) == 1
    assert L.impconv_plan_destroy(None) == 0
    assert L.impconv_conv1d_complex_ragged(0, -1, None, None, None, None, None, None, 0, 0, None) == 2
    assert L.impconv_conv1d_complex_ragged(0, 2, None, None, None, None, None, None, 0, 0, None) == 1


def test_pq_rule_and_validation(L):
    """General p/q rule (host logic only): the automatic choice and the
    block-size checks, which return before any pointer is used."""
    np_, p, q = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
    # one pass above the largest row transform (complex64): P = 3 blocks of 4096, q = 5
    assert L.impconv_conv1d_complex_rule(0, 10000, ctypes.byref(np_), ctypes.byref(p), ctypes.byref(q)) == 0
    assert (np_.value, p.value, q.value) == (4096, 3, 5)
    # complex128 at 5000: three blocks of 2048 instead of the 8192-point 1/2 rule
    assert L.impconv_conv1d_complex_rule(1, 5000, ctypes.byref(np_), ctypes.byref(p), ctypes.byref(q)) == 0
    assert (np_.value, p.value, q.value) == (2048, 3, 5)
    for m in (1024, 1100, 3000, 16384):
        assert L.impconv_conv1d_complex_rule(0, m, ctypes.byref(np_), ctypes.byref(p), ctypes.byref(q)) == 0
        assert (np_.value, p.value, q.value) == (0, 1, 2), m
    fn = L.impconv_conv1d_complex_pq
    fn.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64] + \
        [ctypes.c_void_p] * 4 + [ctypes.c_size_t, ctypes.c_uint32, ctypes.c_void_p]
    fn.restype = ctypes.c_int
    assert fn(0, 1, 1, 1000, 300, None, None, None, None, 0, 0, None) == 2    # not a power of two
    assert fn(0, 1, 1, 1000, 128, None, None, None, None, 0, 0, None) == 2    # P = 8
    assert fn(0, 1, 1, 12000, 8192, None, None, None, None, 0, 0, None) == 2  # block above 4096
    assert fn(1, 1, 1, 5000, 4096, None, None, None, None, 0, 0, None) == 2   # complex128: 2048 at most
    assert fn(0, 1, 1, 1000, 512, None, None, None, None, 0, 0, None) == 1    # valid rule, null pointers
    assert fn(0, 1, 1, 1000, 512, None, None, None, None, 0, 1, None) == 1    # EXPLICIT_PADDED


def test_compensated_flag_validation(L):
    """IMPCONV_COMPENSATED: implicit complex convolutions only, the 1/2 rule,
    m <= 8192 in 1D (host checks, before any device work)."""
    out = ctypes.c_size_t()
    C = 1 << 7
    assert L.impconv_conv1d_workspace(0, 0, 4, 1, 3000, C, ctypes.byref(out)) == 0
    assert L.impconv_conv1d_workspace(1, 0, 4, 1, 3000, C, ctypes.byref(out)) == 1      # Hermitian
    assert L.impconv_conv1d_workspace(0, 0, 4, 1, 3000, C | 1, ctypes.byref(out)) == 1  # explicit
    assert L.impconv_conv1d_workspace(0, 0, 4, 1, 9000, C, ctypes.byref(out)) == 5      # beyond one row pass
    m2 = (ctypes.c_int64 * 2)(64, 64)
    assert L.impconv_convnd_workspace(0, 0, 2, m2, m2, 2, 1, C, ctypes.byref(out)) == 0
    assert L.impconv_convnd_workspace(0, 0, 2, m2, m2, 2, 1, C | 1, ctypes.byref(out)) == 1
    n2 = (ctypes.c_int64 * 2)(127, 64)
    assert L.impconv_convnd_workspace(1, 0, 2, m2, n2, 2, 1, C, ctypes.byref(out)) == 1


def test_ragged_list_form_validation():
    """The Python list form checks its arguments before any device work."""
    import pytest as _pt
    import torch
    import paper_1008_1366_amd as ic
    a = [torch.zeros(3, dtype=torch.complex64), torch.zeros(2, dtype=torch.complex64)]
    assert ic.conv1d_complex_ragged([], []) == []
    with _pt.raises(ValueError):
        ic.conv1d_complex_ragged(a, a[:1])
    with _pt.raises(ValueError):
        ic.conv1d_complex_ragged(a, [a[1], a[0]])
    with _pt.raises(ValueError):
        ic.conv1d_complex_ragged(a, a, ms=[3, 2])
