"""Work memory of the library against the paper's storage counts (Secs. 3.1,
3.2, 3.4 and 4.2, in complex words; tests/golden/paper_formulas.json).

The paper's implicit counts include the input arrays, which its routines
overwrite (the result is returned in f).  The library keeps its inputs read
only and takes separate work arrays (decoupled work memory, Sec. 1), so the
comparison is made two ways:
  * the workspace alone against the paper's implicit total, where the paper
    stores the residues over its inputs (2D);
  * workspace + inputs + output against the explicitly padded method's
    storage, which every implicit configuration must stay below (2D complex,
    3D, ternary).
The workspace queries are host-only (no GPU is touched)."""
import ctypes
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FORM = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_formulas.json")))["memory_complex_words"]
COMPLEX, HERMITIAN, TERNARY = 0, 1, 2


@pytest.fixture(scope="module")
def L():
    import paper_1008_1366_amd as ic
    if not os.path.exists(ic.LIB_PATH):
        pytest.skip("libimpconv.so not built")
    return ic.lib()


def formula(name, **v):
    return eval(FORM[name], {}, v)  # arithmetic on mx, my, mz, m only


def words(L, kind, m, n, dt=0, M=1, B=1, flags=0):
    nd = len(m)
    out = ctypes.c_size_t()
    st = L.impconv_convnd_workspace(kind, dt, nd, (ctypes.c_int64 * nd)(*m), (ctypes.c_int64 * nd)(*n), B, M,
                                    flags, ctypes.byref(out))
    assert st == 0, st
    return out.value // (16 if dt else 8)


def prod(v):
    p = 1
    for x in v:
        p *= x
    return p


@pytest.mark.parametrize("mx,my", [(64, 64), (256, 128), (2048, 2048)])
@pytest.mark.parametrize("dt", [0, 1])
def test_complex_2d(L, mx, my, dt):
    ws = words(L, COMPLEX, (mx, my), (mx, my), dt)
    assert ws <= formula("complex_2d_implicit", mx=mx, my=my)
    assert ws + 3 * mx * my <= formula("complex_2d_explicit", mx=mx, my=my)


@pytest.mark.parametrize("mx,my", [(64, 64), (256, 128), (1024, 1024)])
def test_hermitian_2d(L, mx, my):
    # storage (2mx - 1) x my: the three x residues of f and g fill exactly
    # the paper's 6 mx my words (there: f, g, U, V)
    ws = words(L, HERMITIAN, (mx, my), (2 * mx - 1, my))
    assert ws <= formula("hermitian_2d_implicit", mx=mx, my=my)


@pytest.mark.parametrize("m", [32, 64, 256])
@pytest.mark.parametrize("dt", [0, 1])
def test_complex_3d(L, m, dt):
    ws = words(L, COMPLEX, (m, m, m), (m, m, m), dt)
    data = 3 * m ** 3  # f, g, h
    assert ws + data <= formula("complex_3d_explicit", mx=m, my=m, mz=m)


@pytest.mark.parametrize("m,zs", [(32, 0), (64, 1), (256, 1), (256, 0)])
@pytest.mark.parametrize("dt", [0, 1])
def test_hermitian_3d(L, m, zs, dt):
    """Sec. 3.4: the implicit 3D centered Hermitian convolution with its
    inputs kept and a separate output stays below the explicit method's
    27 mx my mz words; with the 512 x 512 x 257 storage of the zero-slot
    convention as well."""
    n = (2 * m - 1 + zs, 2 * m - 1 + zs, m + zs)
    ws = words(L, HERMITIAN, (m, m, m), n, dt)
    data = 3 * prod(n)
    assert ws + data < formula("hermitian_3d_explicit", mx=m, my=m, mz=m)
    # the x residues of f and g take 12 m^3 (the paper's f, g, U, V); the
    # y-stage region (two sets of y residues for a quarter of the planes,
    # 2 x 1/4 x (power-of-two y size) / (y storage)) is a fraction of it
    x_res = 6 * m * prod(n[1:])
    assert x_res <= ws <= 1.3 * x_res


def test_hermitian_3d_mdot_scales_with_terms(L):
    m, n = (256,) * 3, (512, 512, 257)
    w1 = words(L, HERMITIAN, m, n, M=1)
    w3 = words(L, HERMITIAN, m, n, M=3)
    assert w3 == 3 * w1


@pytest.mark.parametrize("m", [64, 2048])
def test_ternary_1d(L, m):
    out = ctypes.c_size_t()
    assert L.impconv_conv1d_workspace(TERNARY, 0, 1, 1, m, 0, ctypes.byref(out)) == 0
    assert out.value == 0  # fused rows: no work arrays
    assert 4 * m <= formula("ternary_1d_implicit", m=m)


@pytest.mark.parametrize("mx,my", [(64, 64), (512, 256), (1024, 1024)])
def test_ternary_2d(L, mx, my):
    n = (2 * mx - 1, my)
    ws = words(L, TERNARY, (mx, my), n)
    assert ws <= formula("ternary_2d_implicit", mx=mx, my=my)
    assert ws + 4 * prod(n) <= formula("ternary_2d_explicit", mx=mx, my=my)


@pytest.mark.parametrize("m", [32, 256])
def test_complex_3d_explicit_comparator(L, m):
    """The conventional comparator's padded f and g are the paper's explicit
    3D complex storage, 16 mx my mz words (2m per axis, two arrays); its
    pruned form stores only the m data columns of the last axis."""
    EXPLICIT_PADDED, EXPLICIT_PRUNED = 1, 64
    ws = words(L, COMPLEX, (m, m, m), (m, m, m), flags=EXPLICIT_PADDED)
    assert ws == formula("complex_3d_explicit", mx=m, my=m, mz=m)
    wp = words(L, COMPLEX, (m, m, m), (m, m, m), flags=EXPLICIT_PADDED | EXPLICIT_PRUNED)
    assert wp == ws // 2
