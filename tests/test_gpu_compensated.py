"""Compensated twiddle products (IMPCONV_COMPENSATED, complex64): parity
with the oracle, lower error than the plain FP32 products over many pairs,
no effect in complex128, and the adjoint flags through the same path."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m", [1, 2, 7, 64, 100, 1024, 1537, 4096, 8192])
def test_compensated_1d_vs_oracle(m):
    ic = need_gpu()
    say(f"compensated 1d m={m}")
    B, M = 3, 2
    f = synth.unit_disk((B, M, m), 600)
    g = synth.unit_disk((B, M, m), 601)
    h = ic.conv1d_complex(to_dev(f, np.complex64), to_dev(g, np.complex64), flags=ic.COMPENSATED).cpu().numpy()
    for b in range(B):
        ref = oracle.conv1d_complex(rounded(f[b], np.complex64), rounded(g[b], np.complex64))
        assert rel(h[b], ref) < TOL[np.complex64], b


def test_compensated_lowers_error():
    """Over 64 pairs at m = 2048 the median relative error of the compensated
    products is below that of the plain FP32 twiddles."""
    ic = need_gpu()
    B, m = 64, 2048
    f = synth.unit_disk((B, m), 602)
    g = synth.unit_disk((B, m), 603)
    F, G = to_dev(f, np.complex64), to_dev(g, np.complex64)
    hc = ic.conv1d_complex(F, G, flags=ic.COMPENSATED).cpu().numpy()
    hp = ic.conv1d_complex(F, G).cpu().numpy()
    ec, ep = [], []
    for b in range(B):
        ref = oracle.conv1d_complex(rounded(f[b], np.complex64), rounded(g[b], np.complex64))
        ec.append(rel(hc[b], ref))
        ep.append(rel(hp[b], ref))
    say(f"median rel err: compensated {np.median(ec):.3e}, plain {np.median(ep):.3e}")
    assert np.median(ec) < np.median(ep)


@pytest.mark.parametrize("shape", [(1, 1), (40, 33), (300, 257)])
def test_compensated_2d_vs_oracle(shape):
    ic = need_gpu()
    B, M = 2, 2
    f = synth.unit_disk((B, M, *shape), 604)
    g = synth.unit_disk((B, M, *shape), 605)
    h = ic.conv2d(to_dev(f, np.complex64), to_dev(g, np.complex64), flags=ic.COMPENSATED).cpu().numpy()
    for b in range(B):
        ref = oracle.convnd_complex_M(rounded(f[b], np.complex64), rounded(g[b], np.complex64))
        assert rel(h[b], ref) < TOL[np.complex64], b


def test_compensated_2d_2048_sampled():
    """2048^2, batch 2: the compensated column passes (one workgroup per tile)
    at the 2D workload's size, at sampled outputs."""
    ic = need_gpu()
    B, m = 2, 2048
    f = synth.unit_disk((B, m, m), 606)
    g = synth.unit_disk((B, m, m), 607)
    h = ic.conv2d(to_dev(f, np.complex64), to_dev(g, np.complex64), flags=ic.COMPENSATED).cpu().numpy()
    pts = np.array([[0, 0], [2047, 2047], [1000, 5], [7, 1500], [1024, 1024]])
    for b in range(B):
        ref = oracle.convnd_complex_at(rounded(f[b], np.complex64), rounded(g[b], np.complex64), pts)
        assert rel(h[b][pts[:, 0], pts[:, 1]], ref) < TOL[np.complex64], b


def test_compensated_3d_vs_oracle():
    ic = need_gpu()
    shape = (9, 10, 17)
    f = synth.unit_disk((2, *shape), 608)
    g = synth.unit_disk((2, *shape), 609)
    h = ic.conv3d(to_dev(f, np.complex64), to_dev(g, np.complex64), flags=ic.COMPENSATED).cpu().numpy()
    for b in range(2):
        ref = oracle.convnd_complex(rounded(f[b], np.complex64), rounded(g[b], np.complex64))
        assert rel(h[b], ref) < TOL[np.complex64], b


def test_compensated_no_effect_in_complex128():
    ic = need_gpu()
    f = synth.unit_disk((2, 1000), 610)
    g = synth.unit_disk((2, 1000), 611)
    F, G = to_dev(f, np.complex128), to_dev(g, np.complex128)
    a = ic.conv1d_complex(F, G, flags=ic.COMPENSATED).cpu().numpy()
    b = ic.conv1d_complex(F, G).cpu().numpy()
    assert np.array_equal(a, b)
    f2 = synth.unit_disk((1, 30, 40), 612)
    g2 = synth.unit_disk((1, 30, 40), 613)
    F2, G2 = to_dev(f2, np.complex128), to_dev(g2, np.complex128)
    assert np.array_equal(ic.conv2d(F2, G2, flags=ic.COMPENSATED).cpu().numpy(), ic.conv2d(F2, G2).cpu().numpy())


def test_compensated_adjoint_flags():
    ic = need_gpu()
    m = 777
    w = synth.unit_disk((2, m), 614)
    g = synth.unit_disk((2, m), 615)
    fl = ic.REV_F | ic.CONJ_G | ic.REV_OUT | ic.COMPENSATED
    h = ic.conv1d_complex(to_dev(w, np.complex64), to_dev(g, np.complex64), flags=fl).cpu().numpy()
    for b in range(2):
        ref = oracle.conv1d_complex(rounded(w[b], np.complex64)[::-1].copy(), np.conj(rounded(g[b], np.complex64)))[::-1]
        assert rel(h[b], ref) < TOL[np.complex64], b
    w2 = synth.unit_disk((1, 20, 30), 616)
    g2 = synth.unit_disk((1, 20, 30), 617)
    h2 = ic.conv2d(to_dev(w2, np.complex64), to_dev(g2, np.complex64), flags=fl).cpu().numpy()
    ref2 = oracle.convnd_complex(rounded(w2[0], np.complex64)[::-1, ::-1].copy(),
                                 np.conj(rounded(g2[0], np.complex64)))[::-1, ::-1]
    assert rel(h2[0], ref2) < TOL[np.complex64]
