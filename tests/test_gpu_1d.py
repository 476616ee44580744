"""GPU parity of the 1D entry points against the FP64 oracle (relative L2 error
<= 1e-12 in complex128, <= 2e-6 in complex64 against the oracle evaluated on
the complex64-rounded inputs).  Sizes span one and several LDS tiles, ragged
(non power-of-two) lengths, the four-step range and the edge cases m = 1, 2."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu

DT = [np.complex128, np.complex64]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m", [1, 2, 3, 5, 8, 16, 17, 33, 64, 100, 255, 1024, 1500, 4096, 8192])
def test_complex_1d(dt, m):
    ic = need_gpu()
    say(f"complex1d m={m} dt={dt.__name__}")
    B = 3
    f, g = synth.unit_disk((B, m), 11), synth.unit_disk((B, m), 12)
    h = ic.conv1d_complex(to_dev(f, dt), to_dev(g, dt)).cpu().numpy()
    ref = oracle.conv1d_complex(rounded(f, dt)[:, None], rounded(g, dt)[:, None])
    for b in range(B):
        assert rel(h[b], ref[b]) < TOL[dt], (b, rel(h[b], ref[b]))


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m", [7, 64, 1000])
def test_complex_1d_mdot(dt, m):
    ic = need_gpu()
    say(f"complex1d mdot m={m}")
    B, M = 2, 3
    f, g = synth.unit_disk((B, M, m), 13), synth.unit_disk((B, M, m), 14)
    h = ic.conv1d_complex(to_dev(f, dt), to_dev(g, dt)).cpu().numpy()
    ref = oracle.conv1d_complex(rounded(f, dt), rounded(g, dt))
    assert rel(h, ref) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m", [8193, 16384, 65536, 131072])
def test_complex_1d_fourstep(dt, m):
    """Lengths past one workgroup: four-step passes, sampled oracle outputs."""
    ic = need_gpu()
    say(f"complex1d fourstep m={m} dt={dt.__name__}")
    B = 2
    f, g = synth.unit_disk((B, m), 15), synth.unit_disk((B, m), 16)
    h = ic.conv1d_complex(to_dev(f, dt), to_dev(g, dt)).cpu().numpy()
    ks = np.unique(np.concatenate([[0, 1, m // 2, m - 2, m - 1], synth.rng(17).integers(0, m, 20)]))
    for b in range(B):
        ref = oracle.convnd_complex_at(rounded(f[b], dt), rounded(g[b], dt), ks[:, None])
        assert rel(h[b][ks], ref) < TOL[dt]


def test_complex_1d_closed_form_c1():
    """Sec. 2.1 accuracy test at the m = 1024 workload: H_k = FG(k+1)e^{ik}."""
    ic = need_gpu()
    f, g, F, G = synth.closed_form_complex(1024)
    h = ic.conv1d_complex(to_dev(f, np.complex128), to_dev(g, np.complex128)).cpu().numpy()
    k = np.arange(1024)
    assert rel(h, F * G * (k + 1) * np.exp(1j * k)) < 1e-13


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 16, 31, 64, 256, 1000, 4096, 16384])
def test_hermitian_1d(dt, m):
    ic = need_gpu()
    say(f"hermitian1d m={m} dt={dt.__name__}")
    B = 2
    f = synth.power_spectrum_1d(m, 5 / 6, 21, batch=B)
    g = synth.power_spectrum_1d(m, 5 / 6, 22, batch=B)
    h = ic.conv1d_hermitian(to_dev(f, dt), to_dev(g, dt)).cpu().numpy()
    ref = oracle.conv1d_hermitian(rounded(f, dt)[:, None], rounded(g, dt)[:, None])
    for b in range(B):
        assert rel(h[b], ref[b]) < TOL[dt], (b, rel(h[b], ref[b]))


def test_hermitian_1d_closed_form_and_imag_dc():
    """Sec. 2.3 accuracy test H_k = FG(2m-1-k)e^{ik}; Im f_0 is ignored."""
    ic = need_gpu()
    m = 16384
    f, g, F, G = synth.closed_form_hermitian(m)
    f = f.copy()
    f[0] += 3j
    h = ic.conv1d_hermitian(to_dev(f, np.complex128), to_dev(g, np.complex128)).cpu().numpy()
    k = np.arange(m)
    assert rel(h, F * G * (2 * m - 1 - k) * np.exp(1j * k)) < 1e-12


@pytest.mark.parametrize("dt", DT)
def test_hermitian_1d_mdot(dt):
    ic = need_gpu()
    B, M, m = 2, 3, 300
    f = synth.unit_disk((B, M, m), 23)
    g = synth.unit_disk((B, M, m), 24)
    h = ic.conv1d_hermitian(to_dev(f, dt), to_dev(g, dt)).cpu().numpy()
    assert rel(h, oracle.conv1d_hermitian(rounded(f, dt), rounded(g, dt))) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m", [1, 2, 3, 8, 17, 64, 200])
def test_ternary_1d(dt, m):
    ic = need_gpu()
    say(f"ternary1d m={m} dt={dt.__name__}")
    f = synth.power_spectrum_1d(m, 5 / 6, 31)
    g = synth.power_spectrum_1d(m, 5 / 6, 32)
    e = synth.power_spectrum_1d(m, 5 / 6, 33)
    h = ic.conv1d_ternary(to_dev(f, dt), to_dev(g, dt), to_dev(e, dt)).cpu().numpy()
    ref = oracle.conv1d_ternary(rounded(f, dt), rounded(g, dt), rounded(e, dt))
    assert rel(h, ref) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
def test_ternary_1d_m2048_sampled(dt):
    """The m = 2048 ternary workload (batch of 4): the oracle at 64 sampled
    outputs of every convolution, and every output against the FP64 direct
    sum of the Hermitian-extended inputs (two numpy direct convolutions)."""
    ic = need_gpu()
    m, B = 2048, 4
    f = synth.power_spectrum_1d(m, 5 / 6, 34, batch=B)
    g = synth.power_spectrum_1d(m, 5 / 6, 35, batch=B)
    e = synth.power_spectrum_1d(m, 5 / 6, 36, batch=B)
    h = ic.conv1d_ternary(to_dev(f, dt), to_dev(g, dt), to_dev(e, dt)).cpu().numpy()
    rng = synth.rng(37)
    ks = np.unique(np.concatenate([[0, 1, 2, 100, 1023, 1024, 2046, 2047], rng.integers(0, m, 56)]))
    assert len(ks) >= 60
    ext = lambda u: np.concatenate([np.conj(u[:0:-1]), [u[0].real], u[1:]])  # k = -m+1 .. m-1
    for b in range(B):
        fr, gr, er = rounded(f[b], dt), rounded(g[b], dt), rounded(e[b], dt)
        ref = oracle.conv1d_ternary_at(fr, gr, er, ks)
        assert rel(h[b][ks], ref) < TOL[dt], b
        full = np.convolve(np.convolve(ext(fr), ext(gr)), ext(er))[3 * (m - 1):3 * (m - 1) + m]
        assert rel(h[b], full) < TOL[dt], b


@pytest.mark.parametrize("dt", DT)
def test_ternary_1d_m2048_closed_form(dt):
    """f_k = F e^{ik}, g_k = G e^{ik}, e_k = E e^{ik} (F, G, E real, Hermitian
    extension): h_k = F G E N(k) e^{ik} with N(k) the number of triples of
    wavenumbers in [-m+1, m-1] summing to k (an inclusion-exclusion count
    pinned by brute force on the CPU); every output at m = 2048."""
    from test_oracle_pins import ternary_count
    ic = need_gpu()
    m = 2048
    F, G, E = np.sqrt(3), np.sqrt(5), np.sqrt(7)
    k = np.arange(m)
    ph = np.exp(1j * k)
    f, g, e = F * ph, G * ph, E * ph
    h = ic.conv1d_ternary(to_dev(f, dt), to_dev(g, dt), to_dev(e, dt)).cpu().numpy()
    ref = F * G * E * np.array([ternary_count(m, int(q)) for q in k], float) * ph
    # complex64: the inputs are rounded once (relative 6e-8 per entry)
    assert rel(h, ref) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m", [1, 5, 100, 2000])
def test_explicit_complex_matches_oracle(dt, m):
    ic = need_gpu()
    f, g = synth.unit_disk((2, m), 41), synth.unit_disk((2, m), 42)
    h = ic.conv1d_complex(to_dev(f, dt), to_dev(g, dt), method="explicit").cpu().numpy()
    ref = oracle.conv1d_complex(rounded(f, dt)[:, None], rounded(g, dt)[:, None])
    assert rel(h, ref) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m", [1, 5, 100, 2000, 4096])
def test_pruned_explicit_complex_matches_oracle(dt, m):
    """EXPLICIT_PADDED | EXPLICIT_PRUNED: the size-2N cyclic convolution with
    the zero padding read rather than stored, M = 2 dot products."""
    ic = need_gpu()
    f, g = synth.unit_disk((3, 2, m), 45), synth.unit_disk((3, 2, m), 46)
    h = ic.conv1d_complex(to_dev(f, dt), to_dev(g, dt), method="pruned").cpu().numpy()
    ref = oracle.conv1d_complex(rounded(f, dt), rounded(g, dt))
    assert rel(h, ref) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m", [1, 2, 7, 300, 4000])
def test_explicit_hermitian_matches_oracle(dt, m):
    ic = need_gpu()
    f = synth.power_spectrum_1d(m, 5 / 6, 43, batch=2)
    g = synth.power_spectrum_1d(m, 5 / 6, 44, batch=2)
    h = ic.conv1d_hermitian(to_dev(f, dt), to_dev(g, dt), method="explicit").cpu().numpy()
    ref = oracle.conv1d_hermitian(rounded(f, dt)[:, None], rounded(g, dt)[:, None])
    assert rel(h, ref) < TOL[dt]


def test_determinism_and_inputs_unchanged():
    ic = need_gpu()
    import torch
    m = 3000
    f = to_dev(synth.unit_disk((4, m), 51), np.complex64)
    g = to_dev(synth.unit_disk((4, m), 52), np.complex64)
    f0, g0 = f.clone(), g.clone()
    h1 = ic.conv1d_complex(f, g)
    h2 = ic.conv1d_complex(f, g)
    torch.cuda.synchronize()
    assert torch.equal(h1, h2)
    assert torch.equal(f, f0) and torch.equal(g, g0)
