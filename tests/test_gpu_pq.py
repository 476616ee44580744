"""GPU parity of the general p/q padding row kernel (Sec. 2.4) against the
oracle's direct sum: forced block sizes covering P in {2, 3} and q in
{3, 4, 5, 6}, the M-dot form, the adjoint flags, the automatic choice of
conv1d_complex, and one-pass lengths above 8192."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu

CASES = [(2, 1), (3, 1), (5, 2), (9, 4), (33, 16), (100, 64), (129, 64), (150, 64), (191, 64), (300, 128),
         (520, 256), (700, 256), (1100, 512), (1537, 1024), (2500, 1024), (3000, 1024), (5000, 2048),
         (6000, 2048)]


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("m,np_", CASES)
def test_pq_forced_block(dt, m, np_):
    ic = need_gpu()
    say(f"pq m={m} np={np_} {dt.__name__}")
    B, M = 3, 2
    f = synth.unit_disk((B, M, m), 510)
    g = synth.unit_disk((B, M, m), 511)
    h = ic.conv1d_complex_pq(to_dev(f, dt), to_dev(g, dt), np_).cpu().numpy()
    for b in range(B):
        ref = oracle.conv1d_complex(rounded(f[b], dt), rounded(g[b], dt))
        assert rel(h[b], ref) < TOL[dt], b


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("m,np_", [(150, 64), (3000, 1024)])
def test_pq_adjoint_flags(dt, m, np_):
    """REV_F | CONJ_G | REV_OUT through the p/q loads and stores."""
    ic = need_gpu()
    B = 2
    w = synth.unit_disk((B, m), 512)
    g = synth.unit_disk((B, m), 513)
    fl = ic.REV_F | ic.CONJ_G | ic.REV_OUT
    h = ic.conv1d_complex_pq(to_dev(w, dt), to_dev(g, dt), np_, flags=fl).cpu().numpy()
    for b in range(B):
        ref = oracle.conv1d_complex(rounded(w[b], dt)[::-1].copy(), np.conj(rounded(g[b], dt)))[::-1]
        assert rel(h[b], ref) < TOL[dt], b


@pytest.mark.parametrize("m,dt", [(9000, np.complex64), (12288, np.complex64), (5000, np.complex128),
                                  (6000, np.complex128)])
def test_pq_auto_choice(m, dt):
    """conv1d_complex takes the p/q rule for these lengths (one pass above
    8192 in complex64; blocks of 2048 in place of the 8192-point 1/2 rule in
    complex128) and matches the direct sum."""
    ic = need_gpu()
    import torch
    np_, p, q = ic.complex_rule(m, torch.complex64 if dt == np.complex64 else torch.complex128)
    assert np_ > 0 and p >= 2 and q * np_ >= 2 * m - 1
    say(f"pq auto m={m} rule={(np_, p, q)}")
    f = synth.unit_disk((2, m), 514)
    g = synth.unit_disk((2, m), 515)
    h = ic.conv1d_complex(to_dev(f, dt), to_dev(g, dt)).cpu().numpy()
    for b in range(2):
        ref = oracle.conv1d_complex(rounded(f[b], dt), rounded(g[b], dt))
        assert rel(h[b], ref) < TOL[dt], b


def test_pq_multipass_half_rule_forced():
    """np = 2^ceil(log2 m) above 8192 forces the multi-pass 1/2 rule (with
    its workspace); same sum."""
    ic = need_gpu()
    m = 9000
    f = synth.unit_disk((2, m), 520)
    g = synth.unit_disk((2, m), 521)
    h = ic.conv1d_complex_pq(to_dev(f, np.complex64), to_dev(g, np.complex64), 16384).cpu().numpy()
    for b in range(2):
        ref = oracle.conv1d_complex(rounded(f[b], np.complex64), rounded(g[b], np.complex64))
        assert rel(h[b], ref) < TOL[np.complex64], b


def test_pq_half_rule_at_block_size():
    """np >= m runs the 1/2 rule at size np (here twice the power of two)."""
    ic = need_gpu()
    m = 300
    f = synth.unit_disk((2, m), 516)
    g = synth.unit_disk((2, m), 517)
    h = ic.conv1d_complex_pq(to_dev(f, np.complex128), to_dev(g, np.complex128), 1024).cpu().numpy()
    for b in range(2):
        assert rel(h[b], oracle.conv1d_complex(f[b], g[b])) < 1e-12


def test_pq_large_batch_ragged_tail():
    """Many rows (more blocks than CUs) at a length whose last block is
    nearly empty: m = 2 * 512 + 3, np = 512 (P = 3, q = 5)."""
    ic = need_gpu()
    m, B = 1027, 600
    f = synth.unit_disk((B, m), 518)
    g = synth.unit_disk((B, m), 519)
    h = ic.conv1d_complex_pq(to_dev(f, np.complex64), to_dev(g, np.complex64), 512).cpu().numpy()
    for b in (0, 1, 299, 599):
        ref = oracle.conv1d_complex(rounded(f[b], np.complex64), rounded(g[b], np.complex64))
        assert rel(h[b], ref) < TOL[np.complex64], b
