"""CPU check of the general p/q padding reading (Sec. 2.4) that the p/q row
kernel implements: inputs zero-extended to P blocks of np, q = ceil((2m-1)/np)
residues, x_r[s] = zeta_{q np}^{rs} sum_t zeta_q^{rt} f_{t np + s}, size-np
backward FFTs, products, forward FFTs and
q np h_{t np + s} = sum_r zeta_q^{-rt} zeta_{q np}^{-rs} V_r[s].
Written with numpy FFTs and compared with the oracle's direct sum; the
residue count one short of ceil((2m-1)/np) must alias."""
import numpy as np
import pytest

import oracle
import synth


def pq_conv(f, g, np_, q=None):
    m = len(f)
    P = -(-m // np_)
    if q is None:
        q = -(-(2 * m - 1) // np_)
    N = q * np_
    fz = np.zeros(P * np_, complex)
    gz = np.zeros(P * np_, complex)
    fz[:m], gz[:m] = f, g
    s = np.arange(np_)
    h = np.zeros(P * np_, complex)
    for r in range(q):
        zs = np.exp(2j * np.pi * r * s / N)
        zq = np.exp(2j * np.pi * r * np.arange(P) / q)
        xf = zs * (zq[:, None] * fz.reshape(P, np_)).sum(0)
        xg = zs * (zq[:, None] * gz.reshape(P, np_)).sum(0)
        # backward transforms (zeta_np = e^{+2 pi i / np}), product, forward
        W = np.fft.fft((np_ * np.fft.ifft(xf)) * (np_ * np.fft.ifft(xg)))
        h += (np.conj(zq)[:, None] * (np.conj(zs) * W)[None, :]).reshape(-1)
    return h[:m] / N


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("m,np_", [(5, 2), (6, 2), (7, 4), (9, 4), (12, 4), (13, 8), (20, 8), (24, 8), (100, 64),
                                   (300, 128), (383, 128), (384, 128), (1, 1), (3, 1)])
def test_pq_reading_matches_direct_sum(m, np_):
    f, g = synth.unit_disk(m, 500), synth.unit_disk(m, 501)
    assert rel(pq_conv(f, g, np_), oracle.conv1d_complex(f, g)) < 1e-12


@pytest.mark.parametrize("m,np_", [(9, 4), (100, 64), (300, 128)])
def test_pq_one_residue_short_aliases(m, np_):
    f, g = synth.unit_disk(m, 502), synth.unit_disk(m, 503)
    q = -(-(2 * m - 1) // np_)
    if (q - 1) * np_ >= 2 * m - 1:
        pytest.skip("q - 1 residues suffice for this m")
    assert rel(pq_conv(f, g, np_, q - 1), oracle.conv1d_complex(f, g)) > 1e-3
