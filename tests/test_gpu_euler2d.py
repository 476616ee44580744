"""The 2D incompressible Euler nonlinearity through one M = 2 Hermitian 2D
convolution (Sec. 3.3): with f = (i k_x w, i k_y w) and
g = (i k_y w / k^2, -i k_x w / k^2), the dot-product convolution equals
-sum_p (p_x k_y - p_y k_x) / |k - p|^2 w_p w_{k-p} over the dealiased box.
The reference evaluates that sum directly with numpy on the full fields."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu


def euler_inputs(m, seed):
    """Vorticity half spectrum w (storage 2m_x x (m_y+1), k_y = 0 line
    Hermitian) and the two M = 2 input stacks of the Euler term."""
    mx, my = m
    n = (2 * mx, my + 1)
    w = synth.power_spectrum_centered(m, n, 1.0, seed)
    off = n[0] - mx
    ks = np.arange(1, mx)
    w[off - ks, 0] = np.conj(w[off + ks, 0])
    kx = (np.arange(n[0]) - off)[:, None].astype(float)
    ky = np.arange(n[1])[None, :].astype(float)
    k2 = kx * kx + ky * ky
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    f = np.stack([1j * kx * w, 1j * ky * w])
    g = np.stack([1j * ky * w * inv, -1j * kx * w * inv])
    return w, f, g


def euler_direct(w, m):
    """-sum_p (p_x k_y - p_y k_x) / |k-p|^2 w_p w_{k-p}, p and k-p in the box,
    on the Hermitian-extended vorticity (numpy loops over p)."""
    W = oracle.hermitian_expand(w, m)  # full field, k at index k + m - 1
    mx, my = m
    out = np.zeros(w.shape, complex)
    off = w.shape[0] - mx
    for kx in range(-mx + 1, mx):
        for ky in range(0, my):
            s = 0
            for px in range(max(-mx + 1, kx - mx + 1), min(mx - 1, kx + mx - 1) + 1):
                for py in range(max(-my + 1, ky - my + 1), min(my - 1, ky + my - 1) + 1):
                    qx, qy = kx - px, ky - py
                    q2 = qx * qx + qy * qy
                    if q2 == 0:
                        continue
                    s += (px * ky - py * kx) / q2 * W[px + mx - 1, py + my - 1] * W[qx + mx - 1, qy + my - 1]
            out[kx + off, ky] = -s
    return out


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
def test_euler_nonlinearity_small(dt):
    ic = need_gpu()
    say(f"euler 2D {dt.__name__}")
    m = (6, 5)
    w, f, g = euler_inputs(m, 601)
    h = ic.conv2d(to_dev(f[None], dt), to_dev(g[None], dt), kind="hermitian", m=m).cpu().numpy()[0]
    ref = euler_direct(w, m)
    assert rel(h, ref) < (1e-12 if dt == np.complex128 else 2e-6)
    # the same inputs through the oracle's M = 2 sum
    assert rel(h, oracle.convnd_hermitian(rounded(f, dt), rounded(g, dt), m)) < TOL[dt]


def test_euler_nonlinearity_2048_sampled():
    """The benchmarked size: 2048 x 2048 modes (storage 4096 x 2049), M = 2,
    complex64, in the launch configuration the benchmark times; 40 outputs
    (corners, the k_y = 0 line on both sides, random interior points) vs the
    oracle's M = 2 centered Hermitian sums of the same rounded inputs."""
    ic = need_gpu()
    dt = np.complex64
    m = (2048, 2048)
    say("euler 2D 2048^2 sampled")
    w, f, g = euler_inputs(m, 602)
    h = ic.conv2d(to_dev(f[None], dt), to_dev(g[None], dt), kind="hermitian", m=m).cpu().numpy()[0]
    rng = synth.rng(603)
    pts = np.stack([rng.integers(-m[0] + 1, m[0], 32), rng.integers(0, m[1], 32)], 1)
    pts = np.concatenate([[[0, 0], [m[0] - 1, m[1] - 1], [-m[0] + 1, 0], [-m[0] + 1, m[1] - 1],
                           [5, 0], [-5, 0], [1, 1], [-1, 2047]], pts])
    ref = oracle.convnd_hermitian_at(rounded(f, dt), rounded(g, dt), m, pts)
    off = f.shape[1] - m[0]
    assert rel(h[pts[:, 0] + off, pts[:, 1]], ref) < TOL[dt]
