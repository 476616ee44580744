"""Centered Hermitian 2D/3D convolutions with long outer axes (transform
sizes 1024, 2048 and 4096 in the column passes, whose blocks then hold one
workgroup per CU) at batch sizes that fill the chip: the oracle's sums at
sampled outputs, the same pair computed alone, and the Hermitian adjoint
loads at that size."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu


def herm_storage(m, n, seed):
    u = synth.unit_disk(n, seed)
    for d in range(len(m) - 1):
        if n[d] == 2 * m[d]:
            idx = [slice(None)] * len(m)
            idx[d] = 0
            u[tuple(idx)] = 0
    if n[-1] == m[-1] + 1:
        u[..., m[-1]] = 0
    return u


CASES = [
    # dtype, m, n, batch
    (np.complex64, (1000, 1200), (2000, 1201), 4),   # N = 1024
    (np.complex128, (1500, 700), (3000, 701), 2),    # N = 2048
    (np.complex64, (3000, 300), (6000, 301), 4),     # N = 4096
    (np.complex64, (600, 40, 30), (1200, 80, 31), 2),  # 3D, x pass N = 1024
]


@pytest.mark.parametrize("idx", range(len(CASES)))
def test_long_centered_axes(idx):
    ic = need_gpu()
    dt, m, n, B = CASES[idx]
    say(f"long centered axes m={m} n={n} B={B} {dt.__name__}")
    f = np.stack([herm_storage(m, n, 900 + 2 * b) for b in range(B)])
    g = np.stack([herm_storage(m, n, 901 + 2 * b) for b in range(B)])
    fn = ic.conv2d if len(m) == 2 else ic.conv3d
    h = fn(to_dev(f, dt), to_dev(g, dt), kind="hermitian", m=m).cpu().numpy()
    # the first pair alone (a grid of a quarter or half the size)
    h1 = fn(to_dev(f[:1], dt), to_dev(g[:1], dt), kind="hermitian", m=m).cpu().numpy()
    assert rel(h[0], h1[0]) < TOL[dt]
    rng = synth.rng(910 + idx)
    nd = len(m)
    pts = np.stack([rng.integers(-m[d] + 1, m[d], 12) for d in range(nd - 1)] + [rng.integers(0, m[-1], 12)], 1)
    corners = np.array([[0] * nd, [m[d] - 1 for d in range(nd)], [-(m[0] - 1)] + [0] * (nd - 1)])
    pts = np.concatenate([corners, pts])
    offs = [n[d] - m[d] for d in range(nd - 1)] + [0]
    for b in (0, B - 1):
        ref = oracle.convnd_hermitian_at(rounded(f[b], dt), rounded(g[b], dt), m, pts)
        got = h[b][tuple(pts[:, d] + offs[d] for d in range(nd))]
        assert rel(got, ref) < TOL[dt], b


def test_long_centered_axes_adjoint():
    """HERMITIAN_ADJOINT loads (U_k + conj U_-k on the k_y = 0 line) with a
    1024-point x pass: gradient entries vs the adjoint formula on the oracle."""
    from adjoint_ref import hermitian_gamma
    ic = need_gpu()
    import torch
    dt = np.complex64
    m, n, B = (1000, 1200), (2000, 1201), 4
    say("long centered axes, adjoint")
    f = np.stack([herm_storage(m, n, 920 + b) for b in range(B)])
    g = np.stack([herm_storage(m, n, 930 + b) for b in range(B)])
    w = synth.unit_disk((B, *n), 940)
    F = to_dev(f, dt).requires_grad_(True)
    G = to_dev(g, dt).requires_grad_(True)
    h = ic.conv2d_hermitian_ad(F, G, m)
    torch.real(torch.sum(torch.conj(to_dev(w, dt)) * h)).backward()
    gf = F.grad.cpu().numpy()
    pts = np.array([[0, 0], [17, 0], [-17, 0], [-999, 5], [250, 1199], [-3, 600], [0, 77], [999, 0]])
    b = B - 1
    gam = hermitian_gamma(rounded(w[b], dt), m)
    ref = oracle.convnd_hermitian_at(gam, rounded(g[b], dt), m, pts)
    ref[0] = ref[0].real / 2  # origin
    ref[2] = 0                # overwritten half of the k_y = 0 line
    got = gf[b][pts[:, 0] + n[0] - m[0], pts[:, 1]]
    assert abs(got[2]) == 0
    assert rel(got, ref) < TOL[dt]
