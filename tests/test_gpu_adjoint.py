"""GPU checks of the hand-written adjoints beyond complex 1D: the centered
Hermitian 1D convolution (the HERMITIAN_ADJOINT load/store edits) and the
complex 2D/3D convolutions (REV_F / CONJ_G / REV_OUT along every axis):
backward vs the oracle-evaluated adjoint formulas (pinned on the CPU by
finite differences of the oracle) and vs torch.autograd.gradcheck."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu


def herm_adj_ref(w, g):
    wp = w.copy()
    wp[..., 0] = 2 * w[..., 0].real
    an = oracle.conv1d_hermitian(wp, g)
    an[..., 0] = an[..., 0].real / 2
    return an


@pytest.mark.parametrize("m", [1, 2, 7, 100, 3000])
def test_hermitian_1d_backward_vs_oracle(m):
    ic = need_gpu()
    import torch
    say(f"hermitian adjoint m={m}")
    B, M = 2, 2
    f = synth.unit_disk((B, M, m), 361)
    g = synth.unit_disk((B, M, m), 362)
    w = synth.unit_disk((B, m), 363)
    F = to_dev(f, np.complex128).requires_grad_(True)
    G = to_dev(g, np.complex128).requires_grad_(True)
    h = ic.conv1d_hermitian_ad(F, G)
    torch.real(torch.sum(torch.conj(to_dev(w, np.complex128)) * h)).backward()
    for b in range(B):
        for i in range(M):
            assert rel(F.grad[b, i].cpu().numpy(), herm_adj_ref(w[b], g[b, i])) < 1e-12
            assert rel(G.grad[b, i].cpu().numpy(), herm_adj_ref(w[b], f[b, i])) < 1e-12


def test_hermitian_1d_gradcheck():
    ic = need_gpu()
    import torch
    f = to_dev(synth.unit_disk((2, 7), 364), np.complex128).requires_grad_(True)
    g = to_dev(synth.unit_disk((2, 7), 365), np.complex128).requires_grad_(True)
    assert torch.autograd.gradcheck(ic.conv1d_hermitian_ad, (f, g), eps=1e-6, atol=1e-8)


def complex_adj_ref(w, g):
    nd = w.ndim
    rv = tuple(slice(None, None, -1) for _ in range(nd))
    return oracle.convnd_complex(w[rv].copy(), np.conj(g))[rv]


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("shape", [(1, 1), (9, 17), (40, 33), (4, 5, 6), (3, 9, 2)])
def test_complex_nd_backward_vs_oracle(dt, shape):
    ic = need_gpu()
    import torch
    say(f"complex nd adjoint {shape} {dt.__name__}")
    B, M = 2, 2
    f = synth.unit_disk((B, M, *shape), 366)
    g = synth.unit_disk((B, M, *shape), 367)
    w = synth.unit_disk((B, *shape), 368)
    F = to_dev(f, dt).requires_grad_(True)
    G = to_dev(g, dt).requires_grad_(True)
    fn = ic.conv2d_ad if len(shape) == 2 else ic.conv3d_ad
    h = fn(F, G)
    torch.real(torch.sum(torch.conj(to_dev(w, dt)) * h)).backward()
    for b in range(B):
        for i in range(M):
            assert rel(F.grad[b, i].cpu().numpy(), complex_adj_ref(rounded(w[b], dt), rounded(g[b, i], dt))) < TOL[dt]
            assert rel(G.grad[b, i].cpu().numpy(), complex_adj_ref(rounded(w[b], dt), rounded(f[b, i], dt))) < TOL[dt]


def test_complex_2d_backward_long_columns_sampled():
    """m = (1100, 700), batch 6: the outer passes run in their persistent
    form (N0 = 2048, more than two tiles per CU), whose reversed loads and
    stores are checked at sampled gradient entries."""
    ic = need_gpu()
    import torch
    B, m = 6, (1100, 700)
    f = synth.unit_disk((B, *m), 369)
    g = synth.unit_disk((B, *m), 370)
    w = synth.unit_disk((B, *m), 371)
    F = to_dev(f, np.complex64).requires_grad_(True)
    G = to_dev(g, np.complex64).requires_grad_(True)
    h = ic.conv2d_ad(F, G)
    torch.real(torch.sum(torch.conj(to_dev(w, np.complex64)) * h)).backward()
    pts = np.array([[0, 0], [m[0] - 1, m[1] - 1], [17, 650], [1000, 3], [550, 350]])
    gf = F.grad.cpu().numpy()
    for b in (0, 5):
        wr = rounded(w[b], np.complex64)[::-1, ::-1].copy()
        ref = oracle.convnd_complex_at(wr, np.conj(rounded(g[b], np.complex64)),
                                       np.stack([m[0] - 1 - pts[:, 0], m[1] - 1 - pts[:, 1]], 1))
        assert rel(gf[b][pts[:, 0], pts[:, 1]], ref) < TOL[np.complex64], b


def test_complex_2d_gradcheck():
    ic = need_gpu()
    import torch
    f = to_dev(synth.unit_disk((1, 2, 5, 6), 372), np.complex128).requires_grad_(True)
    g = to_dev(synth.unit_disk((1, 2, 5, 6), 373), np.complex128).requires_grad_(True)
    assert torch.autograd.gradcheck(ic.conv2d_ad, (f, g), eps=1e-6, atol=1e-8)
