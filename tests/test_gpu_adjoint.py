"""GPU checks of the hand-written adjoints beyond complex 1D: the centered
Hermitian 1D, 2D and 3D convolutions (the HERMITIAN_ADJOINT load/store
edits) and the complex 2D/3D convolutions (REV_F / CONJ_G / REV_OUT along
every axis):
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


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("m", [6000, 16384])
def test_hermitian_1d_adjoint_flag_long_rows(dt, m):
    """HERMITIAN_ADJOINT on the long-row kernels (complex64: the
    register-resident kernel with two-buffer exchanges at 8192 modes;
    complex128: the staged kernel), against the oracle-evaluated adjoint."""
    ic = need_gpu()
    say(f"hermitian adjoint flag m={m} {dt.__name__}")
    w = synth.unit_disk((2, 1, m), 366)
    g = synth.unit_disk((2, 1, m), 367)
    got = ic.conv1d_hermitian(to_dev(w[:, 0], dt), to_dev(g[:, 0], dt), flags=ic.HERMITIAN_ADJOINT).cpu().numpy()
    ref = herm_adj_ref(rounded(w, dt), rounded(g, dt))
    assert rel(got, ref) < TOL[dt]
    assert np.all(got[:, 0].imag == 0)


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


def herm_storage(m, n, seed):
    u = synth.unit_disk(n, seed)
    nd = len(m)
    for d in range(nd - 1):
        if n[d] == 2 * m[d]:
            idx = [slice(None)] * nd
            idx[d] = 0
            u[tuple(idx)] = 0
    if n[-1] == m[-1] + 1:
        u[..., m[-1]] = 0
    return u


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("m,n", [((1, 1), (1, 1)), ((3, 4), (5, 4)), ((4, 3), (8, 4)), ((20, 17), (40, 18)),
                                 ((3, 2, 3), (6, 3, 4)), ((5, 6, 4), (9, 12, 5))])
def test_hermitian_nd_backward_vs_oracle(dt, m, n):
    """Centered Hermitian 2D/3D backward (HERMITIAN_ADJOINT in the outer
    passes) vs the adjoint formula evaluated with the oracle."""
    from adjoint_ref import hermitian_nd_adjoint
    ic = need_gpu()
    import torch
    say(f"hermitian nd adjoint m={m} n={n} {dt.__name__}")
    B, M = 2, 2
    f = np.stack([np.stack([herm_storage(m, n, 380 + 4 * b + i) for i in range(M)]) for b in range(B)])
    g = np.stack([np.stack([herm_storage(m, n, 390 + 4 * b + i) for i in range(M)]) for b in range(B)])
    w = synth.unit_disk((B, *n), 399)
    F = to_dev(f, dt).requires_grad_(True)
    G = to_dev(g, dt).requires_grad_(True)
    fn = ic.conv2d_hermitian_ad if len(m) == 2 else ic.conv3d_hermitian_ad
    h = fn(F, G, m)
    torch.real(torch.sum(torch.conj(to_dev(w, dt)) * h)).backward()
    for b in range(B):
        wb = rounded(w[b], dt)
        for i in range(M):
            assert rel(F.grad[b, i].cpu().numpy(), hermitian_nd_adjoint(oracle, wb, rounded(g[b, i], dt), m)) < TOL[dt]
            assert rel(G.grad[b, i].cpu().numpy(), hermitian_nd_adjoint(oracle, wb, rounded(f[b, i], dt), m)) < TOL[dt]


def test_hermitian_2d_backward_sampled():
    """m = (300, 200), storage (600, 201), complex64: sampled gradient entries
    on and off the k_y = 0 line (authoritative, overwritten and origin)."""
    from adjoint_ref import hermitian_gamma
    ic = need_gpu()
    import torch
    m, n = (300, 200), (600, 201)
    f, g = herm_storage(m, n, 401), herm_storage(m, n, 402)
    w = synth.unit_disk(n, 403)
    F = to_dev(f[None], np.complex64).requires_grad_(True)
    G = to_dev(g[None], np.complex64).requires_grad_(True)
    h = ic.conv2d_hermitian_ad(F, G, m)
    torch.real(torch.sum(torch.conj(to_dev(w[None], np.complex64)) * h)).backward()
    gf = F.grad[0].cpu().numpy()
    pts = np.array([[0, 0], [17, 0], [-17, 0], [-299, 5], [250, 199], [-3, 120], [0, 77]])
    gam = hermitian_gamma(rounded(w, np.complex64), m)
    ref = oracle.convnd_hermitian_at(gam, rounded(g, np.complex64), m, pts)
    ref[0] = ref[0].real / 2  # origin
    ref[2] = 0                # overwritten half of the k_y = 0 line
    got = gf[pts[:, 0] + n[0] - m[0], pts[:, 1]]
    assert abs(got[2]) == 0
    assert rel(got, ref) < TOL[np.complex64]


@pytest.mark.parametrize("m,n", [((2, 3), (4, 4)), ((2, 2, 2), (3, 4, 3))])
def test_hermitian_nd_gradcheck(m, n):
    ic = need_gpu()
    import torch
    f = to_dev(herm_storage(m, n, 404)[None], np.complex128).requires_grad_(True)
    g = to_dev(herm_storage(m, n, 405)[None], np.complex128).requires_grad_(True)
    fn = ic.conv2d_hermitian_ad if len(m) == 2 else ic.conv3d_hermitian_ad
    assert torch.autograd.gradcheck(lambda a, b: fn(a, b, m), (f, g), eps=1e-6, atol=1e-8)
