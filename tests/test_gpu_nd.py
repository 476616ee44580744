"""GPU parity of the 2D / 3D entry points against the FP64 oracle: full fields
on small grids spanning several tiles and ragged sizes, the 2048^2 complex
batch-of-8 workload (sampled outputs plus an exact full-field separability
check) and the 512x512x257 centered Hermitian M=3 workload (sampled)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu

DT = [np.complex128, np.complex64]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (16, 16), (33, 20), (64, 130), (200, 9)])
def test_complex_2d(dt, shape):
    ic = need_gpu()
    say(f"complex2d {shape} {dt.__name__}")
    B, M = 2, 2
    f = synth.unit_disk((B, M, *shape), 61)
    g = synth.unit_disk((B, M, *shape), 62)
    h = ic.conv2d(to_dev(f, dt), to_dev(g, dt)).cpu().numpy()
    for b in range(B):
        ref = oracle.convnd_complex_M(rounded(f[b], dt), rounded(g[b], dt))
        assert rel(h[b], ref) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("shape", [(2, 3, 4), (8, 8, 8), (5, 17, 9)])
def test_complex_3d(dt, shape):
    ic = need_gpu()
    say(f"complex3d {shape} {dt.__name__}")
    M = 2
    f = synth.unit_disk((1, M, *shape), 63)
    g = synth.unit_disk((1, M, *shape), 64)
    h = ic.conv3d(to_dev(f, dt), to_dev(g, dt)).cpu().numpy()
    ref = oracle.convnd_complex_M(rounded(f[0], dt), rounded(g[0], dt))
    assert rel(h[0], ref) < TOL[dt]


def herm_input(m, n, seed, M=None):
    shape = n if M is None else (M, *n)
    u = synth.unit_disk(shape, seed)
    return u


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m,n", [((1, 1), (1, 1)), ((2, 2), (4, 3)), ((5, 6), (9, 6)),
                                 ((16, 16), (32, 17)), ((17, 40), (33, 41)), ((40, 7), (80, 7))])
def test_hermitian_2d(dt, m, n):
    ic = need_gpu()
    say(f"hermitian2d m={m} n={n} {dt.__name__}")
    M = 2
    f, g = herm_input(m, n, 65, M), herm_input(m, n, 66, M)
    h = ic.conv2d(to_dev(f[None], dt), to_dev(g[None], dt), kind="hermitian", m=m).cpu().numpy()[0]
    ref = oracle.convnd_hermitian(rounded(f, dt), rounded(g, dt), m)
    assert rel(h, ref) < TOL[dt]
    # zero slots are written as exact zeros
    if n[0] == 2 * m[0]:
        assert np.all(h[0] == 0)
    if n[1] == m[1] + 1:
        assert np.all(h[:, m[1]] == 0)


def test_hermitian_2d_no_symmetrize_projection():
    ic = need_gpu()
    m, n = (9, 8), (17, 9)
    f, g = herm_input(m, n, 67), herm_input(m, n, 68)
    h = ic.conv2d(to_dev(f, np.complex128), to_dev(g, np.complex128), kind="hermitian", m=m,
                  symmetrize=False).cpu().numpy()
    ref = oracle.convnd_hermitian(f, g, m, symmetrize=False)
    assert rel(h, ref) < 1e-12


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m,n", [((2, 2, 2), (4, 4, 3)), ((4, 3, 5), (7, 6, 5)), ((8, 8, 8), (16, 16, 9)),
                                 ((5, 9, 6), (10, 17, 7))])
def test_hermitian_3d(dt, m, n):
    ic = need_gpu()
    say(f"hermitian3d m={m} n={n} {dt.__name__}")
    M = 3
    f, g = herm_input(m, n, 69, M), herm_input(m, n, 70, M)
    h = ic.conv3d(to_dev(f[None], dt), to_dev(g[None], dt), kind="hermitian", m=m).cpu().numpy()[0]
    ref = oracle.convnd_hermitian(rounded(f, dt), rounded(g, dt), m)
    assert rel(h, ref) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
def test_complex_2d_c3_workload(dt):
    """2048^2, batch of 8 independent pairs in one call; (1+|k|^2)^-1 Gaussian
    spectra; sampled outputs vs the oracle, plus one rank-1 pair checked on
    the full field against outer products of 1D oracle results."""
    ic = need_gpu()
    say(f"complex2d C3 {dt.__name__}")
    mx = my = 2048
    B = 8
    f = np.stack([synth.gaussian_2d(mx, my, 100 + 2 * b) for b in range(B)])
    g = np.stack([synth.gaussian_2d(mx, my, 101 + 2 * b) for b in range(B)])
    a, bb, c, d = (synth.unit_disk(2048, s) for s in (90, 91, 92, 93))
    f[B - 1] = np.outer(a, bb)
    g[B - 1] = np.outer(c, d)
    h = ic.conv2d(to_dev(f, dt), to_dev(g, dt)).cpu().numpy()
    rng = synth.rng(5)
    pts = np.concatenate([[[0, 0], [mx - 1, my - 1], [1, 2047], [2047, 0]], rng.integers(0, mx, (12, 2))])
    for b in range(0, B - 1, 3):
        ref = oracle.convnd_complex_at(rounded(f[b], dt), rounded(g[b], dt), pts)
        assert rel(h[b][pts[:, 0], pts[:, 1]], ref) < TOL[dt], b
    # every output of the rank-one pair; in complex64 the products a b and
    # c d are rounded once on input (relative 6e-8 per entry), which the FP32
    # tolerance covers
    full = np.outer(oracle.conv1d_complex(a, c), oracle.conv1d_complex(bb, d))
    assert rel(h[B - 1], full) < TOL[dt]
    ref = oracle.convnd_complex_at(rounded(f[B - 1], dt), rounded(g[B - 1], dt), pts)
    assert rel(h[B - 1][pts[:, 0], pts[:, 1]], ref) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
def test_complex_2d_long_columns_ragged(dt):
    """Long outer axis (m0 = 1500 -> N0 = 2048, the persistent column-pass
    form), ragged inner axis (700 columns: a partial last tile), M = 2,
    enough tiles that workgroups walk uneven tile sequences.  Sampled outputs
    vs the oracle; pair 0 is rank one and checked on the full field against
    outer products of 1D oracle results."""
    ic = need_gpu()
    say(f"complex2d long columns {dt.__name__}")
    B, M, m0, m1 = 3, 2, 1500, 700
    f = synth.unit_disk((B, M, m0, m1), 71)
    g = synth.unit_disk((B, M, m0, m1), 72)
    vec = [synth.unit_disk(n, s) for n, s in ((m0, 73), (m1, 74), (m0, 75), (m1, 76))]
    for i in range(M):
        f[0, i] = np.outer(vec[0], vec[1]) * (i + 1)
        g[0, i] = np.outer(vec[2], vec[3])
    h = ic.conv2d(to_dev(f, dt), to_dev(g, dt)).cpu().numpy()
    rng = synth.rng(77)
    pts = np.concatenate([[[0, 0], [m0 - 1, m1 - 1], [m0 - 1, 0], [0, m1 - 1], [1024, 696]],
                          np.stack([rng.integers(0, m0, 8), rng.integers(0, m1, 8)], 1)])
    for b in range(1, B):
        ref = sum(oracle.convnd_complex_at(rounded(f[b, i], dt), rounded(g[b, i], dt), pts) for i in range(M))
        assert rel(h[b][pts[:, 0], pts[:, 1]], ref) < TOL[dt], b
    va, vb, vc, vd = vec
    full = sum((i + 1) for i in range(M)) * np.outer(oracle.conv1d_complex(va, vc), oracle.conv1d_complex(vb, vd))
    assert rel(h[0], full) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
def test_hermitian_3d_c4_workload(dt):
    """512 x 512 x 257 storage (m = 256 per axis, zero slots), M = 3 pairs,
    |k|^-11/6 random-phase spectra; sampled outputs vs the oracle."""
    ic = need_gpu()
    say(f"hermitian3d C4 {dt.__name__}")
    m, n = (256, 256, 256), (512, 512, 257)
    f = np.stack([synth.power_spectrum_centered(m, n, 11 / 6, 200 + i) for i in range(3)])
    g = np.stack([synth.power_spectrum_centered(m, n, 11 / 6, 203 + i) for i in range(3)])
    h = ic.conv3d(to_dev(f[None], dt), to_dev(g[None], dt), kind="hermitian", m=m).cpu().numpy()[0]
    pts = np.array([[0, 0, 0], [255, 255, 255], [-255, 0, 3], [5, -7, 0], [-3, -250, 128], [100, 100, 200]])
    ref = oracle.convnd_hermitian_at(rounded(f, dt), rounded(g, dt), m, pts)
    got = h[pts[:, 0] + 256, pts[:, 1] + 256, pts[:, 2]]
    assert rel(got, ref) < TOL[dt]
    assert np.all(h[0] == 0) and np.all(h[:, 0] == 0) and np.all(h[:, :, 256] == 0)


def _herm_full_1d(m, seed):
    """A Hermitian-symmetric centered 1D field, wavenumbers -m+1..m-1."""
    a = synth.power_spectrum_1d(m, 11 / 6, seed)
    return np.concatenate([np.conj(a[:0:-1]), [a[0].real], a[1:]])


@pytest.mark.parametrize("dt", DT)
def test_hermitian_3d_c4_separable_full_field(dt):
    """Every output of the 512 x 512 x 257 (m = 256 per axis), M = 3
    workload on separable inputs: pair i is f_i = A_i (x) B_i (x) c_i with
    A, B Hermitian centered fields along x and y and c a Hermitian half along
    z (c_0 real), so the k_z = 0 plane is already symmetric and the sum
    factors, per pair, into the full centered 1D sums along x and y and the
    centered Hermitian 1D sum along z (Sec. 3.4 builds the 3D convolution from
    these axes).  Reference: sum over i of outer products of the 1D oracle
    results, compared on the whole stored field (zero slots included)."""
    ic = need_gpu()
    say(f"hermitian3d C4 separable full field {dt.__name__}")
    m, n = 256, (512, 512, 257)
    f = np.zeros((3, *n), complex)
    g = np.zeros((3, *n), complex)
    ref = np.zeros(n, complex)
    for i in range(3):
        A, B, A2, B2 = (_herm_full_1d(m, 400 + 10 * i + j) for j in range(4))
        c, c2 = (synth.power_spectrum_1d(m, 11 / 6, 450 + 10 * i + j) for j in range(2))
        c[0], c2[0] = c[0].real, c2[0].real
        f[i, 1:, 1:, :m] = np.einsum("x,y,z->xyz", A, B, c)
        g[i, 1:, 1:, :m] = np.einsum("x,y,z->xyz", A2, B2, c2)
        ref[1:, 1:, :m] += np.einsum("x,y,z->xyz", oracle.conv1d_centered(A, A2),
                                     oracle.conv1d_centered(B, B2), oracle.conv1d_hermitian(c, c2))
    h = ic.conv3d(to_dev(f[None], dt), to_dev(g[None], dt), kind="hermitian", m=(m, m, m)).cpu().numpy()[0]
    # complex64: the products A B c are rounded once on input (relative 6e-8
    # per entry); the FP32 tolerance covers it
    assert rel(h, ref) < TOL[dt]
    assert np.all(h[0] == 0) and np.all(h[:, 0] == 0) and np.all(h[:, :, m] == 0)


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("shape", [(1, 1), (5, 7), (33, 64), (100, 3)])
def test_explicit_complex_2d_matches_oracle(dt, shape):
    ic = need_gpu()
    B, M = 2, 2
    f = synth.unit_disk((B, M, *shape), 81)
    g = synth.unit_disk((B, M, *shape), 82)
    h = ic.conv2d(to_dev(f, dt), to_dev(g, dt), method="explicit").cpu().numpy()
    for b in range(B):
        assert rel(h[b], oracle.convnd_complex_M(rounded(f[b], dt), rounded(g[b], dt))) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("shape", [(1, 1), (5, 7), (33, 64), (100, 3)])
def test_pruned_complex_2d_matches_oracle(dt, shape):
    ic = need_gpu()
    B, M = 2, 2
    f = synth.unit_disk((B, M, *shape), 83)
    g = synth.unit_disk((B, M, *shape), 84)
    h = ic.conv2d(to_dev(f, dt), to_dev(g, dt), method="pruned").cpu().numpy()
    for b in range(B):
        assert rel(h[b], oracle.convnd_complex_M(rounded(f[b], dt), rounded(g[b], dt))) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("method", ["explicit", "pruned"])
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 4), (8, 8, 8), (5, 17, 9), (20, 3, 33)])
def test_explicit_complex_3d_matches_oracle(dt, method, shape):
    """The conventional 3D complex comparator (padding to 2N per axis, full
    transforms on every axis; pruned: padding fused into the loads, no
    transform of an all-zero column) gives the dealiased sum."""
    ic = need_gpu()
    say(f"explicit complex3d {method} {shape} {dt.__name__}")
    B, M = 2, 2
    f = synth.unit_disk((B, M, *shape), 85)
    g = synth.unit_disk((B, M, *shape), 86)
    F, G = to_dev(f, dt), to_dev(g, dt)
    h = ic.conv3d(F, G, method=method).cpu().numpy()
    for b in range(B):
        assert rel(h[b], oracle.convnd_complex_M(rounded(f[b], dt), rounded(g[b], dt))) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("kind", ["hermitian", "complex"])
def test_3d_overlapped_chunks_equal_one_stream(dt, kind):
    """3D: the rows and y forward pass of one chunk of planes run on an
    auxiliary stream beside the next chunk's y backward pass (two y-residue
    sets in turn); IMPCONV_ONE_STREAM runs the same launches in order on one
    stream.  Many chunks (64 planes), results equal bit for bit, and against
    the oracle; repeated calls agree (the sets are reused)."""
    ic = need_gpu()
    import torch
    say(f"3d overlap vs one stream {kind} {dt.__name__}")
    B, M = 2, 2
    if kind == "hermitian":
        m, n = (20, 17, 9), (40, 34, 10)
    else:
        m = n = (20, 17, 9)
    f = synth.unit_disk((B, M, *n), 87)
    g = synth.unit_disk((B, M, *n), 88)
    F, G = to_dev(f, dt), to_dev(g, dt)
    h1 = ic.conv3d(F, G, kind=kind, m=m, flags=ic.ONE_STREAM)
    for _ in range(3):
        assert torch.equal(ic.conv3d(F, G, kind=kind, m=m), h1)
    ref = (oracle.convnd_hermitian(rounded(f[1], dt), rounded(g[1], dt), m) if kind == "hermitian"
           else oracle.convnd_complex_M(rounded(f[1], dt), rounded(g[1], dt)))
    assert rel(h1[1].cpu().numpy(), ref) < TOL[dt]


def test_3d_overlapped_chunks_graph_replay():
    """A captured 3D convolution (fork to the auxiliary stream and join)
    replays correctly, with eager 3D calls between the replays."""
    ic = need_gpu()
    import torch
    m, n = (20, 17, 9), (40, 34, 10)
    f = synth.unit_disk((1, 3, *n), 89)
    g = synth.unit_disk((1, 3, *n), 90)
    F, G = to_dev(f, np.complex64), to_dev(g, np.complex64)
    eager = ic.conv3d(F, G, kind="hermitian", m=m)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        out = ic.conv3d(F, G, kind="hermitian", m=m)
    for rep in range(3):
        assert torch.equal(ic.conv3d(F, G, kind="hermitian", m=m), eager)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
