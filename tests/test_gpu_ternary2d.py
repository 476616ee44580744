"""GPU parity of the 2D centered Hermitian ternary convolution (Sec. 4,
tconv2) against the FP64 oracle: full fields on small grids spanning several
tiles, odd and even storage and ragged sizes; the symmetrization readings;
rank-one inputs on x axes of 2048 to 4096 modes checked on the full field
against outer products of 1D oracle results (with the comparator); random
inputs on the longest x axes with a narrow y axis; sampled outputs of
random inputs."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu

DT = [np.complex128, np.complex64]


def storage(m, n, seed):
    u = synth.unit_disk(n, seed)
    if n[0] == 2 * m[0]:
        u[0] = 0
    if n[1] == m[1] + 1:
        u[:, m[1]] = 0
    return u


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m,n", [((1, 1), (1, 1)), ((1, 1), (2, 2)), ((2, 2), (4, 3)), ((3, 5), (5, 5)),
                                 ((5, 4), (10, 5)), ((8, 8), (16, 9)), ((9, 17), (17, 17)),
                                 ((16, 20), (32, 21))])
def test_tconv2_full_field(dt, m, n):
    ic = need_gpu()
    say(f"tconv2 m={m} n={n} {dt.__name__}")
    B = 2
    f = np.stack([storage(m, n, 301 + b) for b in range(B)])
    g = np.stack([storage(m, n, 303 + b) for b in range(B)])
    e = np.stack([storage(m, n, 305 + b) for b in range(B)])
    h = ic.conv2d_ternary(to_dev(f, dt), to_dev(g, dt), to_dev(e, dt), m).cpu().numpy()
    for b in range(B):
        ref = oracle.convnd_ternary(rounded(f[b], dt), rounded(g[b], dt), rounded(e[b], dt), m)
        assert rel(h[b], ref) < TOL[dt], b
    if n[0] == 2 * m[0]:
        assert np.all(h[:, 0] == 0)
    if n[1] == m[1] + 1:
        assert np.all(h[:, :, m[1]] == 0)


def test_tconv2_symmetrization_readings():
    ic = need_gpu()
    m, n = (6, 5), (12, 6)
    f, g, e = storage(m, n, 311), storage(m, n, 312), storage(m, n, 313)
    F, G, E = (to_dev(x, np.complex128) for x in (f, g, e))
    h = ic.conv2d_ternary(F, G, E, m).cpu().numpy()
    assert rel(h, oracle.convnd_ternary(f, g, e, m)) < 1e-12
    hp = ic.conv2d_ternary(F, G, E, m, symmetrize=False).cpu().numpy()
    assert rel(hp, oracle.convnd_ternary(f, g, e, m, symmetrize=False)) < 1e-12


def rank_one_case(mx, my, n, dt):
    """Rank-one inputs U = A (x) b (A a centered Hermitian vector, b a half
    with b_0 real) and the exact result: a full centered ternary sum in x
    (two numpy convolutions of the FP64 vectors) times the 1D Hermitian
    ternary oracle in y."""
    vecs = []
    for s in (321, 322, 323):
        a = synth.unit_disk(mx, s)
        a[0] = a[0].real
        vecs.append(np.concatenate([np.conj(a[:0:-1]), a]))  # k = -mx+1 .. mx-1
    ys = []
    for s in (324, 325, 326):
        b = synth.unit_disk(my, s)
        b[0] = b[0].real
        ys.append(b)
    off = n[0] - (2 * mx - 1)  # storage row of k_x = -mx+1
    fields = []
    for A, b in zip(vecs, ys):
        u = np.zeros(n, complex)
        u[off:, :my] = np.outer(A, b)
        fields.append(u)
    Ar = [rounded(A, dt) for A in vecs]
    br = [rounded(b, dt) for b in ys]
    xfull = np.convolve(np.convolve(Ar[0], Ar[1]), Ar[2])[2 * (mx - 1):4 * (mx - 1) + 1]
    ref = np.zeros(n, complex)
    ref[off:, :my] = np.outer(xfull, oracle.conv1d_ternary(*br))
    return fields, ref


@pytest.mark.parametrize("mx,my,n", [(2049, 8, (4097, 8)), (3000, 64, (5999, 64)), (4096, 256, (8192, 257))])
def test_tconv2_rank_one_longest_x(mx, my, n):
    """Complex64 x axes of 2049 to 4096 modes (transforms of 8192 points
    along x, column tiles of two columns), full field against the factored
    exact result; the explicit comparator and its pruned form as well
    (x FFTs of 4 N0' = 16384 points, one column per tile)."""
    dt = np.complex64
    ic = need_gpu()
    say(f"tconv2 rank one {mx} x {my} {dt.__name__}")
    fields, ref = rank_one_case(mx, my, n, dt)
    args = [to_dev(u, dt) for u in fields]
    h = ic.conv2d_ternary(*args, (mx, my)).cpu().numpy()
    assert rel(h, ref) < TOL[dt]
    if n[0] == 2 * mx:
        assert np.all(h[0] == 0)
    if n[1] == my + 1:
        assert np.all(h[:, my] == 0)
    for method in ("explicit", "pruned"):
        he = ic.conv2d_ternary(*args, (mx, my), method=method).cpu().numpy()
        assert rel(he, ref) < TOL[dt], method


def test_tconv2_longest_x_limits():
    """Beyond the column passes: complex128 x axes stop at 2048 modes (1024
    for the comparator), complex64 at 4096."""
    ic = need_gpu()
    import torch
    for dt, mx, method in [(torch.complex128, 2049, "implicit"), (torch.complex128, 1025, "explicit"),
                           (torch.complex64, 4097, "implicit"), (torch.complex64, 4097, "explicit")]:
        z = torch.zeros((1, 2 * mx, 3), dtype=dt, device="cuda")
        with pytest.raises(ic.ImpconvError):
            ic.conv2d_ternary(z, z, z, (mx, 2), method=method)


@pytest.mark.parametrize("m,n", [((4096, 1), (8192, 1)), ((3000, 1), (5999, 1))])
def test_tconv2_longest_x_random(m, n):
    """Random inputs on the longest x axes with a one-mode y axis: the whole
    field is the k_y = 0 line, symmetrized on load from its k_x >= 0 half
    (Im of the origin dropped), so the result is the full centered ternary
    sum of the symmetrized x vectors (two numpy convolutions in FP64);
    complex64, the dtype whose x axis reaches 4096 modes."""
    dt = np.complex64
    ic = need_gpu()
    say(f"tconv2 random m={m} n={n} {dt.__name__}")
    mx = m[0]
    off = n[0] - mx  # storage row of k_x = 0
    us = [storage(m, n, s) for s in (361, 362, 363)]
    h = ic.conv2d_ternary(*(to_dev(u, dt) for u in us), m).cpu().numpy()
    full = []
    for u in us:
        a = rounded(u[off:off + mx, 0], dt).copy()
        a[0] = a[0].real
        full.append(np.concatenate([np.conj(a[:0:-1]), a]))
    x = np.convolve(np.convolve(full[0], full[1]), full[2])[2 * (mx - 1):4 * (mx - 1) + 1]
    ref = np.zeros(n, complex)
    ref[n[0] - (2 * mx - 1):, 0] = x
    assert rel(h, ref) < TOL[dt]


@pytest.mark.parametrize("dt", DT)
def test_tconv2_rank_one_long_x(dt):
    """U = A (x) b per input, m = (2048, 512): the result factors into a
    full centered ternary sum in x (two numpy convolutions of the FP64
    vectors) and the 1D Hermitian ternary oracle in y."""
    ic = need_gpu()
    say(f"tconv2 rank one 2048 x 512 {dt.__name__}")
    mx, my = 2048, 512
    n = (2 * mx, my + 1)
    vecs = []
    for s in (321, 322, 323):
        a = synth.unit_disk(mx, s)
        a[0] = a[0].real
        full = np.concatenate([np.conj(a[:0:-1]), a])  # k = -mx+1 .. mx-1
        vecs.append(full)
    ys = []
    for s in (324, 325, 326):
        b = synth.unit_disk(my, s)
        b[0] = b[0].real
        ys.append(b)
    fields = []
    for A, b in zip(vecs, ys):
        u = np.zeros(n, complex)
        u[1:, :my] = np.outer(A, b)
        fields.append(u)
    h = ic.conv2d_ternary(*(to_dev(u, dt) for u in fields), (mx, my)).cpu().numpy()
    Ar = [rounded(A, dt) for A in vecs]
    br = [rounded(b, dt) for b in ys]
    xfull = np.convolve(np.convolve(Ar[0], Ar[1]), Ar[2])[2 * (mx - 1):4 * (mx - 1) + 1]
    yref = oracle.conv1d_ternary(*br)
    ref = np.zeros(n, complex)
    ref[1:, :my] = np.outer(xfull, yref)
    # the input products of rounded vectors differ from the rounded products
    # by one rounding; the FP32 tolerance covers it
    assert rel(h, ref) < TOL[dt]
    assert np.all(h[0] == 0) and np.all(h[:, my] == 0)


@pytest.mark.parametrize("dt", DT)
def test_tconv2_sampled(dt):
    ic = need_gpu()
    m, n = (64, 48), (127, 49)
    f, g, e = storage(m, n, 331), storage(m, n, 332), storage(m, n, 333)
    h = ic.conv2d_ternary(to_dev(f, dt), to_dev(g, dt), to_dev(e, dt), m).cpu().numpy()
    pts = np.array([[0, 0], [-63, 47], [63, 0], [5, 3], [-20, 40], [31, 1]])
    ref = oracle.convnd_ternary_at(rounded(f, dt), rounded(g, dt), rounded(e, dt), m, pts)
    got = h[pts[:, 0] + 63, pts[:, 1]]
    assert rel(got, ref) < TOL[dt]


def symmetric_storage(m, n, seed):
    """Storage whose k_y = 0 line is already Hermitian (the comparator reads
    that line as its projection, the implicit path by its positive half)."""
    u = storage(m, n, seed)
    off = n[0] - m[0]
    for k in range(1, m[0]):
        u[off - k, 0] = np.conj(u[off + k, 0])
    u[off, 0] = u[off, 0].real
    return u


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m,n", [((1, 1), (1, 1)), ((2, 3), (4, 4)), ((5, 4), (9, 5)), ((12, 17), (24, 18))])
def test_tconv2_explicit_comparator(dt, m, n):
    ic = need_gpu()
    say(f"tconv2 explicit m={m} n={n} {dt.__name__}")
    B = 2
    f = np.stack([symmetric_storage(m, n, 341 + b) for b in range(B)])
    g = np.stack([symmetric_storage(m, n, 343 + b) for b in range(B)])
    e = np.stack([symmetric_storage(m, n, 345 + b) for b in range(B)])
    args = [to_dev(x, dt) for x in (f, g, e)]
    he = ic.conv2d_ternary(*args, m, method="explicit").cpu().numpy()
    hp = ic.conv2d_ternary(*args, m, method="pruned").cpu().numpy()
    hi = ic.conv2d_ternary(*args, m).cpu().numpy()
    for b in range(B):
        ref = oracle.convnd_ternary(rounded(f[b], dt), rounded(g[b], dt), rounded(e[b], dt), m)
        assert rel(he[b], ref) < TOL[dt], b
        assert rel(hp[b], ref) < TOL[dt], b
        assert rel(hi[b], ref) < TOL[dt], b
    if n[0] == 2 * m[0]:
        assert np.all(he[:, 0] == 0)
    if n[1] == m[1] + 1:
        assert np.all(he[:, :, m[1]] == 0)


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m", [1, 2, 7, 64, 300])
def test_ternary_1d_explicit_comparator(dt, m):
    ic = need_gpu()
    f, g, e = (synth.unit_disk((3, m), s) for s in (351, 352, 353))
    h = ic.conv1d_ternary(to_dev(f, dt), to_dev(g, dt), to_dev(e, dt), method="explicit").cpu().numpy()
    for b in range(3):
        ref = oracle.conv1d_ternary(rounded(f[b], dt), rounded(g[b], dt), rounded(e[b], dt))
        assert rel(h[b], ref) < TOL[dt]
