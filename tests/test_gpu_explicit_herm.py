"""The explicitly zero-padded centered Hermitian 2D/3D comparator (padding
to powers of two >= 3m - 2, full-size transforms, real cyclic products,
crop) and its pruned form against the oracle, on inputs whose k_last = 0 hyperplane is already
Hermitian (the comparator reads that hyperplane by its real transforms)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu


def sym_storage(m, n, seed):
    """Stored half of a Hermitian field: random, zero slots zero, the
    k_last = 0 hyperplane made Hermitian (via the oracle's expansion)."""
    u = synth.unit_disk(n, seed)
    nd = len(m)
    full = oracle.hermitian_expand(u, m)
    out = np.zeros(n, complex)
    dst = tuple(slice(n[d] - 2 * m[d] + 1, n[d]) for d in range(nd - 1)) + (slice(0, m[-1]),)
    srcs = tuple(slice(None) for _ in range(nd - 1)) + (slice(m[-1] - 1, None),)
    out[dst] = full[srcs]
    return out


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("m,n", [((1, 1), (1, 1)), ((3, 4), (5, 4)), ((4, 3), (8, 4)), ((20, 17), (40, 18)),
                                 ((3, 2, 3), (6, 3, 4)), ((5, 6, 4), (9, 12, 5)), ((7, 3, 9), (14, 5, 10))])
def test_explicit_hermitian_nd_vs_oracle(dt, m, n):
    ic = need_gpu()
    say(f"explicit hermitian m={m} n={n} {dt.__name__}")
    B, M = 2, 2
    f = np.stack([np.stack([sym_storage(m, n, 800 + 4 * b + i) for i in range(M)]) for b in range(B)])
    g = np.stack([np.stack([sym_storage(m, n, 810 + 4 * b + i) for i in range(M)]) for b in range(B)])
    F, G = to_dev(f, dt), to_dev(g, dt)
    fn = ic.conv2d if len(m) == 2 else ic.conv3d
    he = fn(F, G, kind="hermitian", m=m, method="explicit").cpu().numpy()
    hp = fn(F, G, kind="hermitian", m=m, method="pruned").cpu().numpy()
    hi = fn(F, G, kind="hermitian", m=m).cpu().numpy()
    for b in range(B):
        ref = oracle.convnd_hermitian(rounded(f[b], dt), rounded(g[b], dt), m)
        assert rel(he[b], ref) < TOL[dt], b
        assert rel(hp[b], ref) < TOL[dt], b
        assert rel(hi[b], ref) < TOL[dt], b


def test_explicit_hermitian_3d_c4_shape_sampled():
    """256 modes per axis (storage 512 x 512 x 257), M = 3, complex64: the
    comparator's padded sizes 1024^2 x 1024 (real), at sampled outputs."""
    ic = need_gpu()
    m, n = (256, 256, 256), (512, 512, 257)
    M = 3
    f = np.stack([sym_storage(m, n, 820 + i) for i in range(M)])
    g = np.stack([sym_storage(m, n, 830 + i) for i in range(M)])
    F, G = to_dev(f[None], np.complex64), to_dev(g[None], np.complex64)
    pts = np.array([[0, 0, 0], [255, -255, 255], [-100, 37, 0], [3, -4, 200], [-255, 0, 17]])
    ref = oracle.convnd_hermitian_at(rounded(f, np.complex64), rounded(g, np.complex64), m, pts)
    for method in ("explicit", "pruned"):
        he = ic.conv3d(F, G, kind="hermitian", m=m, method=method).cpu().numpy()[0]
        got = he[pts[:, 0] + 256, pts[:, 1] + 256, pts[:, 2]]
        assert rel(got, ref) < TOL[np.complex64], method
        assert np.all(he[0] == 0) and np.all(he[:, 0] == 0) and np.all(he[..., 256] == 0), method  # zero slots
