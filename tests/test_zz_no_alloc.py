"""impconv_conv2d_noalloc, the allocation-free form of impconv_conv2d: its
work arrays are the library's fixed per-device region.  Two calls in a row
(the second smaller, so it runs over what the first left in the region)
must equal impconv_conv2d on the same inputs bit for bit -- same kernels,
same launches -- and a small case is checked against the FP64 oracle too.
Sizes beyond the region are rejected on the host."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu


def _pair(shape, seeds, dt):
    return tuple(to_dev(synth.unit_disk(shape, s), dt) for s in seeds)


@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_noalloc_complex_2d_matches_conv2d(dt):
    ic = need_gpu()
    import torch
    # (B, M, m0, m1): the first needs 46 MB of the 64 MiB region
    B0 = 2 if dt == np.complex64 else 1
    for (B, M, m0, m1), seeds in [((B0, 1, 600, 700), (701, 702)), ((1, 2, 100, 37), (703, 704))]:
        say(f"noalloc complex2d B={B} M={M} m=({m0},{m1}) {dt.__name__}")
        F, G = _pair((B, M, m0, m1), seeds, dt)
        h = ic.conv2d_noalloc(F, G)
        torch.cuda.synchronize()
        ref = ic.conv2d(F, G)
        assert torch.equal(h, ref)
    f = synth.unit_disk((1, 2, 100, 37), 703)
    g = synth.unit_disk((1, 2, 100, 37), 704)
    assert rel(h[0].cpu().numpy(), oracle.convnd_complex_M(rounded(f[0], dt), rounded(g[0], dt))) < TOL[dt]


@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_noalloc_hermitian_2d_matches_conv2d(dt):
    ic = need_gpu()
    import torch
    for (B, M, m, n), seeds in [((2, 2, (200, 200), (400, 201)), (711, 712)),
                                ((1, 1, (17, 40), (33, 41)), (713, 714))]:
        say(f"noalloc hermitian2d B={B} M={M} m={m} n={n} {dt.__name__}")
        F, G = _pair((B, M, *n), seeds, dt)
        out = torch.empty((B, *n), dtype=F.dtype, device=F.device)
        h = ic.conv2d_noalloc(F, G, kind="hermitian", m=m, out=out)
        assert h.data_ptr() == out.data_ptr()
        torch.cuda.synchronize()
        ref = ic.conv2d(F, G, kind="hermitian", m=m)
        assert torch.equal(h, ref)
    f = synth.unit_disk((1, 1, 33, 41), 713)
    g = synth.unit_disk((1, 1, 33, 41), 714)
    assert rel(h[0].cpu().numpy(), oracle.convnd_hermitian(rounded(f[0], dt), rounded(g[0], dt), (17, 40))) < TOL[dt]


def test_noalloc_rejects_sizes_beyond_the_region():
    ic = need_gpu()
    L = ic.lib()
    assert L.impconv_init() == 0
    cap = ic.noalloc_capacity()
    assert cap == 64 << 20
    m = (ctypes.c_int64 * 2)(2048, 2048)
    need = ctypes.c_size_t()
    assert L.impconv_convnd_workspace(0, 1, 2, m, m, 4, 1, 0, ctypes.byref(need)) == 0
    assert need.value > cap
    # rejected before any pointer is looked at or any kernel launched
    assert L.impconv_conv2d_noalloc(0, 1, 4, 1, m, m, None, None, None, 0, None) == 3
    assert b"work memory" in L.impconv_last_error()
