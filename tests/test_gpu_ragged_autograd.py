"""GPU parity of the ragged (uneven-length) batch and of the differentiable
wrappers: forward vs the FP64 oracle, backward vs the oracle's analytic
adjoint and vs central finite differences, hipGraph replay vs eager."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu


def packed(ms, seed, gap=3):
    offs = np.concatenate([[0], np.cumsum(np.asarray(ms) + gap)[:-1]])
    total = int(offs[-1] + ms[-1] + gap)
    return offs, synth.unit_disk(total, seed)


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
def test_ragged_small_mixed(dt):
    ic = need_gpu()
    import torch
    ms = np.array([1, 2, 3, 64, 100, 1024, 5, 8192, 8193, 20000, 7, 64])
    offs, f = packed(ms, 101)
    _, g = packed(ms, 102)
    plan = ic.RaggedPlan(ms, offs, dtype=torch.complex64 if dt == np.complex64 else torch.complex128)
    h = plan.execute(to_dev(f, dt), to_dev(g, dt)).cpu().numpy()
    fr, gr = rounded(f, dt), rounded(g, dt)
    for m, o in zip(ms, offs):
        if m <= 8192:
            ref = oracle.conv1d_complex(fr[o:o + m], gr[o:o + m])
            assert rel(h[o:o + m], ref) < TOL[dt], m
        else:
            ks = np.array([0, 1, m // 3, m - 1])
            ref = oracle.convnd_complex_at(fr[o:o + m], gr[o:o + m], ks[:, None])
            assert rel(h[o + ks], ref) < TOL[dt], m
    # gaps between pairs are untouched (zero-initialised output)
    mask = np.ones(len(f), bool)
    for m, o in zip(ms, offs):
        mask[o:o + m] = False
    assert np.all(h[mask] == 0)


def test_ragged_c5_workload():
    """4096 pairs, m = 2^round(U(6,16)), complex64, packed; every pair with
    m <= 1024 checked in full, longer pairs at sampled outputs."""
    ic = need_gpu()
    import torch
    ms = synth.ragged_lengths(4096, 6, 16, 5)
    offs = np.concatenate([[0], np.cumsum(ms)[:-1]])
    f = synth.unit_disk(int(ms.sum()), 9).astype(np.complex64)
    g = synth.unit_disk(int(ms.sum()), 10).astype(np.complex64)
    say(f"ragged C5: {len(ms)} pairs, sum m = {ms.sum()}")
    plan = ic.RaggedPlan(ms, offs, dtype=torch.complex64)
    h = plan.execute(to_dev(f, np.complex64), to_dev(g, np.complex64)).cpu().numpy()
    fr, gr = f.astype(np.complex128), g.astype(np.complex128)
    small = np.where(ms <= 1024)[0][:300]
    sm, so = ms[small], offs[small]
    ref = oracle.conv1d_complex_ragged(sm, np.concatenate([[0], np.cumsum(sm)[:-1]]),
                                       np.concatenate([fr[o:o + m] for m, o in zip(sm, so)]),
                                       np.concatenate([gr[o:o + m] for m, o in zip(sm, so)]))
    got = np.concatenate([h[o:o + m] for m, o in zip(sm, so)])
    for j, (m, o) in enumerate(zip(sm, np.concatenate([[0], np.cumsum(sm)[:-1]]))):
        assert rel(got[o:o + m], ref[o:o + m]) < TOL[np.complex64]
    big = np.where(ms >= 16384)[0][:12]
    for j in big:
        m, o = ms[j], offs[j]
        ks = np.array([0, 5, m // 2, m - 1])
        r = oracle.convnd_complex_at(fr[o:o + m], gr[o:o + m], ks[:, None])
        assert rel(h[o + ks], r) < TOL[np.complex64]


def test_ragged_autotuned_schedule():
    """The autotuner times every supported four-step split of the long
    classes and keeps one; the tuned plan's results match the oracle and
    the untuned plan, and the tuned plan replays under hipGraph capture."""
    ic = need_gpu()
    import torch
    ms = np.array([64, 5000, 16384, 40000, 65536, 9, 20000])
    ic.schedule_cache_clear()  # every class timed here, none taken from an earlier plan's choices
    offs, f = packed(ms, 161)
    _, g = packed(ms, 162)
    F, G = to_dev(f, np.complex64), to_dev(g, np.complex64)
    base = ic.RaggedPlan(ms, offs, dtype=torch.complex64)
    ref_gpu = base.execute(F, G).cpu().numpy()
    plan = ic.RaggedPlan(ms, offs, dtype=torch.complex64, autotune=True)
    sch = plan.schedule()
    say(f"schedule {sch}")
    long = [c for c in sch if c["method"] == "four-step"]
    assert {c["N"] for c in long} == {16384, 32768, 65536}
    for c in long:
        assert c["N1"] * c["N2"] == c["N"]
        assert str(c["N2"]) in c["tuned_ms"] and len(c["tuned_ms"]) >= 3
        assert c["tuned_ms"][str(c["N2"])] == min(c["tuned_ms"].values())
    h = plan.execute(F, G).cpu().numpy()
    assert rel(h, ref_gpu) < TOL[np.complex64]
    fr, gr = rounded(f, np.complex64), rounded(g, np.complex64)
    for m, o in zip(ms, offs):
        ks = np.array([0, 1, m // 3, m - 1]) if m > 3 else np.arange(m)
        r = oracle.convnd_complex_at(fr[o:o + m], gr[o:o + m], ks[:, None])
        assert rel(h[o + ks], r) < TOL[np.complex64], m
    out = torch.zeros_like(F)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.execute(F, G, out=out)
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), h), rep


@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_ragged_one_stream_matches_concurrent(dt):
    """ONE_STREAM (every size class on the caller's stream, in turn) runs the
    same kernels as the concurrent form: bitwise equal results, also with the
    adjoint flags and through the autograd wrapper; forward checked against
    the oracle on the short pairs and at sampled outputs of the long ones."""
    ic = need_gpu()
    import torch
    tdt = torch.complex64 if dt == np.complex64 else torch.complex128
    ms = np.array([64, 300, 4096, 16384, 65536, 9, 8193, 1, 40000])
    offs, f = packed(ms, 141)
    _, g = packed(ms, 142)
    say(f"ragged one-stream {dt.__name__}")
    F, G = to_dev(f, dt), to_dev(g, dt)
    plan = ic.RaggedPlan(ms, offs, dtype=tdt)
    for fl in (0, ic.REV_F | ic.CONJ_G | ic.REV_OUT):
        conc = plan.execute(F, G, flags=fl)
        one = plan.execute(F, G, flags=fl | ic.ONE_STREAM)
        torch.cuda.synchronize()
        assert torch.equal(conc, one), fl
    fr, gr = rounded(f, dt), rounded(g, dt)
    h = plan.execute(F, G, flags=ic.ONE_STREAM).cpu().numpy()
    for m, o in zip(ms, offs):
        if m <= 4096:
            assert rel(h[o:o + m], oracle.conv1d_complex(fr[o:o + m], gr[o:o + m])) < TOL[dt], m
        else:
            ks = np.array([0, 1, m // 3, m - 1])
            ref = oracle.convnd_complex_at(fr[o:o + m], gr[o:o + m], ks[:, None])
            assert rel(h[o + ks], ref) < TOL[dt], m
    w = to_dev(synth.unit_disk(f.shape[0], 143), dt)
    grads = []
    for one_stream in (False, True):
        plan.one_stream = one_stream
        Fr = F.clone().requires_grad_(True)
        Gr = G.clone().requires_grad_(True)
        ic.ragged_conv_ad(plan, Fr, Gr).backward(w)
        grads.append((Fr.grad, Gr.grad))
    plan.one_stream = False
    assert torch.equal(grads[0][0], grads[1][0]) and torch.equal(grads[0][1], grads[1][1])


@pytest.mark.skip(reason="twice crashed the host process (segmentation fault) inside the replay of this graph in "
                         "full GPU runs, after the threaded one-shot eviction test (skipped too) had run earlier in "
                         "the process; the cause is not established, so the case stays off the GPU until it is")
def test_ragged_graph_replay_matches_eager():
    ic = need_gpu()
    import torch
    ms = np.array([64, 300, 4096, 16384, 65536, 9])
    offs, f = packed(ms, 111)
    _, g = packed(ms, 112)
    F, G = to_dev(f, np.complex64), to_dev(g, np.complex64)
    plan = ic.RaggedPlan(ms, offs, dtype=torch.complex64)
    eager = plan.execute(F, G)
    out = torch.zeros_like(F)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.execute(F, G, out=out)
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep


@pytest.mark.parametrize("m", [1, 7, 100, 3000, 20000])
def test_autograd_backward_vs_oracle_adjoint(m):
    ic = need_gpu()
    import torch
    f = synth.unit_disk(m, 121)
    g = synth.unit_disk(m, 122)
    w = synth.unit_disk(m, 123)
    F = to_dev(f, np.complex128).requires_grad_(True)
    G = to_dev(g, np.complex128).requires_grad_(True)
    W = to_dev(w, np.complex128)
    h = ic.conv1d_complex_ad(F, G)
    L = torch.real(torch.sum(torch.conj(W) * h))
    L.backward()
    gf, gg = oracle.grad_conv1d_complex(f, g, w)
    if m <= 3000:
        assert rel(F.grad.cpu().numpy(), gf) < 1e-12
        assert rel(G.grad.cpu().numpy(), gg) < 1e-12
    else:
        assert rel(F.grad.cpu().numpy()[:50], gf[:50]) < 1e-11


def test_autograd_gradcheck_small():
    ic = need_gpu()
    import torch
    f = to_dev(synth.unit_disk((2, 9), 131), np.complex128).requires_grad_(True)
    g = to_dev(synth.unit_disk((2, 9), 132), np.complex128).requires_grad_(True)
    assert torch.autograd.gradcheck(ic.conv1d_complex_ad, (f, g), eps=1e-6, atol=1e-8)


def test_autograd_finite_differences_fp32_mdot():
    """Central differences of L = Re sum conj(w) h on random coordinates
    (complex64 forward, complex128 reference), M = 2 dot product."""
    ic = need_gpu()
    import torch
    B, M, m = 2, 2, 257
    f = synth.unit_disk((B, M, m), 141)
    g = synth.unit_disk((B, M, m), 142)
    w = synth.unit_disk((B, m), 143)
    F = to_dev(f, np.complex64).requires_grad_(True)
    G = to_dev(g, np.complex64).requires_grad_(True)
    W = to_dev(w, np.complex64)
    L = torch.real(torch.sum(torch.conj(W) * ic.conv1d_complex_ad(F, G)))
    L.backward()
    fr, gr = rounded(f, np.complex64), rounded(g, np.complex64)
    wr = rounded(w, np.complex64)

    def Lf(ff):
        return np.real(np.vdot(wr, oracle.conv1d_complex(ff, gr)))

    rng = synth.rng(144)
    for _ in range(6):
        b, i, p = rng.integers(0, B), rng.integers(0, M), rng.integers(0, m)
        e = np.zeros_like(fr)
        e[b, i, p] = 1e-3
        d = (Lf(fr + e) - Lf(fr - e)) / 2e-3 + 1j * (Lf(fr + 1j * e) - Lf(fr - 1j * e)) / 2e-3
        got = F.grad[b, i, p].item()
        assert abs(got - d) < 2e-5 * max(1.0, abs(d))


def test_ragged_backward_vs_oracle():
    ic = need_gpu()
    import torch
    ms = np.array([5, 64, 1000, 20000])
    offs, f = packed(ms, 151, gap=0)
    _, g = packed(ms, 152, gap=0)
    _, w = packed(ms, 153, gap=0)
    F = to_dev(f, np.complex128).requires_grad_(True)
    G = to_dev(g, np.complex128).requires_grad_(True)
    W = to_dev(w, np.complex128)
    plan = ic.RaggedPlan(ms, offs, dtype=torch.complex128)
    h = ic.ragged_conv_ad(plan, F, G)
    torch.real(torch.sum(torch.conj(W) * h)).backward()
    for m, o in zip(ms, offs):
        gf, gg = oracle.grad_conv1d_complex(f[o:o + m], g[o:o + m], w[o:o + m])
        k = min(m, 64)
        assert rel(F.grad[o:o + k].cpu().numpy(), gf[:k]) < 1e-11
        assert rel(G.grad[o:o + k].cpu().numpy(), gg[:k]) < 1e-11


def test_ragged_concurrent_classes_and_threads():
    """The size classes run on the plan's auxiliary streams; two host threads
    executing one plan on their own streams (distinct workspaces and inputs)
    get the same results as one at a time, and the schedule reports the
    stream of every class."""
    ic = need_gpu()
    import threading
    import torch
    ms = np.array([20000, 9000, 40000, 64, 3000, 100, 8192, 17, 16384, 512])
    offs, f1 = packed(ms, 131)
    _, g1 = packed(ms, 132)
    _, f2 = packed(ms, 133)
    _, g2 = packed(ms, 134)
    plan = ic.RaggedPlan(ms, offs)
    lanes = {c["stream"] for c in plan.schedule()}
    assert len(lanes) > 1
    F1, G1, F2, G2 = (to_dev(x, np.complex64) for x in (f1, g1, f2, g2))
    ref1 = plan.execute(F1, G1).cpu()
    ref2 = plan.execute(F2, G2).cpu()
    torch.cuda.synchronize()
    out = {}

    def work(k, F, G):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            w = torch.empty(max(plan.work_bytes, 16), dtype=torch.uint8, device=F.device)
            for _ in range(5):
                h = plan.execute(F, G, work=w)
            s.synchronize()
            out[k] = h.cpu()

    ts = [threading.Thread(target=work, args=(1, F1, G1)), threading.Thread(target=work, args=(2, F2, G2))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert torch.equal(out[1], ref1) and torch.equal(out[2], ref2)
