"""The persistent work-queue launch of ragged batches: the queued size classes
(one launch, items taken from an atomic counter, longest class first) give
the same results as one launch per class, bit for bit with the same values
per thread; with the other values per thread they match the FP64 oracle; the
counter is cleared by every execution (eager repeats and hipGraph replays);
the autotuner chooses per class and records its choices in the schedule
cache, which a later plan takes without timing."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say, to_dev

pytestmark = pytest.mark.gpu

# every fused size class N = 1 .. 8192, ragged lengths within a class, and
# two four-step pairs beside them
MS = np.array([1, 2, 3, 4, 5, 7, 8, 9, 16, 17, 31, 33, 64, 65, 100, 128, 129, 200, 256, 300, 512, 700,
               1024, 1500, 2048, 3000, 4096, 5000, 8192, 6000, 20000, 40000, 64, 64, 64, 1, 8, 4095])


def packed(ms, seed, gap=2):
    offs = np.concatenate([[0], np.cumsum(np.asarray(ms) + gap)[:-1]])
    total = int(offs[-1] + ms[-1] + gap)
    return offs, synth.unit_disk(total, seed)


def torch_dt(dt):
    import torch
    return torch.complex64 if dt == np.complex64 else torch.complex128


def check_oracle(h, f, g, ms, offs, dt):
    fr, gr = rounded(f, dt), rounded(g, dt)
    for m, o in zip(ms, offs):
        if m <= 5000:
            ref = oracle.conv1d_complex(fr[o:o + m], gr[o:o + m])
            assert rel(h[o:o + m], ref) < TOL[dt], m
        else:
            ks = np.array([0, 1, m // 3, m - 1])
            ref = oracle.convnd_complex_at(fr[o:o + m], gr[o:o + m], ks[:, None])
            assert rel(h[o + ks], ref) < TOL[dt], m


@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_queue_equals_per_class_launches(dt):
    ic = need_gpu()
    import torch
    say(f"queue vs per-class {dt.__name__}")
    offs, f = packed(MS, 901)
    _, g = packed(MS, 902)
    F, G = to_dev(f, dt), to_dev(g, dt)
    plan = ic.RaggedPlan(MS, offs, dtype=torch_dt(dt))
    info = plan.schedule_info()
    assert info["fused_launch"] == "queue"
    queued = [c for c in info["classes"] if c["method"] == "queue"]
    top = 8192 if dt == np.complex64 else 4096
    assert {c["N"] for c in queued} == {int(n) for n in 2 ** np.ceil(np.log2(MS)).astype(int) if n <= top}
    hq = [plan.execute(F, G) for _ in range(3)]  # the counter restarts at every execution
    plan.set_fused(False)
    assert plan.schedule_info()["fused_launch"] == "per-class"
    hc = plan.execute(F, G)
    for h in hq:
        assert torch.equal(h, hc)
    check_oracle(hc.cpu().numpy(), f, g, MS, offs, dt)


@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_queue_half_values_per_thread_vs_oracle(dt):
    ic = need_gpu()
    import torch
    say(f"queue with half E {dt.__name__}")
    offs, f = packed(MS, 903)
    _, g = packed(MS, 904)
    F, G = to_dev(f, dt), to_dev(g, dt)
    plan = ic.RaggedPlan(MS, offs, dtype=torch_dt(dt))
    full = {c["N"]: c["E"] for c in plan.schedule() if c["method"] == "queue"}
    plan.set_fused(True, elems=max(full.values()) // 2)
    half = {c["N"]: c["E"] for c in plan.schedule() if c["method"] == "queue"}
    assert any(half[n] != full[n] for n in full)
    h = plan.execute(F, G)
    check_oracle(h.cpu().numpy(), f, g, MS, offs, dt)
    # adjoint flags through the queue: dL/df = rev(conv(rev(w), conj g))
    w = synth.unit_disk(len(f), 905)
    W = to_dev(w, dt)
    gf = plan.execute(W, G, flags=ic.REV_F | ic.CONJ_G | ic.REV_OUT).cpu().numpy()
    for m, o in zip(MS, offs):
        if m > 3000:
            continue
        rf, _ = oracle.grad_conv1d_complex(rounded(f, dt)[o:o + m], rounded(g, dt)[o:o + m], rounded(w, dt)[o:o + m])
        assert rel(gf[o:o + m], rf) < TOL[dt], m


def test_queue_graph_replay():
    """A captured queue execution replays correctly every time, with eager
    executions of the same plan (other workspace) between the replays."""
    ic = need_gpu()
    import torch
    say("queue graph replay")
    offs, f = packed(MS, 906)
    _, g = packed(MS, 907)
    F, G = to_dev(f, np.complex64), to_dev(g, np.complex64)
    plan = ic.RaggedPlan(MS, offs, dtype=torch.complex64, autotune=True)
    plan.set_fused(True)
    eager = plan.execute(F, G)
    out = torch.zeros_like(F)
    work = torch.empty(max(plan.work_bytes, 16), dtype=torch.uint8, device=F.device)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.execute(F, G, out=out, work=work)
    for rep in range(3):
        out.zero_()
        assert torch.equal(plan.execute(F, G), eager)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep


def test_autotune_records_and_reuses_schedule_cache():
    ic = need_gpu()
    import torch
    say("autotune + schedule cache")
    ic.schedule_cache_clear()
    offs, f = packed(MS, 908)
    _, g = packed(MS, 909)
    F, G = to_dev(f, np.complex64), to_dev(g, np.complex64)
    plan = ic.RaggedPlan(MS, offs, dtype=torch.complex64, autotune=True)
    info = plan.schedule_info()
    say(f"schedule {info}")
    assert info["fused_launch"] in ("queue", "per-class")
    assert set(info["fused_tuned_ms"]) == {"queue", "per-class"}
    faster = min(info["fused_tuned_ms"], key=info["fused_tuned_ms"].get)
    assert info["fused_launch"] == faster
    for c in info["classes"]:
        assert c["source"] == "timed", c
        t = c["tuned_ms"]
        choice = str(c["E"] if c["N"] <= 8192 else c["N2"])
        assert t[choice] == min(t.values())
    cache = ic.schedule_cache_export()
    keys = {(e["variant"], e["N"]): e["choice"] for e in cache if e["dtype"] == "c64"}
    for c in info["classes"]:
        if c["N"] <= 8192:
            assert keys[("fused", c["N"])] == c["E"]
        else:
            assert keys[("fourstep", c["N"])] == c["N2"]
    assert all(e["arch"].startswith("gfx") for e in cache)
    h = plan.execute(F, G).cpu().numpy()
    check_oracle(h, f, g, MS, offs, np.complex64)
    # a second plan with the same classes takes every class choice from the cache
    plan2 = ic.RaggedPlan(MS, offs, dtype=torch.complex64, autotune=True)
    for c in plan2.schedule():
        assert c["source"] == "cache", c
        assert keys[("fused" if c["N"] <= 8192 else "fourstep", c["N"])] == (c["E"] if c["N"] <= 8192 else c["N2"])
    # import into a cleared cache: the same choices again
    ic.schedule_cache_clear()
    ic.schedule_cache_import(cache)
    plan3 = ic.RaggedPlan(MS, offs, dtype=torch.complex64, autotune=True)
    for c3, c in zip(plan3.schedule(), info["classes"]):
        assert c3["source"] == "cache"
        assert (c3.get("E"), c3.get("N2")) == (c.get("E"), c.get("N2"))
    check_oracle(plan3.execute(F, G).cpu().numpy(), f, g, MS, offs, np.complex64)
    ic.schedule_cache_clear()
