#!/usr/bin/env python3
"""Benchmark of the implicitly dealiased convolution on one MI355X.

Default workload (c3): 2D complex dealiased convolutions of 2048 x 2048
complex64 inputs, a batch of 8 independent pairs per step, one call of
conv2d.  Each step's result is a batch of 8 dealiased convolutions; value =
convolutions per second, with inputs resident in HBM before the timed region.
The explicitly zero-padded comparator (same FFT kernels, padded 4096 x 4096
arrays materialized in HBM) is timed the same way.

Other workloads (--workload): c1 (1D complex m=1024 complex128, batch 16384),
c2 (1D centered Hermitian m=16384, batch 256), c4 (3D centered Hermitian
512x512x257, M=3), c5 (4096 uneven 1D complex pairs, forward + backward).

Output: one JSON line (rank 0) with the metric, per-step time, the roofline
of the dominant kernel (HIP-event durations recorded by the library around
each launch, on the launch stream) and the FP64 oracle timed on the host on
a bounded sample (the only place bench.py touches the oracle).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dealiased convs/sec + HBM GB/s, implicit vs explicit-padded, FP32/FP64 at rel err"
HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1008_1366_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hpp", ".hip")):
            h.update(open(os.path.join(csrc, fn), "rb").read())
    return h.hexdigest()[:16]


def timed(fn, steps, warmup, backlog=False):
    """Average ms per step over `steps` calls, bracketed by events on the
    current stream.  backlog=True first queues a ~20 ms spin kernel so the
    host enqueues every step before the GPU reaches them: per-launch event
    pairs recorded inside the library then time the kernels alone, not the
    host's launch gaps."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    if backlog:
        torch.cuda._sleep(50_000_000)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


# --------------------------------------------------------------------------- workloads

def wl_c3(args):
    """2D complex 2048^2, batch 8 pairs (Gaussian spectra times (1+|k|^2)^-1)."""
    import torch
    import paper_1008_1366_amd as ic
    import synth
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    mx = my = 2048
    B = 8
    f = np.stack([synth.gaussian_2d(mx, my, 100 + 2 * b) for b in range(B)])
    g = np.stack([synth.gaussian_2d(mx, my, 101 + 2 * b) for b in range(B)])
    F = torch.from_numpy(f).to("cuda", cdt)
    G = torch.from_numpy(g).to("cuda", cdt)
    cs = 8 if cdt == torch.complex64 else 16
    S = B * mx * my * cs                      # one stored batch of inputs
    run = lambda: ic.conv2d(F, G)
    expl = lambda: ic.conv2d(F, G, method="explicit")
    # algorithmic bytes per launch: every pass moves 3 S (Sec. 3.1 schedule)
    kbytes = {"colpass_pad_bwd": 3 * S, "k_conv1d_complex": 3 * S, "colpass_pad_fwd": 3 * S}
    step_bytes = 15 * S

    def cpu_baseline(h_gpu):
        """Oracle at stratified sample points of every pair: the whole
        low-wavenumber block [0,L)^2 (where the energy of the (1+|k|^2)^-1
        spectra concentrates) plus uniform random points elsewhere.  The
        strata weights give an estimate of the full-field relative L2 error;
        the time gives the oracle's rate, extrapolated by multiply-add count."""
        import oracle
        rng = synth.rng(7)
        L = 16
        blk = np.array([(i, j) for i in range(L) for j in range(L)])
        nrand = max(1, args.cpu_points // B)
        dt_np = np.complex64 if cdt == torch.complex64 else np.complex128
        num = den = pnum = pden = 0.0
        macs = 0.0
        t_oracle = 0.0
        for b in range(B):
            rp = rng.integers(0, mx, (4 * nrand, 2))
            rp = rp[(rp[:, 0] >= L) | (rp[:, 1] >= L)][:nrand]
            pts = np.concatenate([blk, rp])
            fr = np.asarray(f[b].astype(dt_np), np.complex128)
            gr = np.asarray(g[b].astype(dt_np), np.complex128)
            t0 = time.perf_counter()
            ref = oracle.convnd_complex_at(fr, gr, pts)
            t_oracle += time.perf_counter() - t0
            macs += float(np.sum((pts[:, 0] + 1.0) * (pts[:, 1] + 1.0)))
            got = h_gpu[b][pts[:, 0], pts[:, 1]]
            e2 = np.abs(got - ref) ** 2
            r2 = np.abs(ref) ** 2
            wb = (mx * my - L * L) / len(rp)
            num += e2[:len(blk)].sum() + wb * e2[len(blk):].sum()
            den += r2[:len(blk)].sum() + wb * r2[len(blk):].sum()
            pnum += e2[len(blk):].sum()
            pden += r2[len(blk):].sum()
        full = (mx * (mx + 1) / 2.0) * (my * (my + 1) / 2.0)
        convs_per_s = 1.0 / (t_oracle / macs * full)
        errs = {"full_field_estimate": float(np.sqrt(num / den)),
                "uniform_random_points": float(np.sqrt(pnum / pden))}
        return {"value": convs_per_s, "unit": "convs/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"per pair the {L}x{L} low-wavenumber block plus {nrand} uniform random "
                          f"output points, direct FP64 sums ({t_oracle:.2f} s), extrapolated to whole "
                          f"convolutions by multiply-add count"}, errs

    cfg = {"workload": f"2D complex implicit dealiased convolution {mx}x{my}, batch {B} pairs per step, "
                       f"{'complex64' if cdt == torch.complex64 else 'complex128'}",
           "m": [mx, my], "batch": B, "M": 1, "dtype": args.dtype}
    return dict(run=run, explicit=expl, convs=B, step_bytes=step_bytes, kbytes=kbytes, cfg=cfg,
                cpu=cpu_baseline, out=lambda: run().cpu().numpy())


def wl_c2(args):
    """1D centered Hermitian m=16384, |k|^-5/6 random phase, batch of B convolutions."""
    import torch
    import paper_1008_1366_amd as ic
    import synth
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    m, B = 16384, args.batch or 256
    f = synth.power_spectrum_1d(m, 5 / 6, 3, batch=B)
    g = synth.power_spectrum_1d(m, 5 / 6, 4, batch=B)
    F = torch.from_numpy(f).to("cuda", cdt)
    G = torch.from_numpy(g).to("cuda", cdt)
    cs = 8 if cdt == torch.complex64 else 16
    run = lambda: ic.conv1d_hermitian(F, G)
    kbytes = {"k_conv1d_hermitian": 3 * B * m * cs}

    def cpu_baseline(h_gpu):
        import oracle
        nb = max(1, args.cpu_rows)
        fr = np.asarray(f[:nb].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)
        gr = np.asarray(g[:nb].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)
        t0 = time.perf_counter()
        ref = oracle.conv1d_hermitian(fr[:, None], gr[:, None])
        dt = time.perf_counter() - t0
        err = float(np.linalg.norm(h_gpu[:nb] - ref) / np.linalg.norm(ref))
        return {"value": nb / dt, "unit": "convs/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{nb} of the {B} convolutions, direct FP64 sums ({dt:.2f} s)"}, err

    cfg = {"workload": f"1D centered Hermitian implicit dealiased convolution m={m}, batch {B}, "
                       f"{'complex64' if cdt == torch.complex64 else 'complex128'}",
           "m": m, "batch": B, "dtype": args.dtype}
    expl = None
    return dict(run=run, explicit=expl, convs=B, step_bytes=3 * B * m * cs, kbytes=kbytes, cfg=cfg,
                cpu=cpu_baseline, out=lambda: run().cpu().numpy())


def wl_c1(args):
    """1D complex m=1024 complex128 (unit-disk entries), batch of B pairs."""
    import torch
    import paper_1008_1366_amd as ic
    import synth
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    m, B = 1024, args.batch or 16384
    f = synth.unit_disk((B, m), 1)
    g = synth.unit_disk((B, m), 2)
    F = torch.from_numpy(f).to("cuda", cdt)
    G = torch.from_numpy(g).to("cuda", cdt)
    cs = 8 if cdt == torch.complex64 else 16
    run = lambda: ic.conv1d_complex(F, G)
    expl = lambda: ic.conv1d_complex(F, G, method="explicit")
    kbytes = {"k_conv1d_complex": 3 * B * m * cs}

    def cpu_baseline(h_gpu):
        import oracle
        nb = max(1, args.cpu_rows)
        t0 = time.perf_counter()
        ref = oracle.conv1d_complex(np.asarray(f[:nb].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)[:, None],
                                    np.asarray(g[:nb].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)[:, None])
        dt = time.perf_counter() - t0
        err = float(np.linalg.norm(h_gpu[:nb] - ref) / np.linalg.norm(ref))
        return {"value": nb / dt, "unit": "convs/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{nb} of the {B} pairs, direct FP64 sums ({dt:.2f} s)"}, err

    cfg = {"workload": f"1D complex implicit dealiased convolution m={m}, batch {B}, "
                       f"{'complex64' if cdt == torch.complex64 else 'complex128'}", "m": m, "batch": B,
           "dtype": args.dtype}
    return dict(run=run, explicit=expl, convs=B, step_bytes=3 * B * m * cs, kbytes=kbytes, cfg=cfg,
                cpu=cpu_baseline, out=lambda: run().cpu().numpy())


def wl_c4(args):
    """3D centered Hermitian, storage 512x512x257 (m=256/axis), M=3 pairs summed."""
    import torch
    import paper_1008_1366_amd as ic
    import synth
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    m, n = (256, 256, 256), (512, 512, 257)
    f = np.stack([synth.power_spectrum_centered(m, n, 11 / 6, 200 + i) for i in range(3)])[None]
    g = np.stack([synth.power_spectrum_centered(m, n, 11 / 6, 203 + i) for i in range(3)])[None]
    F = torch.from_numpy(f).to("cuda", cdt)
    G = torch.from_numpy(g).to("cuda", cdt)
    cs = 8 if cdt == torch.complex64 else 16
    S = int(np.prod(n)) * cs
    run = lambda: ic.conv3d(F, G, kind="hermitian", m=m)
    # Sec. 3.4 five-pass schedule, algorithmic bytes per launch
    kbytes = {"colpass_cen_bwd": None, "k_conv1d_hermitian": None, "colpass_cen_fwd": None}
    step_bytes = int(59.5 * S)

    def cpu_baseline(h_gpu):
        import oracle
        pts = np.array([[0, 0, 0], [255, 255, 255], [-255, 0, 3], [5, -7, 0]])
        fr = np.asarray(f[0].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)
        gr = np.asarray(g[0].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)
        t0 = time.perf_counter()
        ref = oracle.convnd_hermitian_at(fr, gr, m, pts)
        dt = time.perf_counter() - t0
        got = h_gpu[0][pts[:, 0] + 256, pts[:, 1] + 256, pts[:, 2]]
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        # terms per output point ~ prod(2m-1) * M / 2 on average; 256^2 * 256 outputs
        per_pt = dt / len(pts)
        nout = 511 * 511 * 256
        return {"value": 1.0 / (per_pt * nout), "unit": "convs/s", "cores": oracle.num_threads(),
                "kind": "oracle", "sample": f"{len(pts)} output points, extrapolated by output count"}, err

    cfg = {"workload": "3D centered Hermitian implicit dealiased convolution, storage 512x512x257 "
                       "(m=256 per axis), M=3 pairs summed, "
                       f"{'complex64' if cdt == torch.complex64 else 'complex128'}",
           "m": list(m), "n": list(n), "M": 3, "dtype": args.dtype}
    return dict(run=run, explicit=None, convs=1, step_bytes=step_bytes, kbytes=kbytes, cfg=cfg,
                cpu=cpu_baseline, out=lambda: run().cpu().numpy())


WORKLOADS = {"c1": wl_c1, "c2": wl_c2, "c3": wl_c3, "c4": wl_c4}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128"])
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-explicit", action="store_true")
    ap.add_argument("--cpu-points", type=int, default=2048)
    ap.add_argument("--cpu-rows", type=int, default=8)
    ap.add_argument("--profile-copy", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported in this build "
              "(the path shards by batch with no exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1008_1366_amd as ic
    ic.lib()  # fail loudly without the HIP library
    torch.cuda.set_device(0)
    W = WORKLOADS[args.workload](args)

    # implicit path, with per-launch event timing inside the library
    ms_clean = timed(W["run"], args.steps, args.warmup)  # the timed region of the metric
    ic.timing_enable(True)  # second pass: per-launch kernel durations
    timed(W["run"], args.steps, 1, backlog=True)
    rep = ic.timing_report()
    ic.timing_enable(False)
    convs_s = W["convs"] * 1000.0 / ms_clean

    kernels = []
    for r in rep:
        avg = r["total_ms"] / max(1, r["count"])
        kernels.append({"name": r["name"], "launches": r["count"], "avg_ms": avg, "total_ms": r["total_ms"]})
    dom = max(kernels, key=lambda k: k["total_ms"]) if kernels else None
    roof = None
    if dom is not None:
        per_launch = W["kbytes"].get(dom["name"])
        traffic = None
        tf = os.path.join(ROOT, "profiles", f"traffic_{args.workload}_{args.dtype}.json")
        if os.path.exists(tf):
            t = json.load(open(tf))
            if t.get("source_hash") == kernel_source_hash() and dom["name"] in t.get("kernels", {}):
                traffic = t["kernels"][dom["name"]]
        if per_launch:
            achieved = per_launch / (dom["avg_ms"] * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom["name"],
                    "kernel_avg_ms": round(dom["avg_ms"], 5), "algorithmic_bytes_per_launch": per_launch}

    out = {"metric": METRIC, "value": round(convs_s, 2), "unit": "convs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_clean, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "fp32" if args.dtype == "c64" else "fp64", "data": "synthetic",
           "config": W["cfg"],
           "hbm_gbps_algorithmic": round(W["step_bytes"] / (ms_clean * 1e-3) / 1e9, 1),
           "kernels": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in kk.items()} for kk in kernels],
           "roofline": roof}

    if W.get("explicit") is not None and not args.no_explicit:
        ms_e = timed(W["explicit"], max(3, args.steps // 2), 1)
        out["explicit_padded"] = {"ms_per_step": round(ms_e, 5), "value": round(W["convs"] * 1000.0 / ms_e, 2),
                                  "unit": "convs/s"}
        out["speedup_vs_explicit"] = round(ms_e / ms_clean, 3)

    if args.profile_copy:
        n = args.profile_copy * (1 << 20) // 4
        x = torch.empty(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_kernel_bytes"] = {"read": n * 4, "write": n * 4}

    if not args.no_cpu:
        h = W["out"]()
        cpu, err = W["cpu"](h)
        out["cpu_baseline"] = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in cpu.items()}
        out["rel_err_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
