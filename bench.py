#!/usr/bin/env python3
"""Benchmark of the implicitly dealiased convolution on one MI355X.

Default workload (c4): the 3D centered Hermitian (2/3 rule) convolution of
the pseudospectral configuration, storage 512 x 512 x 257 (m = 256 per axis,
zero slots), three velocity-vorticity products summed per call (M = 3), in
complex128 (FP64 arithmetic, the paper's precision), with a complex64 leg
(FP32 arithmetic, FP64-generated twiddles) and its error in the same line.
A step is one conv3d call; value = convolutions per second, with inputs
resident in HBM before the timed region.  The explicitly zero-padded
comparator (same FFT kernels, every axis padded to a power of two >= 3m - 2
and materialized in HBM) and its pruned form are timed the same way.

Other workloads (--workload): c1 (1D complex m=1024 complex128, batch 16384),
c2 (1D centered Hermitian m=16384, batch 256), c3 (2D complex 2048^2, batch
8), c5 (4096 uneven 1D complex pairs, forward + backward), t1 (1D Hermitian
ternary m=2048), t2 (2D centered Hermitian ternary, 1024^2 modes, batch 8),
e2 (2D Euler nonlinearity: Hermitian 2D with M = 2, 2048^2 modes).

Output: one JSON line (rank 0) with the metric, per-step time (mean and the
one-sided deviations below and above it), per-kernel algorithmic bytes and
flops, the roofline of the dominant kernel (HIP-event durations recorded by
the library around each launch, on the launch stream), the bandwidth of a
plain device copy for reference, and the FP64 oracle timed on the host on a
bounded sample (the only place bench.py touches the oracle).
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
# Published MI355X vector peaks: FP64 78.6 TFLOP/s, FP32 157.3 TFLOP/s.  The
# FP32 figure counts packed FP32 instructions (two FMAs per lane and cycle),
# which this library is built without, so FP32 kernels also report their
# fraction of the non-packed rate, 256 CUs x 4 SIMDs x 16 lanes x 2 flops x
# 2.4 GHz = 78.6 TFLOP/s.
PEAK_TFLOPS = {"c128": 78.6, "c64": 157.3}
VALU_NONPACKED_TFLOPS = 78.6


def note(msg: str) -> None:
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def flops_row_complex(N: int) -> float:
    """Algorithmic flops of one fused complex row convolution of FFT size N
    (Sec. 2.1): six N-point FFTs at 5 N log2 N, the residue shifts of f and g
    (2N complex products), the residue products (2N) and the recombination
    (N products, N additions, N scalings)."""
    return 6 * 5.0 * N * np.log2(max(N, 2)) + 34.0 * N


def flops_row_ternary(NN: int) -> float:
    """Algorithmic flops of one fused Hermitian ternary row (Sec. 4.2, tconv)
    with packed FFT size NN (real length 2 NN per residue): for each of the
    two residues three c2r and one r2c transform at 2.5 L log2 L (L = 2 NN),
    the residue shifts (3 NN products), the triple real product and the
    recombination."""
    L = 2 * NN
    return 2 * 4 * 2.5 * L * np.log2(max(L, 2)) + 2 * (3 * 6.0 * NN + 4.0 * L) + 8.0 * NN


def flops_row_hermitian(NC: int, M: int = 1) -> float:
    """Algorithmic flops of one fused Hermitian row convolution with NC
    complex modes (m = 2 NC reals per transform, Sec. 2.3): for each of the
    three residues, 2M real-to-complex-sized backward transforms and one
    forward one at 2.5 m log2 m, the residue shifts (2M products of NC), the
    M-dot of real products (2 m M) and the recombination (3 NC products)."""
    m = 2 * NC
    return 3 * (2 * M + 1) * 2.5 * m * np.log2(max(m, 2)) + 3 * (6.0 * 2 * M * NC + 2.0 * m * M) + 3 * 8.0 * NC


# Sources a kernel's traffic depends on: the shared device headers and host
# orchestration, plus its own family (column passes or row kernels).
_SHARED_SOURCES = ("cx.hpp", "fft_wg.hpp", "launch.hpp", "runtime.hpp", "twiddle.hip", "abi.hip",
                   "multid.hip", "multid.hpp", "ragged.hip", "plan.hip", "k_misc.hip")


def kernel_source_hash(kernel: str = "") -> str:
    """Hash of the sources that define `kernel` (all sources if unknown):
    counter readings recorded under one hash are void once it changes."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1008_1366_amd", "csrc")
    if kernel.startswith("colpass"):
        own = lambda fn: fn == "colpass.hpp" or fn.startswith("k_col_")
    elif kernel.startswith("k_conv1d"):
        own = lambda fn: fn in ("rowconv.hpp", "queue.hpp") or fn.startswith("k_row_")
    else:
        own = lambda fn: True
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hpp", ".hip")) and (fn in _SHARED_SOURCES or own(fn)):
            h.update(fn.encode())
            h.update(open(os.path.join(csrc, fn), "rb").read())
    return h.hexdigest()[:16]


def fp32_vs_fp64(h32, run64):
    """Relative L2 difference, per pair over the whole field, between the
    complex64 result h32 (host array, pairs on axis 0) and the complex128
    path run on the GPU on the same (complex64-rounded) inputs; the FP64
    result is itself checked against the oracle in the FP64 runs and tests."""
    import torch
    h64 = run64().cpu().numpy()
    torch.cuda.empty_cache()
    e = [float(np.linalg.norm(h32[b].astype(np.complex128) - h64[b]) / np.linalg.norm(h64[b]))
         for b in range(h64.shape[0])]
    return {"max": max(e), "median": float(np.median(e)), "pairs": len(e)}


def oracle_one_thread(fn, budget_s=2.0):
    """Seconds per call of fn with the oracle on one host thread (repeated up
    to about budget_s), the thread count restored afterwards."""
    import oracle
    n0 = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        calls, t0 = 0, time.perf_counter()
        while True:
            fn()
            calls += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        return (time.perf_counter() - t0) / calls
    finally:
        oracle.set_num_threads(n0)


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


def step_stats(fn, n):
    """Per-step times (events around each step): the mean T and the one-sided
    deviations of the paper's timing statistics, sigma_L (sigma_H) the square
    root of the summed squared deviations of the steps below (above) T
    divided by n/2 - 1."""
    import torch
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
    torch.cuda.synchronize()
    ev[0].record(s)
    for i in range(n):
        fn()
        ev[i + 1].record(s)
    torch.cuda.synchronize()
    t = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(n)])
    mu = t.mean()
    lo, hi = t[t < mu], t[t > mu]
    one_sided = lambda d: float(np.sqrt(np.sum(d ** 2) / (n / 2.0 - 1.0)))
    return {"n": n, "mean_ms": round(float(mu), 5), "sigma_lo_ms": round(one_sided(mu - lo), 5),
            "sigma_hi_ms": round(one_sided(hi - mu), 5)}


def copy_bandwidth(mib=1024):
    """Bandwidth of a plain device-to-device copy (read + write bytes / time)."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    ms = timed(lambda: y.copy_(x), 10, 2)
    del x, y
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


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
    pruned = lambda: ic.conv2d(F, G, method="pruned")
    comp = (lambda: ic.conv2d(F, G, flags=ic.COMPENSATED)) if cdt == torch.complex64 else None
    # algorithmic bytes: every column pass moves 3 S per launch (Sec. 3.1
    # schedule); the rows of both x residues (2 m_x rows per pair, 3 S per
    # residue) run in one launch
    kbytes = {"colpass_pad_bwd": 3 * S, "colpass_pad_fwd": 3 * S}
    kbytes_step = {"k_conv1d_complex": 6 * S}
    kflops_step = {"k_conv1d_complex": 2 * B * mx * flops_row_complex(my)}
    step_bytes = 15 * S

    def cpu_baseline(h_gpu, h_expl=None, h_comp=None):
        """Oracle at stratified sample points of every pair: the whole
        low-wavenumber block [0,L)^2 (where the energy of the (1+|k|^2)^-1
        spectra concentrates) plus uniform random points elsewhere.  The
        strata weights give an estimate of each pair's full-field relative
        L2 error (reported as max and median over the pairs, for the implicit
        result and the explicitly padded one); the time gives the oracle's
        rate, extrapolated by multiply-add count."""
        import oracle
        rng = synth.rng(7)
        L = 16
        blk = np.array([(i, j) for i in range(L) for j in range(L)])
        nrand = max(1, args.cpu_points // B)
        dt_np = np.complex64 if cdt == torch.complex64 else np.complex128
        macs = 0.0
        t_oracle = 0.0
        res = {"implicit": [], "explicit": [], "compensated": [], "uniform_random_points": []}
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
            r2 = np.abs(ref) ** 2
            wb = (mx * my - L * L) / len(rp)
            for key, h in (("implicit", h_gpu), ("explicit", h_expl), ("compensated", h_comp)):
                if h is None:
                    continue
                e2 = np.abs(h[b][pts[:, 0], pts[:, 1]] - ref) ** 2
                num = e2[:len(blk)].sum() + wb * e2[len(blk):].sum()
                den = r2[:len(blk)].sum() + wb * r2[len(blk):].sum()
                res[key].append(float(np.sqrt(num / den)))
                if key == "implicit":
                    res["uniform_random_points"].append(float(np.sqrt(e2[len(blk):].sum() / r2[len(blk):].sum())))
        full = (mx * (mx + 1) / 2.0) * (my * (my + 1) / 2.0)
        convs_per_s = 1.0 / (t_oracle / macs * full)
        errs = {k: {"max": max(v), "median": float(np.median(v)), "pairs": len(v)} for k, v in res.items() if v}
        errs["estimate"] = "full-field relative L2 per pair, from the stratified sample"
        if cdt == torch.complex64:
            errs["fp32_vs_fp64_full_field"] = fp32_vs_fp64(
                h_gpu, lambda: ic.conv2d(F.to(torch.complex128), G.to(torch.complex128)))
        return {"value": convs_per_s, "unit": "convs/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"per pair the {L}x{L} low-wavenumber block plus {nrand} uniform random "
                          f"output points, direct FP64 sums ({t_oracle:.2f} s), extrapolated to whole "
                          f"convolutions by multiply-add count"}, errs

    cfg = {"workload": f"2D complex implicit dealiased convolution {mx}x{my}, batch {B} pairs per step, "
                       f"{'complex64' if cdt == torch.complex64 else 'complex128'}",
           "m": [mx, my], "batch": B, "M": 1, "dtype": args.dtype}
    return dict(run=run, explicit=expl, pruned=pruned, compensated=comp, convs=B, step_bytes=step_bytes,
                kbytes=kbytes, kbytes_step=kbytes_step, kflops_step=kflops_step, cfg=cfg, cpu=cpu_baseline,
                out=lambda: run().cpu().numpy())


def wl_x3(args):
    """3D complex 256^3 (Sec. 3.4's complex 3D timing comparison), batch of 2
    pairs of unit-disk inputs: implicit against the explicitly padded
    comparator (2m per axis) and its pruned form."""
    import torch
    import paper_1008_1366_amd as ic
    import synth
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    m, B = 256, args.batch or 2
    f = synth.unit_disk((B, m, m, m), 301)
    g = synth.unit_disk((B, m, m, m), 302)
    F = torch.from_numpy(f).to("cuda", cdt)
    G = torch.from_numpy(g).to("cuda", cdt)
    del f, g
    cs = 8 if cdt == torch.complex64 else 16
    S = B * m ** 3 * cs  # one stored batch of inputs
    run = lambda: ic.conv3d(F, G)
    expl = lambda: ic.conv3d(F, G, method="explicit")
    pruned = lambda: ic.conv3d(F, G, method="pruned")
    # algorithmic bytes per step (m a power of two, so every residue array
    # has the input's size S): x backward f, g 2S -> 4S; y backward 4S -> 8S;
    # z rows 8S -> 4S; y forward 4S -> 2S; x forward 2S -> S
    step_bytes = 39 * S

    def cpu_baseline(h_gpu, h_expl=None):
        """Oracle direct sums at 32 seeded output points of the first pair
        (about m^3 / 8 multiply-adds each on average), extrapolated to the
        whole step by multiply-add count; errors at those points."""
        import oracle
        rng = synth.rng(8)
        pts = rng.integers(0, m, (32, 3))
        dt_np = np.complex64 if cdt == torch.complex64 else np.complex128
        fr = np.asarray(F[0].cpu().numpy().astype(dt_np), np.complex128)
        gr = np.asarray(G[0].cpu().numpy().astype(dt_np), np.complex128)
        t0 = time.perf_counter()
        ref = oracle.convnd_complex_at(fr, gr, pts)
        t = time.perf_counter() - t0
        macs = float(np.sum(np.prod(pts + 1.0, axis=1)))
        full = B * (m * (m + 1) / 2.0) ** 3
        errs = {"implicit": float(np.linalg.norm(h_gpu[0][tuple(pts.T)] - ref) / np.linalg.norm(ref)), "points": 32}
        if h_expl is not None:
            errs["explicit"] = float(np.linalg.norm(h_expl[0][tuple(pts.T)] - ref) / np.linalg.norm(ref))
        return {"value": B / (t / macs * full), "unit": "convs/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"32 output points of the first pair, direct FP64 sums ({t:.2f} s), extrapolated "
                          f"to whole convolutions by multiply-add count"}, errs

    cfg = {"workload": f"3D complex implicit dealiased convolution {m}^3, batch {B} pairs per step, "
                       f"{'complex64' if cdt == torch.complex64 else 'complex128'}",
           "m": [m, m, m], "batch": B, "M": 1, "dtype": args.dtype}
    return dict(run=run, explicit=expl, pruned=pruned, convs=B, step_bytes=step_bytes, kbytes={}, kflops={},
                cfg=cfg, cpu=cpu_baseline, out=lambda: run().cpu().numpy(), bound="hbm")


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
    kflops = {"k_conv1d_hermitian": B * flops_row_hermitian(m // 2)}

    def cpu_baseline(h_gpu):
        import oracle
        nb = min(B, args.cpu_rows or 256)
        fr = np.asarray(f[:nb].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)
        gr = np.asarray(g[:nb].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)
        t0 = time.perf_counter()
        ref = oracle.conv1d_hermitian(fr[:, None], gr[:, None])
        dt = time.perf_counter() - t0
        err = float(np.linalg.norm(h_gpu[:nb] - ref) / np.linalg.norm(ref))
        t1 = oracle_one_thread(lambda: oracle.conv1d_hermitian(fr[:1, None], gr[:1, None]))
        return {"value": nb / dt, "unit": "convs/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{nb} of the {B} convolutions, direct FP64 sums ({dt:.2f} s)",
                "one_thread_s_per_conv": t1}, err

    cfg = {"workload": f"1D centered Hermitian implicit dealiased convolution m={m}, batch {B}, "
                       f"{'complex64' if cdt == torch.complex64 else 'complex128'}",
           "m": m, "batch": B, "dtype": args.dtype}
    expl = None
    F1, G1 = F[:1].contiguous(), G[:1].contiguous()
    single = {"run": lambda: ic.conv1d_hermitian(F1, G1), "explicit": None,
              "note": "one convolution (one workgroup): latency-bound"}
    return dict(run=run, explicit=expl, convs=B, step_bytes=3 * B * m * cs, kbytes=kbytes, kflops=kflops,
                cfg=cfg, cpu=cpu_baseline, out=lambda: run().cpu().numpy(), single=single)


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
    pruned = lambda: ic.conv1d_complex(F, G, method="pruned")
    comp = (lambda: ic.conv1d_complex(F, G, flags=ic.COMPENSATED)) if cdt == torch.complex64 else None
    kbytes = {"k_conv1d_complex": 3 * B * m * cs}
    kflops = {"k_conv1d_complex": B * flops_row_complex(m)}

    def cpu_baseline(h_gpu, h_expl=None, h_comp=None):
        import oracle
        nb = min(B, args.cpu_rows or 8192)
        t0 = time.perf_counter()
        ref = oracle.conv1d_complex(np.asarray(f[:nb].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)[:, None],
                                    np.asarray(g[:nb].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)[:, None])
        dt = time.perf_counter() - t0
        err = {}
        for key, h in (("implicit", h_gpu), ("explicit", h_expl), ("compensated", h_comp)):
            if h is not None:
                e = [float(np.linalg.norm(h[i] - ref[i]) / np.linalg.norm(ref[i])) for i in range(nb)]
                err[key] = {"max": max(e), "median": float(np.median(e)), "pairs": nb}
        f1 = np.asarray(f[:1].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)
        g1 = np.asarray(g[:1].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)
        t1 = oracle_one_thread(lambda: oracle.conv1d_complex(f1[:, None], g1[:, None]))
        return {"value": nb / dt, "unit": "convs/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{nb} of the {B} pairs, direct FP64 sums ({dt:.2f} s)",
                "one_thread_s_per_conv": t1}, err

    cfg = {"workload": f"1D complex implicit dealiased convolution m={m}, batch {B}, "
                       f"{'complex64' if cdt == torch.complex64 else 'complex128'}", "m": m, "batch": B,
           "dtype": args.dtype}
    F1, G1 = F[:1].contiguous(), G[:1].contiguous()
    single = {"run": lambda: ic.conv1d_complex(F1, G1), "explicit": lambda: ic.conv1d_complex(F1, G1, method="explicit"),
              "note": "one pair (one workgroup): latency-bound"}
    return dict(run=run, explicit=expl, pruned=pruned, compensated=comp, convs=B, step_bytes=3 * B * m * cs, kbytes=kbytes,
                kflops=kflops, cfg=cfg, cpu=cpu_baseline, out=lambda: run().cpu().numpy(), single=single)


def numpy_explicit_hermitian_3d(f, g, m, workers):
    """FP64 explicitly padded FFT convolution on the host (scipy.fft, i.e.
    pocketfft): every axis padded to 3m (the 2/3 rule's size; wavenumber k
    of a centered axis at index k mod 3m, the last axis the half spectrum of
    a real length 3m), the M-dot of the physical-space products, one forward
    real transform, crop.  f, g: [M][2m][2m][m+1] in the library's storage
    (index k + m on the centered axes).  Returns h in that storage."""
    import scipy.fft as sf
    M = f.shape[0]
    P = [3 * x for x in m]
    k0 = np.arange(-(m[0] - 1), m[0])
    k1 = np.arange(-(m[1] - 1), m[1])
    src = np.ix_(k0 + f.shape[1] - m[0], k1 + f.shape[2] - m[1], np.arange(m[2]))
    dst = np.ix_(k0 % P[0], k1 % P[1], np.arange(m[2]))
    buf = np.zeros((P[0], P[1], P[2] // 2 + 1), np.complex128)
    acc = None
    for i in range(M):
        buf[dst] = f[i][src]
        a = sf.irfftn(buf, s=P, workers=workers)
        buf[dst] = g[i][src]
        a *= sf.irfftn(buf, s=P, workers=workers)
        acc = a if acc is None else acc + a
        del a
    H = sf.rfftn(acc, workers=workers)
    del acc
    H *= float(np.prod(P))  # irfftn's 1/N on each factor, rfftn's none
    h = np.zeros(f.shape[1:], np.complex128)
    h[src] = H[dst]
    return h


def wl_c4(args):
    """3D centered Hermitian, storage 512x512x257 (m=256/axis), M=3 pairs
    summed: the headline workload, complex128 by default, with a complex64
    leg (FP64-generated twiddles) timed in the same run."""
    import torch
    import paper_1008_1366_amd as ic
    import synth
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    m, n = (256, 256, 256), (512, 512, 257)

    def hermitian_plane(u):
        # the k_z = 0 plane made Hermitian on the host by the library's own
        # rule (authoritative: k_x > 0, or k_x = 0 and k_y > 0; origin real),
        # which leaves the implicit result unchanged and lets the explicit
        # comparator, whose real transforms read that plane's Hermitian
        # projection, see the same field
        q = u[1:, 1:, 0]
        kx = np.arange(-255, 256)[:, None]
        ky = np.arange(-255, 256)[None, :]
        auth = (kx > 0) | ((kx == 0) & (ky > 0))
        q[...] = np.where(auth, q, np.conj(q[::-1, ::-1]))
        q[255, 255] = q[255, 255].real
        return u

    f = np.stack([hermitian_plane(synth.power_spectrum_centered(m, n, 11 / 6, 200 + i)) for i in range(3)])[None]
    g = np.stack([hermitian_plane(synth.power_spectrum_centered(m, n, 11 / 6, 203 + i)) for i in range(3)])[None]
    F = torch.from_numpy(f).to("cuda", cdt)
    G = torch.from_numpy(g).to("cuda", cdt)
    cs = 8 if cdt == torch.complex64 else 16
    S = int(np.prod(n)) * cs
    # the per-launch timing pass runs every launch in order on one stream
    # (ONE_STREAM: same kernels), so that a launch's duration is its own and
    # not shared with the rows of one chunk that overlap the next chunk's y pass
    mode = {"flags": 0}
    run = lambda: ic.conv3d(F, G, kind="hermitian", m=m, flags=mode["flags"])
    expl = lambda: ic.conv3d(F, G, kind="hermitian", m=m, method="explicit")
    pruned = lambda: ic.conv3d(F, G, kind="hermitian", m=m, method="pruned")

    def kernel_timing_mode(on):
        mode["flags"] = ic.ONE_STREAM if on else 0
        return "launches in order on one stream (ONE_STREAM) for the per-launch timing pass" if on else None
    # Sec. 3.4 five-pass schedule, algorithmic bytes per step (S = one stored
    # array): x back 6S -> 9S and y back 9S -> 13.5S (colpass_cen_bwd), z
    # convolutions 13.5S -> 2.25S (3 m_x x 3 m_y rows, M = 3 per row), y
    # forward 2.25S -> 1.5S and x forward 1.5S -> S (colpass_cen_fwd)
    kbytes_step = {"colpass_cen_bwd": int(37.5 * S), "k_conv1d_hermitian": int(15.75 * S),
                   "colpass_cen_fwd": int(6.25 * S)}
    kflops_step = {"k_conv1d_hermitian": 9 * m[0] * m[1] * flops_row_hermitian(m[2] // 2, 3)}
    step_bytes = int(59.5 * S)

    def oracle_points():
        rng = synth.rng(206)
        return np.concatenate([[[0, 0, 0], [255, 255, 255], [-255, 0, 3], [5, -7, 0], [-3, 9, 0], [0, -200, 0]],
                               np.stack([rng.integers(-255, 256, 10), rng.integers(-255, 256, 10),
                                         rng.integers(0, 256, 10)], 1)])

    def sampled_err(hh, pts, ref):
        got = hh[0][pts[:, 0] + 256, pts[:, 1] + 256, pts[:, 2]]
        return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    def cpu_baseline(h_gpu, h_expl=None):
        import oracle
        pts = oracle_points()
        fr = np.asarray(f[0].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)
        gr = np.asarray(g[0].astype(np.complex64 if cdt == torch.complex64 else np.complex128), np.complex128)
        t0 = time.perf_counter()
        ref = oracle.convnd_hermitian_at(fr, gr, m, pts)
        dt = time.perf_counter() - t0
        err = {}
        for key, hh in (("implicit", h_gpu), ("explicit", h_expl)):
            if hh is not None:
                err[key] = sampled_err(hh, pts, ref)
        err["points"] = len(pts)
        if cdt == torch.complex64:
            err["fp32_vs_fp64_full_field"] = fp32_vs_fp64(
                h_gpu, lambda: ic.conv3d(F.to(torch.complex128), G.to(torch.complex128), kind="hermitian", m=m))
        # terms per output point ~ prod(2m-1) * M / 2 on average; 256^2 * 256 outputs
        per_pt = dt / len(pts)
        nout = 511 * 511 * 256
        cpu = {"value": 1.0 / (per_pt * nout), "unit": "convs/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": f"{len(pts)} output points ({dt:.2f} s), extrapolated to the whole "
                                           "convolution by output count"}
        if not args.no_numpy:
            # the practical CPU method: FP64 explicitly padded FFT convolution
            # (scipy.fft) of the same inputs, whole field, timed once
            workers = len(os.sched_getaffinity(0))
            t0 = time.perf_counter()
            hn = numpy_explicit_hermitian_3d(fr, gr, m, workers)
            tn = time.perf_counter() - t0
            cpu["numpy_explicit_fp64"] = {"value": 1.0 / tn, "unit": "convs/s", "seconds_per_conv": tn,
                                          "cores": workers, "padded_size": [3 * x for x in m],
                                          "rel_err_at_oracle_points": sampled_err(hn[None], pts, ref)}
            err["implicit_vs_numpy_full_field"] = float(np.linalg.norm(h_gpu[0] - hn) / np.linalg.norm(hn))
            del hn
        return cpu, err

    def c64_leg():
        """The complex64 path on the same inputs (rounded), timed like the
        headline, with its error over the whole field against the complex128
        result of the library (itself checked against the oracle) and at the
        oracle's sampled points."""
        import oracle
        if cdt == torch.complex64:
            return None
        F32, G32 = F.to(torch.complex64), G.to(torch.complex64)
        run32 = lambda: ic.conv3d(F32, G32, kind="hermitian", m=m)
        ms32 = timed(run32, args.steps, args.warmup)
        h32 = run32().cpu().numpy()
        h64 = ic.conv3d(F32.to(torch.complex128), G32.to(torch.complex128), kind="hermitian", m=m).cpu().numpy()
        e_full = float(np.linalg.norm(h32.astype(np.complex128) - h64) / np.linalg.norm(h64))
        pts = oracle_points()
        fr = np.asarray(f[0].astype(np.complex64), np.complex128)
        gr = np.asarray(g[0].astype(np.complex64), np.complex128)
        e_pts = sampled_err(h32, pts, oracle.convnd_hermitian_at(fr, gr, m, pts))
        S32 = int(np.prod(n)) * 8
        del F32, G32, h32, h64
        torch.cuda.empty_cache()
        return {"dtype": "fp32 (complex64, FP64-generated twiddles)", "ms_per_step": round(ms32, 5),
                "value": round(1000.0 / ms32, 2), "unit": "convs/s",
                "hbm_gbps_algorithmic": round(59.5 * S32 / (ms32 * 1e-3) / 1e9, 1),
                "rel_err_vs_fp64_full_field": e_full, "rel_err_vs_oracle_sampled": e_pts}

    cfg = {"workload": "3D centered Hermitian implicit dealiased convolution, storage 512x512x257 "
                       "(m=256 per axis), M=3 pairs summed, "
                       f"{'complex64' if cdt == torch.complex64 else 'complex128'}",
           "m": list(m), "n": list(n), "M": 3, "dtype": args.dtype}
    return dict(run=run, explicit=expl, pruned=pruned, convs=1, step_bytes=step_bytes, kbytes_step=kbytes_step,
                kflops_step=kflops_step, cfg=cfg, cpu=cpu_baseline, out=lambda: run().cpu().numpy(),
                bound="hbm", leg=c64_leg, kernel_timing_mode=kernel_timing_mode)


def wl_c5(args):
    """4096 uneven complex 1D pairs, m = 2^round(U(6,16)), packed end to end;
    one step = forward and backward (both input gradients) through the
    differentiable ragged wrapper for the loss L = Re sum conj(w) h, whose
    upstream gradient dL/dh is w."""
    import torch
    import paper_1008_1366_amd as ic
    import synth
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    dt_np = np.complex64 if cdt == torch.complex64 else np.complex128
    ms = synth.ragged_lengths(4096, 6, 16, 5)
    offs = np.concatenate([[0], np.cumsum(ms)[:-1]])
    tot = int(ms.sum())
    f = synth.unit_disk(tot, 9)
    g = synth.unit_disk(tot, 10)
    w = synth.unit_disk(tot, 11)
    F = torch.from_numpy(f).to("cuda", cdt).requires_grad_(True)
    G = torch.from_numpy(g).to("cuda", cdt).requires_grad_(True)
    Wt = torch.from_numpy(w).to("cuda", cdt)
    # schedule: the four-step split of each long class is autotuned at plan
    # creation, outside the timed region
    plan = ic.RaggedPlan(ms, offs, dtype=cdt, autotune=not args.no_autotune)
    info = plan.schedule_info()
    sched = [{k: c[k] for k in ("N", "pairs", "method", "E", "N1", "N2", "source") if k in c} for c in info["classes"]]
    cs = 8 if cdt == torch.complex64 else 16

    def run():
        F.grad = None
        G.grad = None
        h = ic.ragged_conv_ad(plan, F, G)
        h.backward(Wt)
        return h

    # algorithmic bytes per step and kernel: pairs with N = 2^ceil(log2 m)
    # <= 8192 run the fused row kernel (reads f, g, writes h); longer ones the
    # four-step form (pass 1 reads m and writes two N-point residues per
    # input, pass 2 reads four and writes two residues, pass 3 reads two and
    # writes m).  Three executions per step: forward, grad f, grad g.
    Ns = 2 ** np.ceil(np.log2(ms)).astype(np.int64)
    small = Ns <= 8192
    # the fused classes run as one work-queue launch (k_ragged_queue) or one
    # k_conv1d_complex launch per class, as the autotuner chose
    qd = small & (Ns <= (8192 if cdt == torch.complex64 else 4096)) if info["fused_launch"] == "queue" else small & False
    kb = {"k_conv1d_complex": 3 * int(ms[small & ~qd].sum()) * cs,
          "k_ragged_queue": 3 * int(ms[qd].sum()) * cs,
          "colpass_fourstep_bwd": 2 * int((ms[~small] + 2 * Ns[~small]).sum()) * cs,
          "k_conv1d_cyclic": 6 * int(Ns[~small].sum()) * cs,
          "colpass_fourstep_fwd": int((2 * Ns[~small] + ms[~small]).sum()) * cs}
    kbytes_step = {k: 3 * v for k, v in kb.items()}
    kflops_step = {"k_conv1d_complex": 3 * float(sum(flops_row_complex(int(n)) for n in Ns[small & ~qd])),
                   "k_ragged_queue": 3 * float(sum(flops_row_complex(int(n)) for n in Ns[qd]))}
    step_bytes = 9 * tot * cs  # compulsory: f, g, h of each execution

    def cpu_baseline(h_gpu):
        """Oracle forward and both gradients of the pairs with m <= 8192, in
        pair order up to a multiply-add budget, extrapolated to the whole
        step by multiply-add count; errors of the GPU forward and gradients
        on those pairs and at sampled outputs of the longest pairs."""
        import oracle
        gf = F.grad.detach().cpu().numpy()
        gg = G.grad.detach().cpu().numpy()
        fr, gr, wr = (np.asarray(a.astype(dt_np), np.complex128) for a in (f, g, w))
        cand = np.where(ms <= 8192)[0]
        budget = args.cpu_macs  # multiply-adds of the oracle sample
        cum = np.cumsum(3 * ms[cand] * (ms[cand] + 1) / 2.0)
        sel = cand[cum <= budget] if cum[0] <= budget else cand[:1]
        t_or = 0.0
        macs = 0.0
        errs = {"h": [], "grad_f": [], "grad_g": []}
        for j in sel:
            o, m = offs[j], ms[j]
            t0 = time.perf_counter()
            ref = oracle.conv1d_complex(fr[o:o + m], gr[o:o + m])
            rf, rg = oracle.grad_conv1d_complex(fr[o:o + m], gr[o:o + m], wr[o:o + m])
            t_or += time.perf_counter() - t0
            macs += 3 * m * (m + 1) / 2.0
            for key, got, r in (("h", h_gpu[o:o + m], ref), ("grad_f", gf[o:o + m], rf), ("grad_g", gg[o:o + m], rg)):
                errs[key].append(float(np.linalg.norm(got - r) / np.linalg.norm(r)))
        big = np.argsort(ms)[-4:]
        for j in big:
            o, m = offs[j], ms[j]
            ks = np.array([0, 1, m // 2, m - 1])
            r = oracle.convnd_complex_at(fr[o:o + m], gr[o:o + m], ks[:, None])
            errs["h"].append(float(np.linalg.norm(h_gpu[o + ks] - r) / np.linalg.norm(r)))
        full = float(np.sum(3 * ms * (ms + 1) / 2.0))
        err = {k: {"max": max(v), "median": float(np.median(v)), "pairs": len(v)} for k, v in errs.items()}
        return {"value": len(ms) / (t_or / macs * full), "unit": "convs/s", "cores": oracle.num_threads(),
                "kind": "oracle",
                "sample": f"forward + both gradients of {len(sel)} pairs with m <= 8192, direct FP64 sums "
                          f"({t_or:.2f} s), extrapolated to the whole step by multiply-add count"}, err

    cfg = {"workload": f"{len(ms)} uneven complex 1D pairs, m = 2^round(U(6,16)), packed, forward + backward "
                       f"(both gradients) per step, {'complex64' if cdt == torch.complex64 else 'complex128'}",
           "pairs": int(len(ms)), "sum_m": tot, "dtype": args.dtype, "schedule": sched,
           "fused_launch": info["fused_launch"], "fused_tuned_ms": info.get("fused_tuned_ms"),
           "autotuned": not args.no_autotune}
    def graph_step():
        """The same step captured once in a hipGraph (forward, backward and
        the gradient buffers); returns the replay and a check that a replay
        reproduces the eager outputs bit for bit."""
        run()
        torch.cuda.synchronize()
        h_eager = run().detach().clone()
        gf_eager, gg_eager = F.grad.clone(), G.grad.clone()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(graph, stream=side):
            F.grad = None
            G.grad = None
            h_static = ic.ragged_conv_ad(plan, F, G)
            h_static.backward(Wt)
        torch.cuda.synchronize()

        def check():
            graph.replay()
            torch.cuda.synchronize()
            return bool(torch.equal(h_static, h_eager) and torch.equal(F.grad, gf_eager)
                        and torch.equal(G.grad, gg_eager))
        return graph.replay, check

    def kernel_timing_mode(on):
        """Per-launch timing pass: the size classes one after another on one
        stream (ONE_STREAM, same kernels), so that each launch's duration is
        its own and not shared with the classes that overlap it."""
        plan.one_stream = on
        return "size classes serialized on one stream (ONE_STREAM) for the per-launch timing pass" if on else None

    return dict(run=run, explicit=None, convs=len(ms), step_bytes=step_bytes, kbytes_step=kbytes_step,
                kflops_step=kflops_step, cfg=cfg, cpu=cpu_baseline, out=lambda: run().detach().cpu().numpy(),
                graph=graph_step, kernel_timing_mode=kernel_timing_mode)


def wl_t2(args):
    """2D centered Hermitian ternary convolution (Sec. 4, tconv2) of three
    fields per pair: m = (M, M) modes, storage (2M, M + 1), batch B, spectra
    |k|^-1 with random phase and a Hermitian k_y = 0 line."""
    import torch
    import paper_1008_1366_amd as ic
    import synth
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    dt_np = np.complex64 if cdt == torch.complex64 else np.complex128
    mm = args.t2_m
    m, n = (mm, mm), (2 * mm, mm + 1)
    B = args.batch or 8

    def field(mv, nv, seed):
        u = synth.power_spectrum_centered(mv, nv, 1.0, seed)
        off = nv[0] - mv[0]
        u[off - np.arange(1, mv[0]), 0] = np.conj(u[off + np.arange(1, mv[0]), 0])
        return u

    fs = [np.stack([field(m, n, 400 + 3 * b + q) for b in range(B)]) for q in range(3)]
    F, G, E = (torch.from_numpy(x).to("cuda", cdt) for x in fs)
    cs = 8 if cdt == torch.complex64 else 16
    S = B * n[0] * n[1] * cs
    run = lambda: ic.conv2d_ternary(F, G, E, m)
    # the comparator's x transforms have 4 N0' points: up to 16384 (complex64)
    # or 4096 (complex128)
    cmp_ok = mm <= (4096 if cdt == torch.complex64 else 1024)
    expl = (lambda: ic.conv2d_ternary(F, G, E, m, method="explicit")) if cmp_ok else None
    pruned = (lambda: ic.conv2d_ternary(F, G, E, m, method="pruned")) if cmp_ok else None
    P0 = 2 * (1 << int(np.ceil(np.log2(mm))))
    # per launch: x backward reads one input (S) and writes two residues (2S);
    # rows read three residue arrays and write one; x forward reads 2S, writes S
    kbytes = {"colpass_ter_bwd": 3 * S, "k_conv1d_ternary": 4 * S, "colpass_ter_fwd": 3 * S}
    kflops = {"k_conv1d_ternary": B * P0 * flops_row_ternary(1 << int(np.ceil(np.log2(mm))))}
    step_bytes = 20 * S

    def cpu_baseline(h_gpu, h_expl=None):
        """The oracle's direct sum costs O(|box|^2) per output (1.8e13
        multiply-adds per point at M = 1024), so it is timed on the full
        field of a reduced instance of the same recipe (M = 20) and its rate
        extrapolated by multiply-add count.  Errors at full size: a rank-one
        triple (U = A (x) b per field) against outer products of a numpy
        centered ternary sum in x and the 1D ternary oracle in y; on the
        reduced instance, the full field of the GPU result."""
        import oracle
        ms_, ns_ = (20, 20), (40, 21)
        small = [field(ms_, ns_, 500 + q) for q in range(3)]
        sr = [np.asarray(x.astype(dt_np), np.complex128) for x in small]
        t0 = time.perf_counter()
        ref = oracle.convnd_ternary(*sr, ms_)
        t_or = time.perf_counter() - t0
        box = (2 * ms_[0] - 1) * (2 * ms_[1] - 1)
        macs_small = box * box * ms_[0] * (2 * ms_[0] - 1) / 2.0  # ~ |box|^2 / 2 per output, half the outputs
        boxf = (2 * mm - 1) ** 2
        macs_full = boxf * boxf * mm * (2 * mm - 1) / 2.0
        hs = ic.conv2d_ternary(*(torch.from_numpy(x).to("cuda", cdt) for x in small), ms_).cpu().numpy()
        err_small = float(np.linalg.norm(hs - ref) / np.linalg.norm(ref))
        # rank-one triple at full size
        vecs, ys, us = [], [], []
        for q in range(3):
            a = synth.unit_disk(mm, 511 + q)
            a[0] = a[0].real
            A = np.concatenate([np.conj(a[:0:-1]), a])
            b = synth.unit_disk(mm, 521 + q)
            b[0] = b[0].real
            u = np.zeros(n, complex)
            u[1:, :mm] = np.outer(A, b)
            vecs.append(np.asarray(A.astype(dt_np), np.complex128))
            ys.append(np.asarray(b.astype(dt_np), np.complex128))
            us.append(u)
        h1 = ic.conv2d_ternary(*(torch.from_numpy(u).to("cuda", cdt) for u in us), m).cpu().numpy()
        xfull = np.convolve(np.convolve(vecs[0], vecs[1]), vecs[2])[2 * (mm - 1):4 * (mm - 1) + 1]
        if mm <= 1024:
            yref = oracle.conv1d_ternary(*ys)
        else:
            # the oracle's direct triple sum is O(m^3); the same sum over the
            # conjugate-extended halves by two numpy convolutions, k = 0..m-1
            yf = [np.concatenate([np.conj(b[:0:-1]), b]) for b in ys]
            yref = np.convolve(np.convolve(yf[0], yf[1]), yf[2])[3 * (mm - 1):3 * (mm - 1) + mm]
        r1 = np.zeros(n, complex)
        r1[1:, :mm] = np.outer(xfull, yref)
        err = {"rank_one_full_field": float(np.linalg.norm(h1 - r1) / np.linalg.norm(r1)),
               "reduced_instance_full_field": err_small}
        return {"value": 1.0 / (t_or / macs_small * macs_full), "unit": "convs/s", "cores": oracle.num_threads(),
                "kind": "oracle",
                "sample": f"full field of a {ms_[0]}x{ms_[1]} instance of the same recipe ({t_or:.2f} s), "
                          f"extrapolated to M = {mm} by multiply-add count"}, err

    cfg = {"workload": f"2D centered Hermitian ternary convolution (tconv2) {mm}x{mm} modes, storage "
                       f"{n[0]}x{n[1]}, batch {B} triples per step, "
                       f"{'complex64' if cdt == torch.complex64 else 'complex128'}",
           "m": list(m), "n": list(n), "batch": B, "dtype": args.dtype}
    return dict(run=run, explicit=expl, pruned=pruned, convs=B, step_bytes=step_bytes, kbytes=kbytes,
                kflops=kflops, cfg=cfg, cpu=cpu_baseline, out=lambda: run().cpu().numpy())


def wl_e2(args):
    """Nonlinear term of the 2D incompressible Euler equations in vorticity
    form (Sec. 3.3): one centered Hermitian 2D convolution with M = 2,
    f = (i k_x w, i k_y w), g = (i k_y w / k^2, -i k_x w / k^2), for a
    vorticity spectrum w ~ |k|^-1 (random phase, Hermitian k_y = 0 line) on
    m = (M, M) modes, storage (2M, M + 1)."""
    import torch
    import paper_1008_1366_amd as ic
    import synth
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    dt_np = np.complex64 if cdt == torch.complex64 else np.complex128
    mm = args.e2_m
    m, n = (mm, mm), (2 * mm, mm + 1)
    w = synth.power_spectrum_centered(m, n, 1.0, 700)
    off = n[0] - mm
    ks = np.arange(1, mm)
    w[off - ks, 0] = np.conj(w[off + ks, 0])
    kx = (np.arange(n[0]) - off)[:, None].astype(np.float64)
    ky = np.arange(n[1])[None, :].astype(np.float64)
    k2 = kx * kx + ky * ky
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    f = np.stack([1j * kx * w, 1j * ky * w])[None]
    g = np.stack([1j * ky * w * inv, -1j * kx * w * inv])[None]
    del kx, ky, k2, inv
    F = torch.from_numpy(f).to("cuda", cdt)
    G = torch.from_numpy(g).to("cuda", cdt)
    cs = 8 if cdt == torch.complex64 else 16
    S = n[0] * n[1] * cs
    run = lambda: ic.conv2d(F, G, kind="hermitian", m=m)
    N0 = 1 << int(np.ceil(np.log2(mm)))
    NC = max(1 << int(np.ceil(np.log2(mm))), 2) // 2
    # per step (S = one stored array): x backward reads 2S (M = 2) and writes
    # three half-size residues per term (3S) for f and for g; each of the
    # three row launches reads 2S and writes S/2; the x forward reads 1.5S and
    # writes S
    kbytes_step = {"colpass_cen_bwd": int(10 * S), "k_conv1d_hermitian": int(7.5 * S),
                   "colpass_cen_fwd": int(2.5 * S)}
    kflops_step = {"k_conv1d_hermitian": 3 * N0 * flops_row_hermitian(NC, 2)}

    def cpu_baseline(h_gpu):
        import oracle
        rng = synth.rng(701)
        npts = max(8, args.cpu_points // 64)
        pts = np.stack([rng.integers(-mm + 1, mm, npts), rng.integers(0, mm, npts)], 1)
        pts[:4] = [[0, 0], [mm - 1, mm - 1], [-mm + 1, 0], [1, 1]]
        fr = np.asarray(f[0].astype(dt_np), np.complex128)
        gr = np.asarray(g[0].astype(dt_np), np.complex128)
        t0 = time.perf_counter()
        ref = oracle.convnd_hermitian_at(fr, gr, m, pts)
        dt = time.perf_counter() - t0
        got = h_gpu[0][pts[:, 0] + off, pts[:, 1]]
        err = {"sampled_points": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)), "points": int(npts)}
        nout = (2 * mm - 1) * mm
        return {"value": 1.0 / (dt / npts * nout), "unit": "convs/s", "cores": oracle.num_threads(),
                "kind": "oracle", "sample": f"{npts} output points (direct FP64 M = 2 sums, {dt:.2f} s), "
                                            f"extrapolated to the {nout} outputs"}, err

    cfg = {"workload": f"2D Euler nonlinearity: centered Hermitian 2D convolution, M = 2, {mm}x{mm} modes, "
                       f"storage {n[0]}x{n[1]}, {'complex64' if cdt == torch.complex64 else 'complex128'}",
           "m": list(m), "n": list(n), "M": 2, "dtype": args.dtype}
    return dict(run=run, explicit=None, convs=1, step_bytes=int(20 * S), kbytes_step=kbytes_step,
                kflops_step=kflops_step, cfg=cfg, cpu=cpu_baseline, out=lambda: run().cpu().numpy())


def wl_t1(args):
    """1D centered Hermitian ternary convolution (Sec. 4.2, tconv), m = 2048
    non-negative modes, |k|^-5/6 random phase, DC = 1, batch of B."""
    import torch
    import paper_1008_1366_amd as ic
    import synth
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    dt_np = np.complex64 if cdt == torch.complex64 else np.complex128
    m, B = 2048, args.batch or 2048
    f = synth.power_spectrum_1d(m, 5 / 6, 34, batch=B)
    g = synth.power_spectrum_1d(m, 5 / 6, 35, batch=B)
    e = synth.power_spectrum_1d(m, 5 / 6, 36, batch=B)
    F, G, E = (torch.from_numpy(x).to("cuda", cdt) for x in (f, g, e))
    cs = 8 if cdt == torch.complex64 else 16
    run = lambda: ic.conv1d_ternary(F, G, E)
    expl = lambda: ic.conv1d_ternary(F, G, E, method="explicit")
    NN = 1 << int(np.ceil(np.log2(m)))
    kbytes = {"k_conv1d_ternary": 4 * B * m * cs}
    kflops = {"k_conv1d_ternary": B * flops_row_ternary(NN)}

    def cpu_baseline(h_gpu, h_expl=None):
        """Oracle ternary sums (O(m^2) per output) at sampled outputs of the
        first pairs, extrapolated to whole convolutions by output count."""
        import oracle
        rng = synth.rng(37)
        nb, nk = 4, max(8, args.cpu_points // 64)
        t_or, errs = 0.0, {"implicit": [], "explicit": []}
        for b in range(nb):
            ks = np.unique(np.concatenate([[0, 1, m - 1], rng.integers(0, m, nk)]))
            fr, gr, er = (np.asarray(x[b].astype(dt_np), np.complex128) for x in (f, g, e))
            t0 = time.perf_counter()
            ref = oracle.conv1d_ternary_at(fr, gr, er, ks)
            t_or += time.perf_counter() - t0
            for key, h in (("implicit", h_gpu), ("explicit", h_expl)):
                if h is not None:
                    errs[key].append(float(np.linalg.norm(h[b][ks] - ref) / np.linalg.norm(ref)))
            nk_done = len(ks)
        per_out = t_or / (nb * nk_done)
        err = {k: {"max": max(v), "median": float(np.median(v)), "pairs": len(v)} for k, v in errs.items() if v}
        return {"value": 1.0 / (per_out * m), "unit": "convs/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{nk_done} sampled outputs of each of {nb} convolutions, direct FP64 ternary sums "
                          f"({t_or:.2f} s), extrapolated to {m} outputs per convolution"}, err

    cfg = {"workload": f"1D centered Hermitian ternary implicit dealiased convolution m={m}, batch {B}, "
                       f"{'complex64' if cdt == torch.complex64 else 'complex128'}",
           "m": m, "batch": B, "dtype": args.dtype}
    return dict(run=run, explicit=expl, convs=B, step_bytes=4 * B * m * cs, kbytes=kbytes, kflops=kflops,
                cfg=cfg, cpu=cpu_baseline, out=lambda: run().cpu().numpy())


WORKLOADS = {"c1": wl_c1, "c2": wl_c2, "c3": wl_c3, "x3": wl_x3, "c4": wl_c4, "c5": wl_c5, "t1": wl_t1, "t2": wl_t2,
             "e2": wl_e2}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--dtype", default=None, choices=["c64", "c128"],
                    help="default: c128 for c1 and c4 (stated in FP64; c4 adds a complex64 leg), c64 otherwise")
    ap.add_argument("--no-numpy", action="store_true", help="c4: skip the FP64 NumPy explicit-padded CPU time")
    ap.add_argument("--no-leg", action="store_true", help="c4: skip the complex64 leg")
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-explicit", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="c5: skip the captured-graph replay leg")
    ap.add_argument("--no-single", action="store_true", help="c1/c2: skip the one-pair latency leg")
    ap.add_argument("--no-autotune", action="store_true", help="c5: keep the default four-step splits")
    ap.add_argument("--t2-m", type=int, default=1024, help="t2: modes per axis")
    ap.add_argument("--e2-m", type=int, default=2048, help="e2: modes per axis")
    # oracle sample sizes (about 10 s of host work each)
    ap.add_argument("--cpu-points", type=int, default=65536, help="c3: sampled output points over the batch")
    ap.add_argument("--cpu-rows", type=int, default=0, help="c1/c2: convolutions (0: workload default)")
    ap.add_argument("--cpu-macs", type=float, default=4e10, help="c5: multiply-add budget")
    ap.add_argument("--one-stream", action="store_true",
                    help="c4/c5: every launch in order on one stream in the timed steps too (for profiling, so "
                         "that a traced kernel's duration matches the per-launch timing pass)")
    ap.add_argument("--profile-copy", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    args.dtype = args.dtype or ("c128" if args.workload in ("c1", "c4") else "c64")
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the workloads "
              "shard by batch with no exchange between GPUs, so they are measured on one", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1008_1366_amd as ic
    ic.lib()  # fail loudly without the HIP library
    torch.cuda.set_device(0)
    note(f"workload {args.workload} {args.dtype}: preparing inputs")
    W = WORKLOADS[args.workload](args)
    if args.one_stream and "kernel_timing_mode" in W:
        W["kernel_timing_mode"](True)
        W["kernel_timing_mode"] = lambda on: ("every launch in order on one stream (ONE_STREAM) in all steps"
                                              if on else None)
    note("timing the implicit path")

    # implicit path, with per-launch event timing inside the library
    ms_clean = timed(W["run"], args.steps, args.warmup)  # the timed region of the metric
    stats = step_stats(W["run"], max(args.steps, 50))  # at least 50 replays for sigma_L / sigma_H
    timing_note = W["kernel_timing_mode"](True) if "kernel_timing_mode" in W else None
    ic.timing_enable(True)  # second pass: per-launch kernel durations
    timed(W["run"], args.steps, 0, backlog=True)
    rep = ic.timing_report()
    ic.timing_enable(False)
    if timing_note:
        W["kernel_timing_mode"](False)
    convs_s = W["convs"] * 1000.0 / ms_clean
    note(f"implicit: {ms_clean:.4f} ms per step")
    copy_gbs = copy_bandwidth()

    # per-kernel algorithmic bytes and flops: per launch (kbytes / kflops) or
    # per step (kbytes_step / kflops_step, spread over the step's launches)
    kernels = []
    for r in rep:
        cnt = max(1, r["count"])
        per_step = cnt / args.steps
        kb = W.get("kbytes", {}).get(r["name"])
        kf = W.get("kflops", {}).get(r["name"])
        if kb is None and r["name"] in W.get("kbytes_step", {}):
            kb = W["kbytes_step"][r["name"]] / per_step
        if kf is None and r["name"] in W.get("kflops_step", {}):
            kf = W["kflops_step"][r["name"]] / per_step
        avg = r["total_ms"] / cnt
        k = {"name": r["name"], "launches_per_step": round(per_step, 3), "avg_ms": round(avg, 5),
             "ms_per_step": round(r["total_ms"] / args.steps, 5)}
        if kb:
            k["bytes_per_launch"] = int(kb)
            k["gbs"] = round(kb / (avg * 1e-3) / 1e9, 1)
        if kf:
            k["flops_per_launch"] = float(kf)
            k["tflops"] = round(kf / (avg * 1e-3) / 1e12, 2)
        kernels.append(k)
    dom = max(kernels, key=lambda k: k["ms_per_step"]) if kernels else None
    roof = None
    if dom is not None:
        traffic = None
        tf = os.path.join(ROOT, "profiles", f"traffic_{args.workload}_{args.dtype}.json")
        if os.path.exists(tf):
            rec = json.load(open(tf)).get("kernels", {}).get(dom["name"])
            if isinstance(rec, dict) and rec.get("source_hash") == kernel_source_hash(dom["name"]):
                traffic = rec["bytes"]
        hbm_frac = dom["gbs"] / HBM_PEAK_GBS if "gbs" in dom else None
        peak_tf = PEAK_TFLOPS[args.dtype]
        alu_frac = dom["tflops"] / peak_tf if "tflops" in dom else None
        bound = W.get("bound")
        if bound is None:  # by arithmetic intensity: whichever roof the kernel is nearer
            bound = "alu" if alu_frac is not None and (hbm_frac is None or alu_frac > hbm_frac) else "hbm"
        common = {"traffic": traffic, "kernel": dom["name"], "kernel_avg_ms": dom["avg_ms"],
                  "measured_gbs": round(traffic / (dom["avg_ms"] * 1e-3) / 1e9, 1) if traffic else None,
                  "traffic_over_algorithmic": (round(traffic / dom["bytes_per_launch"], 3)
                                               if traffic and dom.get("bytes_per_launch") else None)}
        if bound == "alu" and alu_frac is not None:
            roof = {"bound": "alu", "achieved": dom["tflops"], "peak": peak_tf, "unit": "TFLOP/s",
                    "frac": round(alu_frac, 4), **common,
                    "algorithmic_flops_per_launch": dom["flops_per_launch"],
                    "frac_of_nonpacked_valu": round(dom["tflops"] / VALU_NONPACKED_TFLOPS, 4),
                    "hbm_view": {"achieved_gbs": dom.get("gbs"), "frac": round(hbm_frac, 4) if hbm_frac else None}}
        elif hbm_frac is not None:
            roof = {"bound": "hbm", "achieved": dom["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm_frac, 4), **common,
                    "algorithmic_bytes_per_launch": dom["bytes_per_launch"]}
            if alu_frac is not None:
                roof["alu_view"] = {"achieved_tflops": dom["tflops"], "peak": peak_tf,
                                    "frac": round(alu_frac, 4),
                                    "frac_of_nonpacked_valu": round(dom["tflops"] / VALU_NONPACKED_TFLOPS, 4)}

    alg_gbs = W["step_bytes"] / (ms_clean * 1e-3) / 1e9
    out = {"metric": METRIC, "value": round(convs_s, 2), "unit": "convs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_clean, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "fp32" if args.dtype == "c64" else "fp64", "data": "synthetic",
           "config": W["cfg"], "step_stats": stats,
           "hbm_gbps_algorithmic": round(alg_gbs, 1),
           "hbm_frac_of_peak": round(alg_gbs / HBM_PEAK_GBS, 4),
           "copy_kernel_gbs": round(copy_gbs, 1),
           "hbm_frac_of_copy": round(alg_gbs / copy_gbs, 4),
           "kernels": kernels,
           "roofline": roof}
    if timing_note:
        out["kernel_timing"] = timing_note

    if W.get("explicit") is not None and not args.no_explicit:
        note("timing the explicit comparator")
        ms_e = timed(W["explicit"], max(3, args.steps // 2), 1)
        out["explicit_padded"] = {"ms_per_step": round(ms_e, 5), "value": round(W["convs"] * 1000.0 / ms_e, 2),
                                  "unit": "convs/s"}
        out["speedup_vs_explicit"] = round(ms_e / ms_clean, 3)
    if W.get("pruned") is not None and not args.no_explicit:
        ms_p = timed(W["pruned"], max(3, args.steps // 2), 1)
        out["explicit_pruned"] = {"ms_per_step": round(ms_p, 5), "value": round(W["convs"] * 1000.0 / ms_p, 2),
                                  "unit": "convs/s"}
        out["speedup_vs_pruned"] = round(ms_p / ms_clean, 3)

    if W.get("compensated") is not None and not args.no_explicit:
        ms_c = timed(W["compensated"], max(3, args.steps // 2), 1)
        out["compensated"] = {"ms_per_step": round(ms_c, 5), "value": round(W["convs"] * 1000.0 / ms_c, 2),
                              "unit": "convs/s", "note": "IMPCONV_COMPENSATED: twiddle products from FP32 "
                              "high and low parts; errors under rel_err_vs_oracle.compensated"}

    if W.get("single") is not None and not args.no_single:
        # the same convolution on one pair: a latency figure beside the batch throughput
        sg = W["single"]
        ms_1 = timed(sg["run"], max(args.steps, 50), args.warmup)
        out["single_pair"] = {"ms": round(ms_1, 5), "value": round(1000.0 / ms_1, 2), "unit": "convs/s",
                              "note": sg["note"]}
        if sg.get("explicit") is not None and not args.no_explicit:
            ms_1e = timed(sg["explicit"], max(args.steps, 50), args.warmup)
            out["single_pair"]["explicit_ms"] = round(ms_1e, 5)
            out["single_pair"]["speedup_vs_explicit"] = round(ms_1e / ms_1, 3)

    if W.get("leg") is not None and not args.no_leg:
        note("complex64 leg")
        leg = W["leg"]()
        if leg is not None:
            out["complex64_leg"] = leg

    if W.get("graph") is not None and not args.no_graph:
        replay, check = W["graph"]()
        ms_g = timed(replay, args.steps, args.warmup)
        out["hip_graph"] = {"ms_per_step": round(ms_g, 5), "value": round(W["convs"] * 1000.0 / ms_g, 2),
                            "unit": "convs/s", "replay_equals_eager": check(),
                            "note": "the whole step (forward, both gradients) captured once and replayed"}

    if args.profile_copy:
        n = args.profile_copy * (1 << 20) // 4
        x = torch.empty(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_kernel_bytes"] = {"read": n * 4, "write": n * 4}

    if not args.no_cpu:
        note("CPU baseline (oracle sample)")
        h = W["out"]()
        if W.get("explicit") is not None and not args.no_explicit:
            extra = {}
            if W.get("compensated") is not None:
                extra["h_comp"] = W["compensated"]().cpu().numpy()
            cpu, err = W["cpu"](h, W["explicit"]().cpu().numpy(), **extra)
        else:
            cpu, err = W["cpu"](h)
        out["cpu_baseline"] = {k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in cpu.items()}
        out["rel_err_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
