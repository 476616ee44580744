"""GPU parity of the complex128 1D rows of FFT size N = 8192 with M = 1, whose
transform takes one 1024-thread workgroup: the two residues of Sec. 2.1 run
one after the other in one kernel.  Checked against the FP64 oracle on whole
rows (ragged lengths in the class), with the adjoint flags, inside a ragged
batch (a per-class launch beside the queue and the three-pass classes), and
beside the M > 1 form of the same size, which keeps the paired kernel."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, need_gpu, rel, say, to_dev

pytestmark = pytest.mark.gpu

DT = np.complex128


@pytest.mark.parametrize("m", [4097, 6000, 8191, 8192])
def test_serial_rows_vs_oracle(m):
    """The 1/2 rule at N = 8192 (block size np = N forces it over the
    automatic p/q choice); three rows, every output compared."""
    ic = need_gpu()
    say(f"serial rows m={m}")
    B = 3
    f, g = synth.unit_disk((B, m), 401), synth.unit_disk((B, m), 402)
    h = ic.conv1d_complex_pq(to_dev(f, DT), to_dev(g, DT), np=8192).cpu().numpy()
    ref = oracle.conv1d_complex(f[:, None], g[:, None])
    for b in range(B):
        assert rel(h[b], ref[b]) < TOL[DT], (b, rel(h[b], ref[b]))


@pytest.mark.parametrize("m", [5000, 8192])
def test_serial_rows_adjoint_flags(m):
    """REV_F | CONJ_G | REV_OUT gives the input gradient of Sec. 2.1's sum:
    dL/df = rev(conv(rev(w), conj g)) for L = Re sum conj(w) h."""
    ic = need_gpu()
    say(f"serial rows adjoint m={m}")
    f, g, w = (synth.unit_disk(m, s) for s in (403, 404, 405))
    gf = ic.conv1d_complex_pq(to_dev(w, DT), to_dev(g, DT), np=8192,
                              flags=ic.REV_F | ic.CONJ_G | ic.REV_OUT).cpu().numpy()
    rf, _ = oracle.grad_conv1d_complex(f, g, w)
    assert rel(gf, rf) < TOL[DT]


def test_serial_rows_equal_automatic_choice_at_8192():
    """At m = N = 8192 the automatic choice is the 1/2 rule: conv1d_complex
    and the forced block size give the same bits."""
    ic = need_gpu()
    import torch
    f, g = synth.unit_disk((2, 8192), 406), synth.unit_disk((2, 8192), 407)
    F, G = to_dev(f, DT), to_dev(g, DT)
    assert torch.equal(ic.conv1d_complex(F, G), ic.conv1d_complex_pq(F, G, np=8192))


def test_paired_rows_mdot_at_8192():
    """M = 2 at m = 8192: the M-dot sum of Sec. 3.3 through the paired row
    kernel, against the oracle."""
    ic = need_gpu()
    say("paired rows M=2 m=8192")
    f, g = synth.unit_disk((2, 2, 8192), 408), synth.unit_disk((2, 2, 8192), 409)
    h = ic.conv1d_complex(to_dev(f, DT), to_dev(g, DT)).cpu().numpy()
    assert rel(h, oracle.conv1d_complex(f, g)) < TOL[DT]


def test_serial_class_in_ragged_batch():
    """Complex128 pairs of N = 8192 form a fused class launched on its own
    (the queue holds classes up to 4096 in complex128); every pair matches
    the oracle, and the gaps between pairs are not written."""
    ic = need_gpu()
    import torch
    ms = np.array([8192, 5000, 64, 7000, 40000, 300, 4097, 8000, 5])
    offs = np.concatenate([[0], np.cumsum(ms + 3)[:-1]])
    tot = int(offs[-1] + ms[-1] + 3)
    f, g = synth.unit_disk(tot, 410), synth.unit_disk(tot, 411)
    F, G = to_dev(f, DT), to_dev(g, DT)
    plan = ic.RaggedPlan(ms, offs, dtype=torch.complex128)
    meth = {c["N"]: c["method"] for c in plan.schedule()}
    say(f"ragged serial class {meth}")
    assert meth[8192] == "fused" and meth[65536] == "four-step"
    out = torch.zeros_like(F)
    plan.execute(F, G, out=out)
    h = out.cpu().numpy()
    for m, o in zip(ms, offs):
        if m <= 8192:
            assert rel(h[o:o + m], oracle.conv1d_complex(f[o:o + m], g[o:o + m])) < TOL[DT], m
        else:
            ks = np.array([0, 1, m // 3, m - 1])
            r = oracle.convnd_complex_at(f[o:o + m], g[o:o + m], ks[:, None])
            assert rel(h[o + ks], r) < TOL[DT], m
    gaps = np.ones(tot, bool)
    for m, o in zip(ms, offs):
        gaps[o:o + m] = False
    assert not h[gaps].any()
