"""hipGraph capture of the one-shot entry points (through torch.cuda.graph):
each call is captured once and replayed three times on new inputs copied into
the captured buffers, with eager work and synchronizations between the
replays; every replay must equal the eager result bit for bit (the kernels
are deterministic and the library records no memset or allocation)."""
import numpy as np
import pytest

import synth
from gpu_util import need_gpu, rel, say

pytestmark = pytest.mark.gpu


def herm_storage(m, n, seed):
    u = synth.unit_disk(n, seed)
    for d in range(len(m) - 1):
        if n[d] == 2 * m[d]:
            idx = [slice(None)] * len(m)
            idx[d] = 0
            u[tuple(idx)] = 0
    if n[-1] == m[-1] + 1:
        u[..., m[-1]] = 0
    return u


def cases(ic):
    c64, c128 = np.complex64, np.complex128
    return [
        ("conv1d_complex", lambda a, b: ic.conv1d_complex(a, b), (3, 2, 1000), c64, None),
        ("conv1d_complex_pq", lambda a, b: ic.conv1d_complex_pq(a, b, 256), (3, 700), c64, None),
        ("conv1d_complex_compensated", lambda a, b: ic.conv1d_complex(a, b, flags=ic.COMPENSATED), (2, 1500), c64,
         None),
        ("conv1d_hermitian", lambda a, b: ic.conv1d_hermitian(a, b), (2, 2, 3000), c128, None),
        ("conv2d_complex", lambda a, b: ic.conv2d(a, b), (2, 2, 64, 48), c64, None),
        ("conv2d_hermitian", lambda a, b: ic.conv2d(a, b, kind="hermitian", m=(20, 17)), (2, 40, 18), c64,
         ((20, 17), (40, 18))),
        ("conv3d_hermitian", lambda a, b: ic.conv3d(a, b, kind="hermitian", m=(5, 6, 4)), (2, 9, 12, 5), c128,
         ((5, 6, 4), (9, 12, 5))),
        ("conv2d_ternary", lambda a, b: ic.conv2d_ternary(a, b, a, m=(12, 9)), (2, 24, 10), c64,
         ((12, 9), (24, 10))),
        ("conv3d_complex_adjoint_flags", lambda a, b: ic.conv3d(a, b, flags=ic.REV_F | ic.CONJ_G | ic.REV_OUT),
         (2, 6, 7, 8), c64, None),
    ]


def make(shape, dt, herm, seed):
    if herm is None:
        return synth.unit_disk(shape, seed).astype(dt)
    m, n = herm
    lead = shape[:len(shape) - len(n)]
    return np.stack([herm_storage(m, n, seed + i) for i in range(int(np.prod(lead)))]).reshape(shape).astype(dt)


@pytest.mark.parametrize("idx", range(9))
def test_graph_replay_matches_eager(idx):
    ic = need_gpu()
    import torch
    name, fn, shape, dt, herm = cases(ic)[idx]
    say(f"graph {name} {shape}")
    dev = torch.device("cuda:0")
    A = torch.from_numpy(make(shape, dt, herm, 700)).to(dev)
    B = torch.from_numpy(make(shape, dt, herm, 710)).to(dev)
    fn(A, B)  # eager first call: tables and code objects loaded outside the capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn(A, B)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        out = fn(A, B)
    for rep in range(3):
        a = torch.from_numpy(make(shape, dt, herm, 720 + 10 * rep)).to(dev)
        b = torch.from_numpy(make(shape, dt, herm, 721 + 10 * rep)).to(dev)
        A.copy_(a)
        B.copy_(b)
        graph.replay()
        torch.cuda.synchronize()
        eager = fn(a, b)
        torch.cuda.synchronize()
        assert torch.equal(out, eager), (name, rep)
        _ = (a * 2).sum().item()  # unrelated eager work between replays


def test_plan_first_execution_is_capturable():
    """A descriptor plan creates everything its execution needs: the first
    execution of a long complex 1D plan (three-pass form, whose column
    twiddle table is made at plan creation) may itself be captured, and the
    replays equal an eager execution bit for bit."""
    ic = need_gpu()
    import torch
    m, B = 70000, 2  # power-of-two size 131072, four-step split 512 x 256
    say(f"plan capture complex 1D m={m}")
    dev = torch.device("cuda:0")
    plan = ic.Plan("complex", torch.complex128, (m,), batch=B)
    A = torch.from_numpy(synth.unit_disk((B, m), 741)).to(dev)
    Bv = torch.from_numpy(synth.unit_disk((B, m), 742)).to(dev)
    out = torch.empty((B, m), dtype=torch.complex128, device=dev)
    work = torch.empty(max(plan.work_bytes, 16), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.execute(A, Bv, out=out, work=work)
    for rep in range(2):
        graph.replay()
        torch.cuda.synchronize()
        eager = plan.execute(A, Bv)
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        A.copy_(torch.from_numpy(synth.unit_disk((B, m), 743 + rep)).to(dev))
    ks = np.array([0, 1, 777, m - 1])
    a, b = A.cpu().numpy(), Bv.cpu().numpy()
    graph.replay()
    torch.cuda.synchronize()
    import oracle
    ref = oracle.convnd_complex_at(a[1], b[1], ks[:, None])
    assert rel(out[1].cpu().numpy()[ks], ref) < 1e-11
