"""The C ABI used from plain C (tests/c_abi_client.c, built with gcc
-std=c99 -pedantic -Werror against include/impconv.h and libimpconv.so):
argument validation on the CPU; on the GPU, descriptor plans executed by the
C client on device memory it allocates itself, checked against the FP64
oracle (Sec. 2.1 complex sum, Sec. 3.2 centered Hermitian 2D sum, Sec. 4
ternary sum)."""
import os
import subprocess

import numpy as np
import pytest

import c_abi_build
import oracle
import synth
from gpu_util import TOL, need_gpu, rel, rounded, say


def client():
    return c_abi_build.build()


def test_c_client_builds_and_validates():
    out = subprocess.run([client(), "info"], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    assert "validation ok" in out.stdout


def test_c_client_reports_size_errors(tmp_path):
    # m = 0 fails validation before any device work: status text on stderr
    out = subprocess.run([client(), "run", "0", "1", "1", "0", "0", "0", "0", "0", "0", "1", "1", "0",
                          str(tmp_path)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 1
    assert "impconv_plan_create" in out.stderr and "invalid size" in out.stderr


def run_client(tmp_path, kind, dt, m, n, batch, M, arrays):
    for name, a in arrays.items():
        np.ascontiguousarray(a.astype(dt)).tofile(os.path.join(tmp_path, name + ".bin"))
    m3 = list(m) + [0] * (3 - len(m))
    n3 = list(n) + [0] * (3 - len(n))
    args = [client(), "run", str(kind), "0" if dt == np.complex64 else "1", str(len(m)),
            *map(str, m3), *map(str, n3), str(batch), str(M), "0", str(tmp_path)]
    say(" ".join(args[1:-1]))
    out = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    return np.fromfile(os.path.join(tmp_path, "h.bin"), dtype=dt)


@pytest.mark.gpu
@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
def test_c_client_complex_1d(tmp_path, dt):
    need_gpu()
    B, M, m = 2, 2, 1000
    f = synth.unit_disk((B, M, m), 501)
    g = synth.unit_disk((B, M, m), 502)
    h = run_client(tmp_path, 0, dt, (m,), (m,), B, M, {"f": f, "g": g}).reshape(B, m)
    ref = oracle.conv1d_complex(rounded(f, dt), rounded(g, dt))
    assert rel(h, ref) < TOL[dt]


@pytest.mark.gpu
def test_c_client_hermitian_2d(tmp_path):
    need_gpu()
    dt = np.complex64
    m, n, M = (17, 40), (33, 41), 2
    f = synth.unit_disk((M, *n), 503)
    g = synth.unit_disk((M, *n), 504)
    h = run_client(tmp_path, 1, dt, m, n, 1, M, {"f": f, "g": g}).reshape(n)
    ref = oracle.convnd_hermitian(rounded(f, dt), rounded(g, dt), m)
    assert rel(h, ref) < TOL[dt]


@pytest.mark.gpu
def test_c_client_ternary_1d(tmp_path):
    need_gpu()
    dt = np.complex128
    m = 200
    f = synth.power_spectrum_1d(m, 5 / 6, 505)
    g = synth.power_spectrum_1d(m, 5 / 6, 506)
    e = synth.power_spectrum_1d(m, 5 / 6, 507)
    h = run_client(tmp_path, 2, dt, (m,), (m,), 1, 1, {"f": f, "g": g, "e": e})
    ref = oracle.conv1d_ternary(f, g, e)
    assert rel(h, ref) < TOL[dt]
