"""Seeded synthetic inputs for the convolution workloads.

Random numbers only: nothing here computes any part of a convolution.  Both
the tests (which hand the same arrays to the oracle and to the HIP library)
and bench.py draw from these generators.  Every generator uses numpy's PCG64
(``np.random.default_rng(seed)``) and returns complex128 arrays; FP32 runs
round these values to complex64.

Workload recipes (the paper's benchmarks use synthetic vectors; no public
dataset is involved):

* ``unit_disk``      -- entries uniform in the unit disk: r = sqrt(U), theta = 2 pi V.
* ``power_spectrum`` -- |k|^-alpha e^{i phi}, phi ~ U[0, 2 pi), value 1 at k = 0
                        (1D: k = index; multi-D: |k| the Euclidean wavenumber).
* ``gaussian_2d``    -- (Re, Im) ~ N(0, 1/2) each, times (1 + kx^2 + ky^2)^-1.
* ``ragged_lengths`` -- m = 2^round(U(lo, hi)) per pair.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def unit_disk(shape, seed: int) -> np.ndarray:
    r = rng(seed)
    rad = np.sqrt(r.random(shape))
    th = 2.0 * np.pi * r.random(shape)
    return rad * np.exp(1j * th)


def random_phase(shape, seed: int) -> np.ndarray:
    r = rng(seed)
    return np.exp(2j * np.pi * r.random(shape))


def power_spectrum_1d(m: int, alpha: float, seed: int, batch=None) -> np.ndarray:
    """Hermitian half k = 0..m-1: |k|^-alpha with random phase, real 1 at k = 0."""
    shape = (m,) if batch is None else (*np.atleast_1d(batch), m)
    k = np.arange(m, dtype=np.float64)
    amp = np.ones(m)
    amp[1:] = k[1:] ** (-alpha)
    u = amp * random_phase(shape, seed)
    u[..., 0] = 1.0
    return u


def power_spectrum_centered(m, n, alpha: float, seed: int) -> np.ndarray:
    """Centered Hermitian-half storage array for logical modes m (per axis) and
    storage extents n: leading axes hold wavenumber k at index k + (n_d - m_d),
    the last axis holds k at index k.  Amplitude |k|^-alpha with random phase,
    1 at the origin, zero outside the box |k_d| <= m_d - 1 (zero slots)."""
    m = tuple(int(x) for x in m)
    n = tuple(int(x) for x in n)
    nd = len(m)
    grids = []
    for d in range(nd):
        off = (n[d] - m[d]) if d < nd - 1 else 0
        kd = np.arange(n[d], dtype=np.float64) - off
        grids.append(kd)
    K = np.meshgrid(*grids, indexing="ij")
    k2 = sum(x * x for x in K)
    inside = np.ones(n, bool)
    for d in range(nd):
        inside &= np.abs(K[d]) <= m[d] - 1
    inside &= K[-1] >= 0
    amp = np.zeros(n)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (-alpha / 2.0), 1.0)
    u = amp * random_phase(n, seed)
    origin = tuple((n[d] - m[d]) if d < nd - 1 else 0 for d in range(nd))
    u[origin] = 1.0
    u[~inside] = 0.0
    return u


def gaussian_2d(mx: int, my: int, seed: int) -> np.ndarray:
    r = rng(seed)
    z = (r.normal(0.0, np.sqrt(0.5), (mx, my)) + 1j * r.normal(0.0, np.sqrt(0.5), (mx, my)))
    kx = np.arange(mx, dtype=np.float64)[:, None]
    ky = np.arange(my, dtype=np.float64)[None, :]
    return z / (1.0 + kx * kx + ky * ky)


def ragged_lengths(npairs: int, lo: float, hi: float, seed: int) -> np.ndarray:
    r = rng(seed)
    return (2 ** np.rint(r.uniform(lo, hi, npairs))).astype(np.int64)


def closed_form_complex(m: int):
    """Test vectors f_k = F e^{ik}, g_k = G e^{ik} (Sec. 2.1 accuracy test)."""
    k = np.arange(m)
    F = np.sqrt(3) + 1j * np.sqrt(7)
    G = np.sqrt(5) + 1j * np.sqrt(11)
    return F * np.exp(1j * k), G * np.exp(1j * k), F, G


def closed_form_hermitian(m: int):
    """Test vectors f_k = F e^{ik}, g_k = G e^{ik}, F, G real (Sec. 2.3 test)."""
    k = np.arange(m)
    F, G = np.sqrt(3), np.sqrt(5)
    return F * np.exp(1j * k), G * np.exp(1j * k), F, G
