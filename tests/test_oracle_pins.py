"""Pins for the FP64 oracle: each check uses something other than the oracle
itself -- the paper's printed closed forms, numpy/scipy library routines
(direct linear convolution, explicitly zero-padded FFT convolution), exact
invariants (delta inputs, shifts, linearity, symmetry, separability) and
finite differences.  A dropped term, wrong sign/index or transposed operand in
any oracle function fails at least one test here."""
import json
import os
from math import comb

import numpy as np
import pytest
import scipy.signal

import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_formulas.json")))
TOL = 1e-12


def rnd(shape, seed):
    return synth.unit_disk(shape, seed)


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def herm_full_np(u):
    """Hermitian extension written with numpy slicing (independent of the
    oracle's loop form): index j <-> wavenumber j - (m - 1)."""
    m = len(u)
    full = np.empty(2 * m - 1, np.complex128)
    full[m - 1:] = u
    full[m - 1] = u[0].real
    full[:m - 1] = np.conj(u[1:][::-1])
    return full


# ---------------------------------------------------------------- complex 1D

@pytest.mark.parametrize("m", [1, 2, 7, 64, 333])
def test_complex_closed_form(orc, m):
    cf = GOLD["closed_form_complex"]
    F = complex(*cf["F"])
    G = complex(*cf["G"])
    k = np.arange(m)
    f, g = F * np.exp(1j * k), G * np.exp(1j * k)
    H = F * G * (k + 1) * np.exp(1j * k)
    assert rel(orc.conv1d_complex(f, g), H) < 1e-14


@pytest.mark.parametrize("m", [1, 2, 3, 17, 64, 129])
def test_complex_vs_numpy_convolve(orc, m):
    f, g = rnd(m, 1), rnd(m, 2)
    assert rel(orc.conv1d_complex(f, g), np.convolve(f, g)[:m]) < TOL


@pytest.mark.parametrize("m", [1, 5, 32, 100])
def test_complex_vs_explicit_padded_fft(orc, m):
    f, g = rnd(m, 3), rnd(m, 4)
    N = 2 * m  # Sec. 1: pad to N = 2m
    h = np.fft.ifft(np.fft.fft(f, N) * np.fft.fft(g, N))[:m]
    assert rel(orc.conv1d_complex(f, g), h) < TOL


def test_complex_delta_and_shift(orc):
    m = 16
    for a in range(m):
        for b in range(m):
            f = np.zeros(m, complex); f[a] = 1
            g = np.zeros(m, complex); g[b] = 1
            h = orc.conv1d_complex(f, g)
            ref = np.zeros(m, complex)
            if a + b < m:
                ref[a + b] = 1
            assert np.array_equal(h, ref)
    f, g = rnd(m, 5), rnd(m, 6)
    h = orc.conv1d_complex(f, g)
    fs = np.concatenate([[0, 0, 0], f[:-3]])  # shift f by 3
    assert rel(orc.conv1d_complex(fs, g)[3:], h[:-3]) < TOL
    assert np.all(orc.conv1d_complex(fs, g)[:3] == 0)


def test_complex_commutative_linear_and_mdot(orc):
    m, M = 37, 3
    f, g, f2 = rnd((M, m), 7), rnd((M, m), 8), rnd((M, m), 9)
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    h = orc.conv1d_complex(f[None], g[None])[0]
    assert rel(h, sum(orc.conv1d_complex(f[i], g[i]) for i in range(M))) < TOL
    assert rel(orc.conv1d_complex(g[None], f[None])[0], h) < TOL
    lin = orc.conv1d_complex((a * f + b * f2)[None], g[None])[0]
    ref = a * h + b * orc.conv1d_complex(f2[None], g[None])[0]
    assert rel(lin, ref) < TOL


def test_complex_batch_layout(orc):
    B, M, m = 4, 2, 19
    f, g = rnd((B, M, m), 10), rnd((B, M, m), 11)
    h = orc.conv1d_complex(f, g)
    for b in range(B):
        ref = sum(np.convolve(f[b, i], g[b, i])[:m] for i in range(M))
        assert rel(h[b], ref) < TOL


def test_ragged(orc):
    ms = np.array([1, 4, 9, 32, 2])
    offs = np.concatenate([[0], np.cumsum(ms)[:-1]])
    f, g = rnd(ms.sum(), 12), rnd(ms.sum(), 13)
    h = orc.conv1d_complex_ragged(ms, offs, f, g)
    for m, o in zip(ms, offs):
        assert rel(h[o:o + m], np.convolve(f[o:o + m], g[o:o + m])[:m]) < TOL


# ---------------------------------------------------------------- gradients

@pytest.mark.parametrize("m", [1, 6, 33])
def test_gradient_finite_differences(orc, m):
    f, g, w = rnd(m, 14), rnd(m, 15), rnd(m, 16)

    def L(ff, gg):
        return np.real(np.vdot(w, orc.conv1d_complex(ff, gg)))  # Re sum conj(w) h

    gf, gg = orc.grad_conv1d_complex(f, g, w)
    eps = 1e-3  # L is bilinear: central differences are exact up to rounding
    for p in range(m):
        e = np.zeros(m, complex); e[p] = 1
        dre = (L(f + eps * e, g) - L(f - eps * e, g)) / (2 * eps)
        dim = (L(f + 1j * eps * e, g) - L(f - 1j * eps * e, g)) / (2 * eps)
        assert abs(gf[p] - (dre + 1j * dim)) < 1e-9 * max(1, abs(gf[p]))
        dre = (L(f, g + eps * e) - L(f, g - eps * e)) / (2 * eps)
        dim = (L(f, g + 1j * eps * e) - L(f, g - 1j * eps * e)) / (2 * eps)
        assert abs(gg[p] - (dre + 1j * dim)) < 1e-9 * max(1, abs(gg[p]))


# ---------------------------------------------------------------- centered

@pytest.mark.parametrize("m", [1, 2, 9, 40])
def test_centered_vs_numpy(orc, m):
    f, g = rnd(2 * m - 1, 17), rnd(2 * m - 1, 18)
    full = np.convolve(f, g)  # wavenumber index j <-> j - 2(m-1)
    ref = full[m - 1:3 * m - 2]
    assert rel(orc.conv1d_centered(f, g), ref) < TOL


@pytest.mark.parametrize("m", [2, 5, 16])
def test_centered_vs_explicit_3m_fft(orc, m):
    f, g = rnd(2 * m - 1, 19), rnd(2 * m - 1, 20)
    N = 3 * m  # Sec. 2.2 padding N >= 3m-2
    # place wavenumber k at FFT index k mod N
    def place(u):
        a = np.zeros(N, complex)
        for j in range(2 * m - 1):
            a[(j - (m - 1)) % N] = u[j]
        return a
    c = np.fft.ifft(np.fft.fft(place(f)) * np.fft.fft(place(g)))
    ref = np.array([c[k % N] for k in range(-(m - 1), m)])
    assert rel(orc.conv1d_centered(f, g), ref) < TOL


# ---------------------------------------------------------------- Hermitian 1D

@pytest.mark.parametrize("m", [1, 2, 3, 8, 64, 257])
def test_hermitian_closed_form(orc, m):
    cf = GOLD["closed_form_hermitian"]
    F, G = cf["F"], cf["G"]
    k = np.arange(m)
    f, g = F * np.exp(1j * k), G * np.exp(1j * k)
    H = F * G * (2 * m - 1 - k) * np.exp(1j * k)
    assert rel(orc.conv1d_hermitian(f, g), H) < 1e-14


@pytest.mark.parametrize("m", [1, 2, 4, 11, 64])
def test_hermitian_vs_numpy(orc, m):
    f, g = rnd(m, 21), rnd(m, 22)
    full = np.convolve(herm_full_np(f), herm_full_np(g))  # index j <-> j - 2(m-1)
    ref = full[2 * (m - 1):2 * (m - 1) + m]
    assert rel(orc.conv1d_hermitian(f, g), ref) < TOL


@pytest.mark.parametrize("m", [2, 6, 16])
def test_hermitian_vs_explicit_real_fft(orc, m):
    """Explicit 2/3-rule route: real physical-space product via irfft/rfft."""
    f, g = rnd(m, 23), rnd(m, 24)
    N = 3 * m
    def spec(u):
        a = np.zeros(N // 2 + 1, complex)
        a[:m] = u
        a[0] = u[0].real
        return a
    x = np.fft.irfft(spec(f), N) * N
    y = np.fft.irfft(spec(g), N) * N
    ref = np.fft.rfft(x * y)[:m] / N
    assert rel(orc.conv1d_hermitian(f, g), ref) < TOL


def test_hermitian_ignores_imag_dc_and_output_is_centered_restriction(orc):
    m = 12
    f, g = rnd(m, 25), rnd(m, 26)
    h = orc.conv1d_hermitian(f, g)
    f2 = f.copy(); f2[0] = f[0].real + 5j
    assert np.array_equal(orc.conv1d_hermitian(f2, g), h)
    full = orc.conv1d_centered(herm_full_np(f), herm_full_np(g))
    assert rel(full[m - 1:], h) < TOL
    assert rel(full[:m - 1][::-1], np.conj(h[1:])) < TOL  # Hermitian output


def test_hermitian_mdot_batch(orc):
    B, M, m = 3, 3, 10
    f, g = rnd((B, M, m), 27), rnd((B, M, m), 28)
    h = orc.conv1d_hermitian(f, g)
    for b in range(B):
        assert rel(h[b], sum(orc.conv1d_hermitian(f[b, i], g[b, i]) for i in range(M))) < TOL


# ---------------------------------------------------------------- ternary

def ternary_count(m, k):
    """Number of (p,q,r) in [-(m-1), m-1]^3 with p+q+r = k (inclusion-exclusion)."""
    S, W = k + 3 * (m - 1), 2 * m - 1
    n = 0
    for j in range(4):
        top = S - j * W
        if top >= 0:
            n += (-1) ** j * comb(3, j) * comb(top + 2, 2)
    return n


def brute_count(m, k):
    r = range(-(m - 1), m)
    return sum(1 for p in r for q in r if -(m - 1) <= k - p - q <= m - 1)


def test_ternary_count_formula():
    for m in range(1, 7):
        for k in range(m):
            assert ternary_count(m, k) == brute_count(m, k)


@pytest.mark.parametrize("m", [1, 2, 5, 16, 40])
def test_ternary_closed_form(orc, m):
    F, G, E = np.sqrt(3), np.sqrt(5), np.sqrt(7)
    k = np.arange(m)
    ph = np.exp(1j * k)
    H = F * G * E * np.array([ternary_count(m, kk) for kk in k]) * ph
    assert rel(orc.conv1d_ternary(F * ph, G * ph, E * ph), H) < 1e-13  # O(m^2) rounded terms


@pytest.mark.parametrize("m", [1, 3, 8, 24])
def test_ternary_vs_numpy(orc, m):
    f, g, e = rnd(m, 29), rnd(m, 30), rnd(m, 31)
    full = np.convolve(np.convolve(herm_full_np(f), herm_full_np(g)), herm_full_np(e))
    ref = full[3 * (m - 1):3 * (m - 1) + m]  # index j <-> j - 3(m-1)
    assert rel(orc.conv1d_ternary(f, g, e), ref) < TOL


def test_ternary_delta_and_symmetry(orc):
    m = 13
    f, g, e = rnd(m, 32), rnd(m, 33), rnd(m, 34)
    d0 = np.zeros(m, complex); d0[0] = 1
    assert rel(orc.conv1d_ternary(f, g, d0), orc.conv1d_hermitian(f, g)) < TOL
    h = orc.conv1d_ternary(f, g, e)
    assert rel(orc.conv1d_ternary(e, f, g), h) < TOL
    assert rel(orc.conv1d_ternary(g, e, f), h) < TOL


# ---------------------------------------------------------------- complex nD

@pytest.mark.parametrize("shape", [(5, 7), (8, 8), (3, 4, 5), (1, 6), (6, 1, 2)])
def test_complex_nd_vs_scipy(orc, shape):
    f, g = rnd(shape, 35), rnd(shape, 36)
    ref = scipy.signal.convolve(f, g, method="direct")[tuple(slice(0, s) for s in shape)]
    assert rel(orc.convnd_complex(f, g), ref) < TOL


def test_complex_nd_separable_and_sampled(orc):
    mx, my = 24, 20
    a, b, c, d = rnd(mx, 37), rnd(my, 38), rnd(mx, 39), rnd(my, 40)
    f, g = np.outer(a, b), np.outer(c, d)
    h = orc.convnd_complex(f, g)
    assert rel(h, np.outer(orc.conv1d_complex(a, c), orc.conv1d_complex(b, d))) < TOL
    pts = np.array([[0, 0], [mx - 1, my - 1], [5, 17], [23, 0]])
    assert rel(orc.convnd_complex_at(f, g, pts), h[pts[:, 0], pts[:, 1]]) < TOL


def test_complex_nd_mdot(orc):
    M, shape = 3, (6, 5, 4)
    f, g = rnd((M, *shape), 41), rnd((M, *shape), 42)
    h = orc.convnd_complex_M(f, g)
    assert rel(h, sum(orc.convnd_complex(f[i], g[i]) for i in range(M))) < TOL
    pts = np.array([[5, 4, 3], [0, 2, 1]])
    assert rel(orc.convnd_complex_at(f, g, pts, ndim=3), h[pts[:, 0], pts[:, 1], pts[:, 2]]) < TOL


# ---------------------------------------------------------------- Hermitian nD

def herm_storage(m, n, seed, sym_plane=True):
    u = synth.unit_disk(n, seed)
    nd = len(m)
    # zero slots
    for d in range(nd - 1):
        if n[d] == 2 * m[d]:
            idx = [slice(None)] * nd; idx[d] = 0; u[tuple(idx)] = 0
    if n[-1] == m[-1] + 1:
        u[..., m[-1]] = 0
    return u


def expand_np(u, m):
    """Full centered field written with numpy index arithmetic and the
    authoritative-half rule (independent of the oracle's loop form)."""
    nd = len(m)
    n = u.shape
    full = np.zeros(tuple(2 * x - 1 for x in m), complex)
    for idx in np.ndindex(full.shape):
        p = [idx[d] - (m[d] - 1) for d in range(nd)]
        def at(q):
            return u[tuple((q[d] + (n[d] - m[d]) if d < nd - 1 else q[d]) for d in range(nd))]
        q = [-x for x in p]
        if p[-1] > 0:
            v = at(p)
        elif p[-1] < 0:
            v = np.conj(at(q))
        else:
            lead = [x for x in p[:-1] if x != 0]
            if not lead:
                v = at(p).real
            elif lead[0] > 0:
                v = at(p)
            else:
                v = np.conj(at(q))
        full[idx] = v
    return full


@pytest.mark.parametrize("m,n", [((3, 4), (5, 4)), ((4, 4), (8, 5)), ((3, 3, 4), (6, 5, 5)),
                                 ((2, 3, 2), (3, 6, 2))])
def test_hermitian_nd_vs_scipy(orc, m, n):
    f, g = herm_storage(m, n, 43), herm_storage(m, n, 44)
    F, G = expand_np(f, m), expand_np(g, m)
    assert rel(orc.hermitian_expand(f, m), F) == 0
    full = scipy.signal.convolve(F, G, method="direct")  # index j <-> j - 2(m-1)
    h = orc.convnd_hermitian(f, g, m)
    nd = len(m)
    for idx in np.ndindex(*n):
        k = [idx[d] - (n[d] - m[d]) if d < nd - 1 else idx[d] for d in range(nd)]
        inside = all(abs(k[d]) <= m[d] - 1 for d in range(nd)) and k[-1] >= 0
        if not inside:
            assert h[idx] == 0
        else:
            ref = full[tuple(k[d] + 2 * (m[d] - 1) for d in range(nd))]
            assert abs(h[idx] - ref) < 1e-12 * max(1, abs(ref))


def test_hermitian_nd_symmetrization_reading(orc):
    """Only the authoritative half of the k_last = 0 plane matters when
    symmetrization is on; the output's k_last = 0 plane is Hermitian."""
    m, n = (4, 3, 4), (8, 6, 5)
    f, g = herm_storage(m, n, 45), herm_storage(m, n, 46)
    h = orc.convnd_hermitian(f, g, m)
    f2 = f.copy()
    f2[4 - 1, :, 0] += 3.0  # k_x = -1 line of the k_z = 0 plane: non-authoritative
    assert np.array_equal(orc.convnd_hermitian(f2, g, m), h)
    Hf = orc.hermitian_expand(h, m)
    assert rel(Hf, np.conj(Hf[::-1, ::-1, ::-1])) < 1e-15


def expand_projected_np(u, m):
    """Full centered field under the NO_SYMMETRIZE reading, written with numpy
    array operations (independent of the oracle's per-point loop): off the
    k_last = 0 hyperplane the stored value or the conjugate of its mirror; on
    it the Hermitian projection (U_k + conj U_{-k}) / 2 of the stored plane
    (concluding remarks: the routine reads what a real transform of an
    unsymmetrized plane represents)."""
    nd = len(m)
    n = u.shape
    # dense centered array D[j] = stored value at wavenumber j - (m - 1) for
    # k_last >= 0 (zero elsewhere), gathered by slicing
    sl = tuple(slice(n[d] - m[d] - (m[d] - 1), n[d] - m[d] + m[d]) for d in range(nd - 1))
    pos = u[sl + (slice(0, m[-1]),)]                  # k_last = 0..m-1
    full = np.zeros(tuple(2 * x - 1 for x in m), complex)
    full[(Ellipsis, slice(m[-1] - 1, None))] = pos
    # mirror: U_{-k} = conj U_k for k_last > 0 (flip every axis)
    mir = np.conj(pos[(slice(None, None, -1),) * (nd - 1) + (slice(m[-1] - 1, 0, -1),)])
    full[(Ellipsis, slice(0, m[-1] - 1))] = mir
    plane = pos[..., 0]
    full[..., m[-1] - 1] = 0.5 * (plane + np.conj(plane[(slice(None, None, -1),) * (nd - 1)]))
    return full


@pytest.mark.parametrize("m,n", [((3, 4), (5, 4)), ((4, 4), (8, 5)), ((3, 3, 4), (6, 5, 5)),
                                 ((2, 3, 2), (3, 6, 2))])
def test_hermitian_nd_no_symmetrize_projection(orc, m, n):
    """NO_SYMMETRIZE reading: the k_last = 0 hyperplane enters as its Hermitian
    projection.  The oracle (symmetrize=False) must equal scipy's direct
    convolution of fields expanded by the numpy projection above, for the
    binary and the ternary sums; on already-symmetric input both readings
    agree, and on an unsymmetrized plane they differ."""
    f, g, e = herm_storage(m, n, 141), herm_storage(m, n, 142), herm_storage(m, n, 143)
    F, G, E = expand_projected_np(f, m), expand_projected_np(g, m), expand_projected_np(e, m)
    assert rel(orc.hermitian_expand(f, m, symmetrize=False), F) < 1e-15
    nd = len(m)
    full2 = scipy.signal.convolve(F, G, method="direct")
    full3 = scipy.signal.convolve(full2, E, method="direct")
    h2 = orc.convnd_hermitian(f, g, m, symmetrize=False)
    h3 = orc.convnd_ternary(f, g, e, m, symmetrize=False)
    for idx in np.ndindex(*n):
        k = [idx[d] - (n[d] - m[d]) if d < nd - 1 else idx[d] for d in range(nd)]
        if not (all(abs(k[d]) <= m[d] - 1 for d in range(nd)) and k[-1] >= 0):
            assert h2[idx] == 0 and h3[idx] == 0
            continue
        r2 = full2[tuple(k[d] + 2 * (m[d] - 1) for d in range(nd))]
        r3 = full3[tuple(k[d] + 3 * (m[d] - 1) for d in range(nd))]
        assert abs(h2[idx] - r2) < 1e-12 * max(1, abs(r2))
        assert abs(h3[idx] - r3) < 1e-12 * max(1, abs(r3))
    # the two readings differ on this (unsymmetrized) input ...
    assert rel(h2, orc.convnd_hermitian(f, g, m)) > 1e-3
    # ... and agree once the plane is Hermitian (symmetrized by the numpy rule)
    fs, gs, es = (herm_from_full(expand_np(x, m), m, n) for x in (f, g, e))
    assert rel(orc.convnd_hermitian(fs, gs, m, symmetrize=False), orc.convnd_hermitian(fs, gs, m)) < 1e-14
    assert rel(orc.convnd_ternary(fs, gs, es, m, symmetrize=False), orc.convnd_ternary(fs, gs, es, m)) < 1e-14


def herm_from_full(full, m, n):
    """Stored half (storage extents n, zero slots 0) of a dense centered field."""
    nd = len(m)
    u = np.zeros(n, complex)
    sl = tuple(slice(n[d] - m[d] - (m[d] - 1), n[d]) for d in range(nd - 1))
    u[sl + (slice(0, m[-1]),)] = full[(Ellipsis, slice(m[-1] - 1, None))][
        tuple(slice(0, 2 * m[d] - 1) for d in range(nd - 1))]
    return u


def test_hermitian_2d_separable(orc):
    """F = A (x) B with A, B Hermitian-symmetric 1D fields: the 2D centered
    Hermitian sum factors into a centered 1D sum in x and a Hermitian 1D sum
    in y."""
    mx, my = 9, 12
    A, C = herm_full_np(rnd(mx, 47)), herm_full_np(rnd(mx, 48))
    b, d = rnd(my, 49), rnd(my, 50)
    b[0] = b[0].real; d[0] = d[0].real
    f = np.outer(A, b)  # storage (2mx-1) x my
    g = np.outer(C, d)
    h = orc.convnd_hermitian(f, g, (mx, my))
    ref = np.outer(orc.conv1d_centered(A, C), orc.conv1d_hermitian(b, d))
    assert rel(h, ref) < TOL


def test_hermitian_nd_sampled(orc):
    m, n = (5, 4, 6), (10, 8, 7)
    f = np.stack([herm_storage(m, n, 51 + i) for i in range(2)])
    g = np.stack([herm_storage(m, n, 61 + i) for i in range(2)])
    h = orc.convnd_hermitian(f, g, m)
    pts = np.array([[0, 0, 0], [-4, 3, 5], [4, -3, 0], [2, 0, 1]])
    got = orc.convnd_hermitian_at(f, g, m, pts)
    ref = [h[p[0] + 5, p[1] + 4, p[2]] for p in pts]
    assert rel(got, ref) < TOL
    h0 = orc.convnd_hermitian(f[0], g[0], m) + orc.convnd_hermitian(f[1], g[1], m)
    assert rel(h, h0) < TOL


def test_ternary_sampled_matches_full(orc):
    m = 19
    f, g, e = rnd(m, 71), rnd(m, 72), rnd(m, 73)
    h = orc.conv1d_ternary(f, g, e)
    ks = [0, 5, 18]
    assert rel(orc.conv1d_ternary_at(f, g, e, ks), h[ks]) < TOL


def test_nd_sampled_1d_forms(orc):
    """The sampled nD routines restricted to one axis agree with numpy."""
    m = 40
    f, g = rnd(m, 74), rnd(m, 75)
    ks = np.array([[0], [17], [39]])
    assert rel(orc.convnd_complex_at(f, g, ks), np.convolve(f, g)[ks[:, 0]]) < TOL
    full = np.convolve(herm_full_np(f), herm_full_np(g))
    ref = full[2 * (m - 1) + ks[:, 0]]
    assert rel(orc.convnd_hermitian_at(f, g, (m,), ks), ref) < TOL


# ---------------------------------------------------------------- ternary nD (tconv2)

@pytest.mark.parametrize("m,n", [((3, 4), (5, 4)), ((4, 4), (8, 5)), ((2, 3), (4, 4)), ((3, 2, 3), (6, 3, 4))])
def test_ternary_nd_vs_scipy(orc, m, n):
    """Definition via two library convolutions of the expanded fields:
    (F * G) * E over the full index range, restricted to the box."""
    f, g, e = herm_storage(m, n, 81), herm_storage(m, n, 82), herm_storage(m, n, 83)
    F, G, E = expand_np(f, m), expand_np(g, m), expand_np(e, m)
    full = scipy.signal.convolve(scipy.signal.convolve(F, G, method="direct"), E, method="direct")
    h = orc.convnd_ternary(f, g, e, m)
    nd = len(m)
    for idx in np.ndindex(*n):
        k = [idx[d] - (n[d] - m[d]) if d < nd - 1 else idx[d] for d in range(nd)]
        inside = all(abs(k[d]) <= m[d] - 1 for d in range(nd)) and k[-1] >= 0
        if not inside:
            assert h[idx] == 0
        else:
            ref = full[tuple(k[d] + 3 * (m[d] - 1) for d in range(nd))]
            assert abs(h[idx] - ref) < 1e-12 * max(1, abs(ref))


def test_ternary_2d_brute_force(orc):
    """Four nested loops over p and q on a tiny grid, fields expanded by
    expand_np."""
    m, n = (2, 2), (4, 3)
    f, g, e = herm_storage(m, n, 84), herm_storage(m, n, 85), herm_storage(m, n, 86)
    F, G, E = expand_np(f, m), expand_np(g, m), expand_np(e, m)
    a = [x - 1 for x in m]
    h = orc.convnd_ternary(f, g, e, m)
    for kx in range(-a[0], a[0] + 1):
        for ky in range(0, a[1] + 1):
            s = 0
            for px in range(-a[0], a[0] + 1):
                for py in range(-a[1], a[1] + 1):
                    for qx in range(-a[0], a[0] + 1):
                        for qy in range(-a[1], a[1] + 1):
                            rx, ry = kx - px - qx, ky - py - qy
                            if abs(rx) <= a[0] and abs(ry) <= a[1]:
                                s += F[px + a[0], py + a[1]] * G[qx + a[0], qy + a[1]] * E[rx + a[0], ry + a[1]]
            assert abs(h[kx + n[0] - m[0], ky] - s) < 1e-13


def test_ternary_nd_delta_is_binary(orc):
    """e = delta at the origin reduces the ternary sum to the binary one."""
    m, n = (4, 3), (8, 4)
    f, g = herm_storage(m, n, 87), herm_storage(m, n, 88)
    e = np.zeros(n, complex)
    e[n[0] - m[0], 0] = 1.0
    assert rel(orc.convnd_ternary(f, g, e, m), orc.convnd_hermitian(f, g, m)) < TOL


def test_ternary_2d_separable(orc):
    """U = A (x) b for each field: the sum factors into a full centered
    ternary sum in x (two numpy convolutions) and the 1D Hermitian ternary
    sum in y."""
    mx, my = 7, 9
    A, C, P = (herm_full_np(rnd(mx, s)) for s in (89, 90, 91))
    b, d, q = rnd(my, 92), rnd(my, 93), rnd(my, 94)
    for v in (b, d, q):
        v[0] = v[0].real
    f, g, e = np.outer(A, b), np.outer(C, d), np.outer(P, q)
    h = orc.convnd_ternary(f, g, e, (mx, my))
    xfull = np.convolve(np.convolve(A, C), P)[2 * (mx - 1):4 * (mx - 1) + 1]
    ref = np.outer(xfull, orc.conv1d_ternary(b, d, q))
    assert rel(h, ref) < TOL


def test_ternary_nd_symmetric_and_sampled(orc):
    m, n = (3, 4, 3), (6, 7, 4)
    f, g, e = herm_storage(m, n, 95), herm_storage(m, n, 96), herm_storage(m, n, 97)
    h = orc.convnd_ternary(f, g, e, m)
    assert rel(orc.convnd_ternary(e, f, g, m), h) < TOL
    assert rel(orc.convnd_ternary(g, e, f, m), h) < TOL
    pts = np.array([[0, 0, 0], [-2, 3, 2], [2, -3, 0], [1, 0, 1]])
    got = orc.convnd_ternary_at(f, g, e, m, pts)
    ref = [h[p[0] + 3, p[1] + 3, p[2]] for p in pts]
    assert rel(got, ref) < TOL


# ---------------------------------------------------------------- adjoints (Hermitian 1D, complex nD)

def _fd_grad(L, x, eps=0.5):
    """Central differences of a real function L that is affine in x: exact up
    to rounding for any step.  Returns dL/dRe x + i dL/dIm x."""
    g = np.zeros_like(x)
    for idx in np.ndindex(*x.shape):
        e = np.zeros_like(x)
        e[idx] = eps
        dr = (L(x + e) - L(x - e)) / (2 * eps)
        di = (L(x + 1j * e) - L(x - 1j * e)) / (2 * eps)
        g[idx] = dr + 1j * di
    return g


@pytest.mark.parametrize("m", [1, 2, 5, 12])
def test_hermitian_adjoint_formula(orc, m):
    """For L = Re sum conj(w) h(f, g) the gradient with respect to the stored
    half of f is conv_herm(w', g) with w'_0 = 2 Re w_0, entry 0 halved and
    real -- the reading the library's HERMITIAN_ADJOINT flag implements."""
    f, g, w = rnd(m, 131), rnd(m, 132), rnd(m, 133)
    L = lambda x: float(np.real(np.vdot(w, orc.conv1d_hermitian(x, g))))
    fd = _fd_grad(L, f)
    wp = w.copy()
    wp[0] = 2 * w[0].real
    an = orc.conv1d_hermitian(wp, g)
    an[0] = an[0].real / 2
    assert rel(an, fd) < 1e-12
    assert fd[0].imag == pytest.approx(0, abs=1e-12)  # Im f_0 is ignored


def test_complex_nd_adjoint_formula(orc):
    """grad f = REV(conv(REV(w), conj g)) with every axis reversed."""
    m = (4, 5)
    f, g, w = synth.unit_disk(m, 134), synth.unit_disk(m, 135), synth.unit_disk(m, 136)
    L = lambda x: float(np.real(np.vdot(w, orc.convnd_complex(x, g))))
    fd = _fd_grad(L, f)
    an = orc.convnd_complex(w[::-1, ::-1].copy(), np.conj(g))[::-1, ::-1]
    assert rel(an, fd) < 1e-12


@pytest.mark.parametrize("m,n", [((3, 4), (5, 4)), ((4, 3), (8, 4)), ((3, 2, 3), (6, 3, 4)),
                                 ((2, 3, 2), (3, 6, 2))])
def test_hermitian_nd_adjoint_formula(orc, m, n):
    """Centered Hermitian 2D/3D: the gradient with respect to the stored half
    is conv_herm(Gamma, g), Gamma = w off the k_last = 0 hyperplane and
    w_k + conj(w_{-k}) on it, with the overwritten half of that hyperplane
    zero and DC halved and real.  Finite differences see every stored entry,
    zero slots and the ignored entries included."""
    from adjoint_ref import hermitian_nd_adjoint
    f, g = herm_storage(m, n, 137), herm_storage(m, n, 138)
    w = rnd(n, 139)
    L = lambda x: float(np.real(np.vdot(w, orc.convnd_hermitian(x, g, m))))
    fd = _fd_grad(L, rnd(n, 140))
    an = hermitian_nd_adjoint(orc, w, g, m)
    assert rel(an, fd) < 1e-12
    assert rel(hermitian_nd_adjoint(orc, w, f, m), _fd_grad(
        lambda x: float(np.real(np.vdot(w, orc.convnd_hermitian(f, x, m)))), g)) < 1e-12
