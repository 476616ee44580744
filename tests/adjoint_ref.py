"""Adjoint formulas of the centered Hermitian nD sum, composed from the
oracle's forward convolution (test-side; pinned by finite differences in
test_oracle_pins.py).

For a real loss L = Re sum_k conj(w_k) h_k over the stored half (leading
axes centered, offset n_d - m_d; last axis k >= 0), the gradient with
respect to the stored half of f is the Hermitian convolution of Gamma with g,
where Gamma equals w off the k_last = 0 hyperplane and w_k + conj(w_{-k}) on
it, followed by two edits on the hyperplane: the stored entries that the
symmetrization overwrites get zero gradient, and the DC entry is halved and
real."""
import numpy as np


def _plane_points(m, n):
    """(storage index of the leading axes, wavenumbers) on the k_last = 0
    hyperplane, within the box."""
    nd = len(m)
    for idx in np.ndindex(*n[:nd - 1]):
        k = [idx[d] - (n[d] - m[d]) for d in range(nd - 1)]
        if all(abs(k[d]) < m[d] for d in range(nd - 1)):
            yield idx, k


def hermitian_gamma(w, m):
    nd = len(m)
    n = w.shape[-nd:]
    g = w.copy()
    for idx, k in _plane_points(m, n):
        mi = tuple(-k[d] + (n[d] - m[d]) for d in range(nd - 1))
        g[(..., *idx, 0)] = w[(..., *idx, 0)] + np.conj(w[(..., *mi, 0)])
    return g


def hermitian_grad_edit(a, m):
    nd = len(m)
    n = a.shape[-nd:]
    a = a.copy()
    for idx, k in _plane_points(m, n):
        lead = [x for x in k if x != 0]
        if not lead:
            a[(..., *idx, 0)] = a[(..., *idx, 0)].real / 2
        elif lead[0] < 0:
            a[(..., *idx, 0)] = 0
    return a


def hermitian_nd_adjoint(orc, w, g, m):
    """Gradient of Re sum conj(w) convnd_hermitian(f, g) with respect to f."""
    return hermitian_grad_edit(orc.convnd_hermitian(hermitian_gamma(w, m), g, m), m)
