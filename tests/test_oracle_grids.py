"""Pins of the grids (oracle): closed-form integrals and index-table identities."""
import math

import numpy as np
import pytest

from oracle import grids


@pytest.mark.parametrize("n,a,tol", [(16, 0.5, 1e-11), (16, 2.0, 1e-8), (16, 0.1, 1e-7),
                                     (32, 0.05, 1e-8), (32, 10.0, 1e-8), (48, 0.05, 1e-8), (48, 10.0, 1e-8)])
def test_lorentzian_integral(n, a, tol):
    # int_0^inf dw / (w^2 + a^2) = pi / (2a)
    w, g = grids.frequency_grid(n, 0.5)
    val = np.sum(g / (w * w + a * a))
    assert abs(val - math.pi / (2 * a)) / (math.pi / (2 * a)) < tol


@pytest.mark.parametrize("n", [4, 16, 32])
def test_exact_for_mapped_polynomials(n):
    # (w + x0)^-p becomes a polynomial of degree p-2 in t: exact for p <= 2n+1
    x0 = 0.5
    w, g = grids.frequency_grid(n, x0)
    for p in range(2, 2 * n + 2):
        exact = x0 ** (1 - p) / (p - 1)
        assert abs(np.sum(g * (w + x0) ** (-p)) - exact) <= 1e-13 * exact


def test_grid_is_positive_ascending():
    w, g = grids.frequency_grid(32, 0.5)
    assert np.all(w > 0) and np.all(np.diff(w) > 0) and np.all(g > 0)


@pytest.mark.parametrize("nk", [(2, 2, 2), (6, 6, 6), (4, 3, 2), (1, 1, 1)])
def test_k_tables(nk):
    kint, kfrac = grids.kgrid(nk)
    kpq, kmq, minus = grids.kq_tables(nk)
    n = kint.shape[0]
    assert np.all(np.sort(kpq, axis=1) == np.arange(n)[None, :])  # a permutation per k
    for k in range(n):
        for q in range(n):
            assert kmq[kpq[k, q], q] == k
            d = kfrac[kpq[k, q]] - kfrac[k] - kfrac[q]
            assert np.allclose(d, np.round(d))
    assert np.all(minus[minus] == np.arange(n))
    assert minus[0] == 0
    assert np.all(kpq[np.arange(n), minus] == 0)


def test_pade_nodes():
    idx = grids.pade_nodes(32, 16)
    assert idx[0] == 0 and idx[-1] == 31 and len(idx) == 16 and np.all(np.diff(idx) > 0)
    assert list(grids.pade_nodes(16, 16)) == list(range(16))
    assert list(grids.pade_nodes(5, 1)) == [0]
    ref = np.floor(np.arange(9) * 47 / 8 + 0.5).astype(int)
    assert list(grids.pade_nodes(48, 9)) == list(ref)
