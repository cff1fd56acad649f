"""Grids of the imaginary-frequency G0W0 path (oracle; test infrastructure).

* Gamma-centred uniform k grid, equal weights w_k = 1/N_k (Sec. II A, the
  Green-function definition); the q grid is the k grid.
* Modified Gauss-Legendre imaginary frequencies omega = x0 (1+t)/(1-t) with
  weights g * 2 x0 / (1-t)^2 (t, g: Gauss-Legendre nodes/weights on [-1, 1]).
  The paper does not print its grid; this mapping is the one the workload
  definitions name.
"""
from __future__ import annotations

import numpy as np


def kgrid(nk):
    """Integer coordinates and fractional coordinates of the Gamma-centred grid.
    Index of (i1,i2,i3) is (i1*n2 + i2)*n3 + i3."""
    n1, n2, n3 = nk
    kint = np.array([(a, b, c) for a in range(n1) for b in range(n2) for c in range(n3)], dtype=np.int64)
    return kint, kint / np.array(nk, dtype=np.float64)


def kindex(iv, nk):
    n1, n2, n3 = nk
    iv = np.asarray(iv)
    return ((iv[..., 0] % n1) * n2 + (iv[..., 1] % n2)) * n3 + (iv[..., 2] % n3)


def kq_tables(nk):
    """kpq[k,q] = index of k+q, kmq[k,q] = index of k-q, minus[k] = index of -k."""
    kint, _ = kgrid(nk)
    kpq = kindex(kint[:, None, :] + kint[None, :, :], nk)
    kmq = kindex(kint[:, None, :] - kint[None, :, :], nk)
    minus = kindex(-kint, nk)
    return kpq, kmq, minus


def frequency_grid(n: int, x0: float):
    """Modified Gauss-Legendre grid on (0, inf): ascending omega and weights."""
    t, g = np.polynomial.legendre.leggauss(n)
    omega = x0 * (1.0 + t) / (1.0 - t)
    weight = g * 2.0 * x0 / (1.0 - t) ** 2
    return omega, weight


def pade_nodes(n_freq: int, n_par: int):
    """Indices of the frequency points used by the Pade fit: n_par points
    evenly spread over 0..n_freq-1, j*(n_freq-1)/(n_par-1) rounded half up."""
    n_par = min(n_par, n_freq)
    if n_par == 1:
        return np.zeros(1, dtype=np.int64)
    j = np.arange(n_par, dtype=np.int64)
    return (2 * j * (n_freq - 1) + (n_par - 1)) // (2 * (n_par - 1))
