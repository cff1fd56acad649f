"""Two-level closed form (one k point, one auxiliary function, one occupied and
one unoccupied band): pins chi0, screening, the frequency integral of
Sigma^c, Pade continuation and the QP solve of the oracle against algebra.

  chi0(iw)  = -2 s D |m12|^2 / (D^2 + w^2)
  W^c(iw)   = -A / (Om^2 + w^2),  Om^2 = D^2 + 2 s D v |m12|^2,  A = 2 s D v^2 |m12|^2
  Sigma^c_n(iw) = A/(2 Om) [ |m_n1|^2 / (iw + mu - e1 + Om) + |m_n2|^2 / (iw + mu - e2 - Om) ]
"""
import numpy as np
import pytest

from oracle import grids, response, screening, selfenergy, continuation

E1, E2, MU = -0.3, 0.45, 0.05
V = 0.8
M = np.array([[0.7 + 0.0j, 0.35 - 0.2j], [0.35 + 0.2j, -0.4 + 0.0j]])   # Hermitian m_nm
S = 2.0


def closed_form():
    D = E2 - E1
    m12 = abs(M[0, 1]) ** 2
    Om = np.sqrt(D * D + 2 * S * D * V * m12)
    A = 2 * S * D * V * V * m12
    return D, Om, A


def sigma_exact(z, n):
    """Sigma^c_n at complex frequency argument z = i w (or E - mu)."""
    D, Om, A = closed_form()
    return A / (2 * Om) * (abs(M[n, 0]) ** 2 / (z + MU - E1 + Om) + abs(M[n, 1]) ** 2 / (z + MU - E2 - Om))


def run_grid(n_freq):
    omega, weight = grids.frequency_grid(n_freq, 0.5)
    eig = np.array([[E1, E2]])
    kpq = np.zeros((1, 1), dtype=int)
    B = np.array(M[0, 1]).reshape(1, 1, 1, 1)
    chi = response.chi0_trs(B, eig, kpq, 0, 1, omega)
    eps, Wc = screening.screen(chi, np.array([[V + 0j]]))
    x = M.reshape(1, 1, 2, 2)                        # x^mu_{nm}, n = 0,1 (QP), m = 0,1
    X = selfenergy.pair_weights(x, Wc)
    sig = selfenergy.sigma_c_q(X, eig, kpq, 0, MU, omega, weight, 1)
    return omega, weight, chi, Wc, X, sig


def test_chi0_and_wc_closed_form():
    omega, _, chi, Wc, X, _ = run_grid(16)
    D, Om, A = closed_form()
    ref_chi = -2 * S * D * abs(M[0, 1]) ** 2 / (D * D + omega ** 2)
    ref_wc = -A / (Om * Om + omega ** 2)
    assert np.max(np.abs(chi[:, 0, 0] - ref_chi) / np.abs(ref_chi)) < 1e-14
    # eps^-1 - I cancels where screening is weak (large w): relative error ~ 1e-16 / |eps - 1|
    assert np.max(np.abs(Wc[:, 0, 0] - ref_wc) / np.abs(ref_wc)) < 1e-11
    assert np.all(X.real <= 0) and np.max(np.abs(X.imag)) < 1e-15


# The folded quadrature resolves the near-singular kernel a/(a^2 + w_j^2) only
# where the grid is dense, so convergence is checked for w_i <= 2 Ha (the range
# the Pade nodes that decide the QP energy come from) and w_i <= 10 Ha.
@pytest.mark.parametrize("n_freq,tol2,tol10", [(16, 2e-3, 1e-2), (32, 5e-4, 3e-3), (64, 5e-6, 1e-3),
                                               (128, 1e-9, 3e-4), (256, 1e-14, 5e-5)])
def test_sigma_converges_to_closed_form(n_freq, tol2, tol10):
    omega, _, _, _, _, sig = run_grid(n_freq)
    ex = np.array([[sigma_exact(1j * w, n) for w in omega] for n in range(2)])
    err = np.max(np.abs(sig[0] - ex), axis=0)
    assert err[omega <= 2.0].max() < tol2
    assert err[omega <= 10.0].max() < tol10


def test_unfolded_equals_folded():
    omega, weight, _, _, X, sig = run_grid(32)
    eig = np.array([[E1, E2]])
    unf = selfenergy.sigma_c_unfolded(X, eig, np.zeros((1, 1), dtype=int), 0, MU, omega, weight, 1)
    assert np.max(np.abs(unf - sig)) < 1e-14


def test_qp_closed_form():
    omega, _, _, _, _, sig = run_grid(256)
    D, Om, A = closed_form()
    nodes = grids.pade_nodes(len(omega), 16)
    E, Z, ok = continuation.qp_energies(sig, omega, np.array([[E1, E2]]), np.zeros((1, 2)), MU, nodes)
    assert ok.all()
    for n, en in enumerate((E1, E2)):
        c1 = A / (2 * Om) * abs(M[n, 0]) ** 2
        c2 = A / (2 * Om) * abs(M[n, 1]) ** 2
        p1, p2 = E1 - Om, E2 + Om
        # (E - en)(E - p1)(E - p2) - c1 (E - p2) - c2 (E - p1) = 0
        poly = np.polymul(np.polymul([1, -en], [1, -p1]), [1, -p2])
        poly = np.polysub(poly, np.polyadd(np.polymul([c1], [1, -p2]), np.polymul([c2], [1, -p1])))
        roots = np.roots(poly)
        real = roots[np.abs(roots.imag) < 1e-12].real
        ref = real[np.argmin(np.abs(real - en))]
        assert abs(E[0, n] - ref) < 1e-9
        dsig = -(c1 / (ref - p1) ** 2 + c2 / (ref - p2) ** 2)
        assert abs(Z[0, n] - 1 / (1 - dsig)) < 1e-7
