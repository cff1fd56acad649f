"""Pins of the truncated-Coulomb screening (oracle): Sec. III B replaces V by
V^cut(q) in the numerator of Eq. screened_W_matr and keeps the full V in the
symmetrised dielectric matrix,
    W^c = Vcut^{1/2} (eps~^{-1} - I) Vcut^{1/2},   eps~ = I - V^{1/2} chi V^{1/2},
with the Hermitian square roots the equation writes.  Expanding
eps~^{-1} - I = V^{1/2} chi (I - V chi)^{-1} V^{1/2} gives the pins:

* V^cut = V: the plain screening;
* N_aux = 1: W^c = v_c (1/(1 - v chi) - 1);
* V^cut a function of V (common eigenvectors): W^c = (V^cut V)^{1/2} chi_RPA
  (V V^cut)^{1/2}, chi_RPA = chi (I - V chi)^{-1}, from one eigenbasis;
* a unitary change of the auxiliary basis carries W^c along (the Hermitian
  roots are basis-covariant; a Cholesky factor of V^cut in their place is not);
* it differs from V^cut in both places and from the Cholesky-factor form.
"""
import numpy as np
import pytest

from oracle import screening
from oracle.pipeline import Oracle
from synth.systems import make_config, make_custom, truncated_coulomb


def _hpd(rng, n, lo=0.1):
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    return A @ A.conj().T + lo * np.eye(n)


def _chi(rng, n, nw):
    # Hermitian negative semidefinite responses
    out = np.empty((nw, n, n), dtype=np.complex128)
    for w in range(nw):
        B = (rng.standard_normal((n, 3 * n)) + 1j * rng.standard_normal((n, 3 * n))) / np.sqrt(6 * n)
        out[w] = -(0.3 + w) * (B @ B.conj().T)
    return out


def test_vcut_equal_to_v_is_the_plain_screening():
    rng = np.random.default_rng(1)
    V = _hpd(rng, 9)
    chi = _chi(rng, 9, 3)
    a = screening.screen(chi, V)[1]
    b = screening.screen(chi, V, V.copy())[1]
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


def test_single_function_closed_form():
    for v, vc, x in ((3.0, 0.7, -0.4), (12.0, 2.5, -2.0), (0.5, 0.5, -0.01)):
        W = screening.screen(np.array([[[x + 0j]]]), np.array([[v + 0j]]), np.array([[vc + 0j]]))[1]
        assert abs(W[0, 0, 0] - vc * (1.0 / (1.0 - v * x) - 1.0)) < 1e-14


def test_commuting_truncation_closed_form():
    rng = np.random.default_rng(2)
    n = 11
    V = _hpd(rng, n)
    lam, U = np.linalg.eigh(V)
    g = lam / (1.0 + 0.5 * lam) + 0.05          # V^cut = g(V): bounded, positive
    Vc = (U * g[None, :]) @ U.conj().T
    chi = _chi(rng, n, 4)
    W = screening.screen(chi, V, Vc)[1]
    M = (U * np.sqrt(g * lam)[None, :]) @ U.conj().T     # (V^cut V)^{1/2} = (V V^cut)^{1/2} here
    for w in range(chi.shape[0]):
        rpa = chi[w] @ np.linalg.inv(np.eye(n) - V @ chi[w])
        ref = M @ rpa @ M
        assert np.max(np.abs(W[w] - ref)) < 1e-12 * np.max(np.abs(ref))


def test_unitary_covariance_and_distinct_readings():
    rng = np.random.default_rng(3)
    n = 10
    V, Vc = _hpd(rng, n), _hpd(rng, n, lo=0.05)
    chi = _chi(rng, n, 2)
    W = screening.screen(chi, V, Vc)[1]
    Q = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))[0]
    Wr = screening.screen(np.einsum("ij,wjk,kl->wil", Q.conj().T, chi, Q), Q.conj().T @ V @ Q,
                          Q.conj().T @ Vc @ Q)[1]
    assert np.max(np.abs(np.einsum("ij,wjk,kl->wil", Q, Wr, Q.conj().T) - W)) < 1e-12 * np.max(np.abs(W))
    # V^cut in the dielectric matrix as well is another result
    Wboth = screening.screen(chi, Vc)[1]
    assert np.max(np.abs(Wboth - W)) > 1e-3 * np.max(np.abs(W))
    # Cholesky factors in place of the Hermitian roots: not covariant, and off
    L, Lc = np.linalg.cholesky(V), np.linalg.cholesky(Vc)
    eye = np.eye(n)
    for w in range(chi.shape[0]):
        eL = eye - L.conj().T @ chi[w] @ L
        naive = Lc @ (np.linalg.inv(eL) - eye) @ Lc.conj().T
        assert np.max(np.abs(naive - W[w])) > 1e-3 * np.max(np.abs(W[w]))


def test_synthetic_truncation_and_pass():
    """The synthetic V^cut(q): positive definite, V^cut(-q) = conj V^cut(q), equal
    to V except on auxiliary function 0; a whole oracle pass with it keeps
    W^c negative semidefinite and Sigma^c(k) = Sigma^c(-k) on a grid whose k
    are all time-reversal invariant."""
    s = make_config(1)
    Vc = truncated_coulomb(s)
    for q in range(s.n_k):
        assert np.linalg.eigvalsh(Vc[q]).min() > 0.0
        d = Vc[q] - s.V[q]
        d[0, 0] = 0.0
        assert np.max(np.abs(d)) == 0.0
    assert np.max(np.abs(Vc[0] - s.V[0])) == 0.0
    s2 = make_custom(n_atoms=2, nb_per_atom=4, naux_per_atom=9, nk=(3, 1, 2), n_occ=2, n_freq=6, seed=43)
    Vc2 = truncated_coulomb(s2)
    from oracle import grids
    _, _, minus = grids.kq_tables(s2.spec.nk)
    for q in range(s2.n_k):
        assert np.max(np.abs(Vc2[minus[q]] - Vc2[q].conj())) < 1e-14 * np.max(np.abs(Vc2[q]))
    s.Vcut = Vc
    o = Oracle(s)
    Wc = o.wc(3)
    for w in Wc:
        lw = np.linalg.eigvalsh(w)
        assert lw.max() <= 1e-12 * np.abs(lw).max()
    plain = Oracle(make_config(1)).wc(3)
    assert np.max(np.abs(Wc - plain)) > 1e-6 * np.max(np.abs(plain))
