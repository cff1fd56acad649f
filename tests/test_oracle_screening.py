"""Screening pins (oracle): spectral bounds, NSD W^c, Cholesky-factor invariance,
Gamma-point special cases."""
import numpy as np
import pytest

from oracle import screening, response, grids
from synth.systems import make_config


def test_spectral_bounds(c1_oracle):
    s = c1_oracle.sys
    for q in (1, 4):
        chi = c1_oracle.result["per_q"][q]["chi"]
        eps, Wc = screening.screen(chi, s.V[q])
        for e, w in zip(eps, Wc):
            le = np.linalg.eigvalsh(e)
            assert le.min() >= 1.0 - 1e-12
            li = np.linalg.eigvalsh(np.linalg.inv(e) - np.eye(len(e)))
            assert li.min() > -1.0 and li.max() <= 1e-12
            lw = np.linalg.eigvalsh(w)
            assert lw.max() <= 1e-12 * np.abs(lw).max()


def test_pair_weights_real_nonpositive(c1_oracle):
    X = c1_oracle.result["per_q"][3]["X"]
    assert np.max(np.abs(X.imag)) <= 1e-13 * np.max(np.abs(X))
    assert X.real.max() <= 1e-14 * np.max(np.abs(X))


def test_cholesky_factor_gives_same_w(c1_oracle):
    # W^c = L (eps_L^-1 - I) L^H with V = L L^H, eps_L = I - L^H chi L, equals the
    # square-root form: eps_L = Q^H eps Q with Q = V^-1/2 L unitary.
    s = c1_oracle.sys
    q = 3
    chi = c1_oracle.result["per_q"][q]["chi"]
    _, Wc = screening.screen(chi, s.V[q])
    L = np.linalg.cholesky(s.V[q])
    eye = np.eye(s.n_aux)
    for iw in (0, 7, 15):
        eL = eye - L.conj().T @ chi[iw] @ L
        W2 = L @ (np.linalg.inv(eL) - eye) @ L.conj().T
        assert np.linalg.norm(W2 - Wc[iw]) <= 1e-12 * np.linalg.norm(Wc[iw])


def test_gamma_zero_momentum_reduces_to_projected_regular_form(c1_oracle):
    s = c1_oracle.sys
    o = c1_oracle
    B0 = o.B(0)
    p0 = np.zeros_like(s.p)
    eps_l, eps_mu, Wc = screening.screen_gamma(B0, s.eig, s.n_occ, p0, s.omega_cell, s.V[0], o.omega)
    v, X = screening.coulomb_eigenbasis(s.V[0])
    chi = o.chi0(0, B0)
    Vh = screening.sqrt_hpd(s.V[0])
    for iw in (0, 5):
        assert abs(eps_l[iw][0, 0] - 1.0) < 1e-15
        assert np.max(np.abs(eps_l[iw][0, 1:])) < 1e-15
        reg = np.eye(s.n_aux) - Vh @ chi[iw] @ Vh
        reg_l = X.conj().T @ reg @ X
        assert np.max(np.abs(reg_l[1:, 1:] - eps_l[iw][1:, 1:])) < 1e-11 * np.max(np.abs(reg_l))


def test_gamma_single_aux_closed_form():
    # N_aux = 1: eps = 1 + s/N_k sum_k sum_ia 2D/(D^2+w^2) (4 pi/Omega) |p/D|^2
    rng = np.random.default_rng(2)
    nk, no, nu = 3, 2, 3
    eig = np.sort(np.concatenate([rng.uniform(-0.8, -0.1, (nk, no)), rng.uniform(0.1, 1.5, (nk, nu))], axis=1), axis=1)
    p = rng.standard_normal((nk, no, nu)) + 1j * rng.standard_normal((nk, no, nu))
    B0 = rng.standard_normal((nk, 1, no, nu)) + 0j
    om = np.array([0.1, 1.0, 4.0])
    Om = 270.0
    v = 3.7
    eps_l, eps_mu, Wc = screening.screen_gamma(B0, eig, no, p, Om, np.array([[v + 0j]]), om)
    for iw, w in enumerate(om):
        tot = 0.0
        for k in range(nk):
            d = eig[k, no:][None, :] - eig[k, :no][:, None]
            tot += np.sum(2 * d / (d * d + w * w) * (4 * np.pi / Om) * np.abs(p[k] / d) ** 2)
        e = 1 + 2.0 / nk * tot
        assert abs(eps_l[iw][0, 0] - e) < 1e-13
        assert abs(Wc[iw][0, 0] - v * (1 / e - 1)) < 1e-13


def test_gamma_head_matches_printed_band_pair_sum(c1_oracle):
    # The head of Eq. dielectric_func_gamma as printed (insulator: no intraband
    # term): 1 - (4 pi / Omega) sum_{k, sigma} sum_{m<n} 2 (f_m - f_n) |p_mn|^2 /
    # ([(e_m - e_n)^2 + w^2] (e_m - e_n)), summed over every band pair with its
    # occupation difference and signed denominator, Omega the crystal volume
    # N_k * Omega_cell and two spin channels, against the oracle's Gram form
    # over (occupied, unoccupied) pairs for the full auxiliary set
    s, o = c1_oracle.sys, c1_oracle
    rng = np.random.default_rng(11)
    p = rng.standard_normal(s.p.shape) + 1j * rng.standard_normal(s.p.shape)
    eps_l, _, _ = screening.screen_gamma(o.B(0), s.eig, s.n_occ, p, s.omega_cell, s.V[0], o.omega)
    nb = s.spec.n_bands
    f = np.zeros(nb)
    f[:s.n_occ] = 1.0
    omega_crystal = s.n_k * s.omega_cell
    for iw in (0, 7, len(o.omega) - 1):
        w = o.omega[iw]
        tot = 0.0
        for k in range(s.n_k):
            for m in range(nb):
                for n in range(m + 1, nb):
                    if f[m] == f[n]:
                        continue
                    pmn = p[k, m, n - s.n_occ]
                    d = s.eig[k, m] - s.eig[k, n]
                    tot += 2.0 * (f[m] - f[n]) * abs(pmn) ** 2 / ((d * d + w * w) * d)
        head = 1.0 - (4.0 * np.pi / omega_crystal) * 2.0 * tot
        assert abs(eps_l[iw][0, 0] - head) < 1e-12 * abs(head)


def test_gamma_wing_phase_is_the_unpinned_convention(c1_oracle):
    """The limit of the Gamma pins: a constant phase on the momentum elements
    (a sign error of the wing is one) changes only the wing blocks of
    eps~_lambda, so the head, the body and the eigenvalue bound hold for
    either phase, and the average over +-q_hat is the same for both.
    Conjugated momentum elements also keep head, body and bound, but change
    the averaged W^c(0): that error would pass the pins and move results."""
    s, o = c1_oracle.sys, c1_oracle
    B0 = o.B(0)
    rng = np.random.default_rng(5)
    p = rng.standard_normal(s.p.shape) + 1j * rng.standard_normal(s.p.shape)
    e1, _, _ = screening.screen_gamma(B0, s.eig, s.n_occ, p, s.omega_cell, s.V[0], o.omega)
    e2, _, _ = screening.screen_gamma(B0, s.eig, s.n_occ, np.exp(0.7j) * p, s.omega_cell, s.V[0], o.omega)
    assert np.max(np.abs(e1[:, 0, 0] - e2[:, 0, 0])) < 1e-13
    assert np.max(np.abs(e1[:, 1:, 1:] - e2[:, 1:, 1:])) < 1e-13
    assert np.max(np.abs(e1[:, 0, 1:] - e2[:, 0, 1:])) > 1e-3 * np.max(np.abs(e1[:, 0, 1:]))
    for e in (e1, e2):
        assert min(np.linalg.eigvalsh(m).min() for m in e) >= 1.0 - 1e-12
    w = np.array([0.5, 0.5])
    a1 = screening.screen_gamma_average(B0, s.eig, s.n_occ, np.stack([p, -p]), w, s.omega_cell, s.V[0], o.omega)
    a2 = screening.screen_gamma_average(B0, s.eig, s.n_occ, np.stack([p.conj(), -p.conj()]), w, s.omega_cell,
                                        s.V[0], o.omega)
    a3 = screening.screen_gamma_average(B0, s.eig, s.n_occ, np.stack([np.exp(0.7j) * p, -np.exp(0.7j) * p]), w,
                                        s.omega_cell, s.V[0], o.omega)
    assert np.linalg.norm(a1 - a3) < 1e-12 * np.linalg.norm(a1)
    e3, _, _ = screening.screen_gamma(B0, s.eig, s.n_occ, p.conj(), s.omega_cell, s.V[0], o.omega)
    assert np.max(np.abs(e1[:, 0, 0] - e3[:, 0, 0])) < 1e-13
    assert np.max(np.abs(e1[:, 1:, 1:] - e3[:, 1:, 1:])) < 1e-13
    assert min(np.linalg.eigvalsh(m).min() for m in e3) >= 1.0 - 1e-12
    assert np.linalg.norm(a1 - a2) > 1e-6 * np.linalg.norm(a1)
