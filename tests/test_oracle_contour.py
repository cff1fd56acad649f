"""Pins of the contour-deformation oracle (`oracle.contour`) and, through the
exact pole form of the RPA self-energy, of the imaginary-axis Sigma^c.

The pole form: with chi~(w) = -A (D^2 - w^2)^{-1} A^H (A's columns
sqrt(2 s D_t / N_k) V^{1/2} B_t, one per occupied/unoccupied pair t), the
Woodbury identity gives W^c(w) = -sum_s v_s v_s^H / (Omega_s^2 - w^2), where
Omega_s^2 and u_s are the eigenpairs of D^2 + A^H A and v_s = V^{1/2} A u_s.
Each pair weight is then a sum of one-pole terms, and
Sigma^c_n(k,E) = 1/N_k sum_q sum_m sum_s a_s / (E - e_m +- Omega_s) in closed
form (+ for occupied m, - for unoccupied), a_s = |x_nm^T v_s|^2 / (2 Omega_s).
This holds at complex E = i w + mu (the imaginary-axis formula) and at real E
(contour deformation) alike, and uses neither the quadrature grid nor the
residue bookkeeping."""
import numpy as np
import pytest

from oracle import contour, grids, screening
from oracle.pipeline import Oracle
from synth.systems import make_custom


def _poles(o, q, gamma):
    """Omega_s and v_s [N_aux][S] of W^c(q, w) = -sum_s v_s v_s^H / (Omega_s^2 - w^2)."""
    s = o.sys
    B = o.B(q)
    n_k, n_aux = B.shape[0], B.shape[1]
    D, cols = [], []
    if q == 0 and gamma:
        # the Gamma treatment's Gram form in the V^cut(0) eigenbasis (its head
        # and wings are pinned in test_oracle_screening)
        v, X = screening.coulomb_eigenbasis(s.V[0])
        sv = np.sqrt(v)
        for k in range(n_k):
            d = (s.eig[k][s.n_occ:][None, :] - s.eig[k][:s.n_occ][:, None]).reshape(-1)
            Y = sv[:, None] * (X.conj().T @ B[k].reshape(n_aux, -1))
            Y[0, :] = np.sqrt(4 * np.pi / s.omega_cell) * s.p[k].reshape(-1) / d
            D.append(d)
            cols.append(Y)
        T = X * sv[None, :]
    else:
        lam, U = np.linalg.eigh(s.V[q])
        T = (U * np.sqrt(lam)[None, :]) @ U.conj().T
        for k in range(n_k):
            d = (s.eig[o.kpq[k, q]][s.n_occ:][None, :] - s.eig[k][:s.n_occ][:, None]).reshape(-1)
            D.append(d)
            cols.append(T @ B[k].reshape(n_aux, -1))
    D = np.concatenate(D)
    A = np.concatenate(cols, axis=1) * np.sqrt(2.0 * 2.0 / n_k * D)[None, :]
    lam, U = np.linalg.eigh(np.diag(D * D) + A.conj().T @ A)
    return np.sqrt(lam), T @ A @ U


def _exact_sigma(o, E, gamma):
    """Closed-form Sigma^c at energies E[..., k, n] (complex or real)."""
    s = o.sys
    out = np.zeros(E.shape, dtype=np.complex128)
    sg = np.where(np.arange(s.n_bands) < s.n_occ, 1.0, -1.0)
    for q in range(s.n_k):
        Om, v = _poles(o, q, gamma)
        x = o.x(q)
        a = np.abs(np.einsum("kanm,as->knms", x, v)) ** 2 / (2.0 * Om)
        for k in range(s.n_k):
            em = s.eig[o.kmq[k, q]]
            for n in range(x.shape[2]):
                den = E[..., k, n][..., None, None] - em[:, None] + sg[:, None] * Om[None, :]
                out[..., k, n] += np.sum(a[k, n] / den, axis=(-1, -2))
    return out / s.n_k


def _tiny(n_freq=32):
    return make_custom(n_atoms=2, nb_per_atom=5, naux_per_atom=6, nk=(2, 1, 1), n_occ=3, n_freq=n_freq,
                       qp_lo=1, n_qp=4, seed=5)


def test_interpolation_exact_on_cubics():
    rng = np.random.default_rng(0)
    omr, h = contour.real_grid(9, 0.4)
    c = rng.standard_normal(4)
    poly = lambda w: c[0] + c[1] * w + c[2] * w ** 2 + c[3] * w ** 3
    w = rng.uniform(h, omr[-1], 50)            # away from the reflected end
    got = contour.interp_real(np.broadcast_to(poly(omr), (50, 9)), h, w)
    assert np.max(np.abs(got - poly(w))) < 1e-13
    even = lambda w: c[0] + c[2] * w ** 2      # even: exact on the whole range
    w = rng.uniform(0.0, omr[-1], 50)
    got = contour.interp_real(np.broadcast_to(even(omr), (50, 9)), h, w)
    assert np.max(np.abs(got - even(w))) < 1e-13
    assert np.allclose(contour.interp_real(np.broadcast_to(poly(omr), (9, 9)), h, omr), poly(omr), atol=1e-14)


def _multipole(seed=3, nb=9, n_occ=4, S=5):
    rng = np.random.default_rng(seed)
    em = np.concatenate([np.sort(rng.uniform(-0.8, -0.05, n_occ)), np.sort(rng.uniform(0.05, 1.5, nb - n_occ))])
    dmin = em[n_occ:].min() - em[:n_occ].max()
    Om = rng.uniform(dmin, 1.5, (nb, S))
    a = rng.uniform(0.01, 0.2, (nb, S))
    return em, dmin, Om, a


@pytest.mark.parametrize("n_r,tol", [(16, 1e-5), (32, 5e-7)])
def test_one_pole_sums_closed_form(n_r, tol):
    """X_nm(w) = sum_s 2 a_s Omega_s / (w^2 - Omega_s^2): contour deformation
    against sum_m sum_s a_s/(E - e_m +- Omega_s), through the band gap."""
    em, dmin, Om, a = _multipole()
    n_occ = 4
    om, wt = grids.frequency_grid(32, 0.5)
    omr, h = contour.real_grid(n_r, 0.6 * dmin)
    Xi = np.sum(-2 * a[:, None, :] * Om[:, None, :] / (om[None, :, None] ** 2 + Om[:, None, :] ** 2), -1)
    Xr = np.sum(2 * a[:, None, :] * Om[:, None, :] / (omr[None, :, None] ** 2 - Om[:, None, :] ** 2), -1)
    E = np.linspace(em[n_occ - 1] - 0.5 * dmin, em[n_occ] + 0.5 * dmin, 41)
    got = contour.sigma_cd_q(Xi[None, None], Xr[None, None], em[None], np.zeros((1, 1), int), 0, n_occ, om, wt, h,
                             E[:, None, None], 1)[:, 0, 0]
    sg = np.where(np.arange(len(em)) < n_occ, 1.0, -1.0)
    ex = np.array([np.sum(a / (e - em[:, None] + sg[:, None] * Om)) for e in E])
    assert np.max(np.abs(got - ex)) / np.max(np.abs(ex)) < tol


def test_continuous_through_a_level_and_beyond_grid_is_nan():
    """At E = e_m the residue counts half (Sigma^c is smooth there); a residue
    frequency beyond the real grid's top gives NaN."""
    em, dmin, Om, a = _multipole()
    n_occ = 4
    om, wt = grids.frequency_grid(32, 0.5)
    omr, h = contour.real_grid(32, 0.6 * dmin)
    Xi = np.sum(-2 * a[:, None, :] * Om[:, None, :] / (om[None, :, None] ** 2 + Om[:, None, :] ** 2), -1)
    Xr = np.sum(2 * a[:, None, :] * Om[:, None, :] / (omr[None, :, None] ** 2 - Om[:, None, :] ** 2), -1)
    e0 = em[n_occ - 1]
    E = np.array([e0 - 1e-7, e0, e0 + 1e-7, em[0] - 0.01])[:, None, None]
    if e0 - em[0] + 0.01 <= 0.6 * dmin:
        pytest.skip("levels too close for the NaN case")
    got = contour.sigma_cd_q(Xi[None, None], Xr[None, None], em[None], np.zeros((1, 1), int), 0, n_occ, om, wt, h, E,
                             1)[:, 0, 0]
    assert abs(got[1] - 0.5 * (got[0] + got[2])) < 1e-6 * abs(got[1])
    assert abs(got[0] - got[2]) < 1e-5 * abs(got[1])
    assert np.isnan(got[3])


@pytest.mark.parametrize("gamma", [False, True])
def test_real_energies_against_rpa_poles(gamma):
    """Contour deformation of the whole oracle path (response on both axes,
    screening, pair weights, residues) against the closed-form pole sum."""
    s = _tiny()
    o = Oracle(s)
    vbm, cbm = s.eig[:, :s.n_occ].max(), s.eig[:, s.n_occ:].min()
    dmin = cbm - vbm
    E = np.random.default_rng(1).uniform(vbm - 0.5 * dmin, cbm + 0.5 * dmin, (3, s.n_k, s.spec.n_qp))
    ex = _exact_sigma(o, E, gamma)
    assert np.max(np.abs(ex.imag)) == 0.0
    for n_r, tol in ((8, 2e-6), (16, 2e-7)):
        got = o.sigma_cd(n_r, 0.6 * dmin, E, gamma=gamma)
        assert np.max(np.abs(got - ex.real)) / np.max(np.abs(ex)) < tol, n_r


@pytest.mark.parametrize("gamma", [False, True])
def test_imaginary_axis_against_rpa_poles(gamma):
    """The imaginary-axis Sigma^c (Eq. GW_selfe_element on the modified
    Gauss-Legendre grid) equals the pole sum at i w + mu wherever the grid
    resolves the integrand: w_i below 0.15 Ha with 32 points.  Higher w_i put
    the integrand's near-pole at w = w_i onto the grid itself."""
    s = _tiny(32)
    o = Oracle(s)
    sig = sum(o.sigma_q(q, o.wc(q, gamma=gamma))[0] for q in range(s.n_k))
    Ei = np.moveaxis(np.broadcast_to(1j * o.omega[None, None, :] + s.mu, sig.shape), -1, 0)
    ex = np.moveaxis(_exact_sigma(o, Ei, gamma), 0, -1)
    low = o.omega < 0.15
    assert low.sum() >= 10
    assert np.max(np.abs(sig[..., low] - ex[..., low])) / np.max(np.abs(ex[..., low])) < 1e-9


def test_real_axis_response_ordering():
    """Below the first transition the real-axis weight 2D/(D^2 - w^2) exceeds
    the static one, which exceeds every imaginary-axis one: -chi~ grows in the
    Loewner order from i w through 0 to real w."""
    s = _tiny(8)
    o = Oracle(s)
    dmin = s.eig[:, s.n_occ:].min() - s.eig[:, :s.n_occ].max()
    q = 1
    B = o.B(q)
    c_im = o.chi0(q, B, omega=np.array([0.3]))[0]
    c_0 = o.chi0(q, B, omega=np.array([0.0]))[0]
    c_re = o.chi0_real(q, np.array([0.0, 0.7 * dmin]), B)
    assert np.max(np.abs(c_re[0] - c_0)) < 1e-15 * np.max(np.abs(c_0)) + 1e-300
    for lo, hi in ((c_im, c_0), (c_0, c_re[1])):
        ev = np.linalg.eigvalsh(lo - hi)
        assert ev.min() > -1e-12 * np.max(np.abs(ev))


def test_linearised_qp():
    """E = e + Z (S(e) + e_static), Z = 1/(1 - S'(e)): exact for a linear S."""
    eps = np.array([-0.1, 0.2])
    slope, off = -0.25, np.array([0.03, -0.02])
    S = lambda E: off + slope * (E - eps)
    E, Z = contour.qp_linear(S(eps - 0.01), S(eps), S(eps + 0.01), 0.01, eps, np.array([0.1, 0.0]))
    assert np.allclose(Z, 1.0 / 1.25)
    assert np.allclose(E - eps, S(E) + np.array([0.1, 0.0]))


def _exact_broadened(o, E, eta, gamma):
    """Re Sigma^c of contour deformation with the residues of W^c taken at
    w + i eta, in closed form from the pole decomposition: the eta = 0 pole
    sum plus sum_m theta_m Re[X_nm(|z| + i eta) - X_nm(|z|)], with
    X(w) = -sum_s |x^T v_s|^2 / (Omega_s^2 - w^2) for any complex w (the
    imaginary-axis integral does not depend on eta)."""
    s = o.sys
    out = _exact_sigma(o, E, gamma).real
    occ = np.arange(s.n_bands) < s.n_occ
    for q in range(s.n_k):
        Om, v = _poles(o, q, gamma)
        x = o.x(q)
        c2 = np.abs(np.einsum("kanm,as->knms", x, v)) ** 2
        for k in range(s.n_k):
            em = s.eig[o.kmq[k, q]]
            for n in range(x.shape[2]):
                z = E[..., k, n][..., None] - em                         # [..., m]
                th = contour.residue_sign(z, occ)
                w = np.abs(z)[..., None]
                Xb = -np.sum(c2[k, n][None] / (Om ** 2 - (w + 1j * eta) ** 2), -1)
                X0 = -np.sum(c2[k, n][None] / (Om ** 2 - w ** 2), -1)
                out[..., k, n] += np.sum(th * (Xb.real - X0), -1) / s.n_k
    return out


@pytest.mark.parametrize("gamma", [False, True])
def test_broadened_screening_is_the_pole_form(gamma):
    """W^c at w + i eta from the complex-weight response and the general
    (non-Hermitian) screening equals the analytic pole form
    -sum_s v_s v_s^H / (Omega_s^2 - (w + i eta)^2) above the first transition
    as well as below it."""
    s = _tiny(8)
    o = Oracle(s)
    omr = np.linspace(0.0, 3.0, 13)
    eta = 0.05
    for q in (0, 1):
        Om, v = _poles(o, q, gamma)
        W = o.wc_real(q, omr, gamma=gamma, eta=eta)
        z = omr + 1j * eta
        ref = -np.einsum("as,ws,bs->wab", v, 1.0 / (Om[None, :] ** 2 - z[:, None] ** 2), v.conj())
        assert np.max(np.abs(W - ref)) < 1e-11 * np.max(np.abs(ref)), q
        assert np.max(np.abs(W[3] - W[3].conj().T)) > 1e-6 * np.max(np.abs(W[3]))   # not Hermitian


@pytest.mark.parametrize("gamma", [False, True])
def test_broadened_contour_deformation_every_state(gamma):
    """Re Sigma^c by contour deformation with the broadened real grid, for
    energies across the whole band range (residues far above the first
    transition), against the closed form; the interpolation error falls with
    the grid step."""
    s = _tiny()
    o = Oracle(s)
    eta = 0.05
    E = np.random.default_rng(2).uniform(s.eig.min() - 0.1, s.eig.max() + 0.1, (2, s.n_k, s.spec.n_qp))
    top = float(np.max(np.abs(E[..., None] - s.eig[:, None, None, :]))) + 0.01
    ex = _exact_broadened(o, E, eta, gamma)
    errs = []
    for h in (eta / 4, eta / 8):
        n_r = int(np.ceil(top / h)) + 1
        got = o.sigma_cd(n_r, (n_r - 1) * h, E, gamma=gamma, eta=eta)
        assert np.all(np.isfinite(got))
        errs.append(np.max(np.abs(got - ex)) / np.max(np.abs(ex)))
    assert errs[1] < 2e-4 and errs[1] < errs[0] / 4, errs


def test_qp_iteration_solves_the_qp_equation():
    """Newton steps on E - e - Re Sigma^c(E) from e: after four the QP equation
    holds to 1e-9 Ha for every state, and the first step is the linearised
    energy."""
    s = _tiny()
    o = Oracle(s)
    eta = 0.05
    top = float(s.eig.max() - s.eig.min()) + 1.0
    h = eta / 4
    n_r = int(np.ceil(top / h)) + 1
    E1, Z1, _ = o.qp_cd(n_r, (n_r - 1) * h, eta, 1)
    eps = s.eig[:, o.qp]
    S3 = o.sigma_cd(n_r, (n_r - 1) * h, np.stack([eps - 0.002, eps, eps + 0.002]), eta=eta)
    El, Zl = contour.qp_linear(S3[0], S3[1], S3[2], 0.002, eps, s.e_static)
    assert np.max(np.abs(E1 - El)) < 1e-13
    E, Z, S = o.qp_cd(n_r, (n_r - 1) * h, eta, 4)
    res = E - eps - s.e_static - o.sigma_cd(n_r, (n_r - 1) * h, E[None], eta=eta)[0]
    assert np.max(np.abs(res)) < 1e-9
