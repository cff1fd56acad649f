"""Pins of the oracle's exchange self-energy (the bare-Coulomb term of
Eq. GW_selfe_element with the occupied sum), each against something other
than the formula it evaluates."""
import numpy as np
import pytest

from oracle import selfenergy


@pytest.fixture(scope="module")
def c1_sigma_x(c1_oracle):
    return c1_oracle.sigma_x()


def test_nonpositive(c1_oracle, c1_sigma_x):
    # V(q) is Hermitian positive definite, so every x^H V x >= 0 and
    # Sigma^x <= 0 for every state
    assert c1_sigma_x.shape == (c1_oracle.sys.n_k, c1_oracle.sys.spec.n_qp)
    assert np.all(c1_sigma_x < 0.0)


def test_quadratic_form_through_cholesky_factor(c1_oracle):
    # X = sum_{mu nu} x_mu V_{mu nu} conj(x_nu) = || L^T x ||^2 for V = L L^H:
    # a transposed or conjugated V in the contraction breaks the equality
    s = c1_oracle.sys
    for q in (1, s.n_k - 1):
        xo = c1_oracle.x_occ(q)                      # [k][mu][n][m]
        L = np.linalg.cholesky(s.V[q])
        direct = selfenergy.pair_weights(xo, s.V[q][None])[..., 0]
        via_l = np.sum(np.abs(np.einsum("mu,kmab->kuab", L, xo)) ** 2, axis=1)
        assert np.max(np.abs(direct.imag)) < 1e-12 * np.max(np.abs(direct.real))
        assert np.allclose(direct.real, via_l, rtol=1e-12, atol=0)


@pytest.fixture(scope="module")
def nontrim_oracle():
    # a 3x1x2 grid: most q are not time-reversal invariant, so V(q) is complex
    from oracle.pipeline import Oracle
    from synth.systems import make_custom
    return Oracle(make_custom(n_atoms=2, nb_per_atom=4, naux_per_atom=7, nk=(3, 1, 2), n_occ=2, n_freq=8,
                              qp_lo=0, n_qp=4, seed=31))


def test_minus_q_relabelling(nontrim_oracle):
    # The sum runs over every q, so q -> -q gives the same total from the
    # pairs (k, k+q) with V(-q) = conj(V(q)).  Pairing V(q) with k+q instead
    # (the conjugation slip of the response's V pairing) does not.
    o, s = nontrim_oracle, nontrim_oracle.sys
    ref = o.sigma_x()
    tot = np.zeros_like(ref)
    wrong = np.zeros_like(ref)
    for q in range(s.n_k):
        xp = np.stack([o.tb.mo(k, o.kpq[k, q], o.qp, o.occ) for k in range(s.n_k)])
        tot += selfenergy.sigma_x_q(xp, np.conj(s.V[q]), s.n_k)
        wrong += selfenergy.sigma_x_q(xp, s.V[q], s.n_k)
    assert np.max(np.abs(s.V[2].imag)) > 1e-3   # q = (1/3, 0, 0)
    assert np.allclose(tot, ref, rtol=1e-12, atol=1e-14)
    assert np.max(np.abs(wrong - ref)) > 1e-6 * np.max(np.abs(ref))


def test_occupied_subspace_rotation(c1_oracle):
    # A unitary mixing of the occupied bands at k-q leaves the occupied sum
    # unchanged; mixing an occupied band with an unoccupied one does not
    o, s = c1_oracle, c1_oracle.sys
    q = 1
    xo = o.x_occ(q)
    ref = selfenergy.sigma_x_q(xo, s.V[q], s.n_k)
    rng = np.random.default_rng(7)
    a = rng.standard_normal((s.n_occ, s.n_occ)) + 1j * rng.standard_normal((s.n_occ, s.n_occ))
    U, _ = np.linalg.qr(a)
    rot = np.einsum("kuam,mp->kuap", xo, U)
    assert np.allclose(selfenergy.sigma_x_q(rot, s.V[q], s.n_k), ref, rtol=1e-12, atol=1e-14)
    xa = np.stack([o.tb.mo(k, o.kmq[k, q], o.qp, slice(0, s.n_occ + 1)) for k in range(s.n_k)])
    c, sn = np.cos(0.3), np.sin(0.3)
    mixed = xa[..., :s.n_occ].copy()
    mixed[..., -1] = c * xa[..., s.n_occ - 1] + sn * xa[..., s.n_occ]
    assert np.max(np.abs(selfenergy.sigma_x_q(mixed, s.V[q], s.n_k) - ref)) > 1e-6 * np.max(np.abs(ref))


def test_time_reversal(c1_oracle, c1_sigma_x):
    # time-reversal symmetric inputs: Sigma^x_n(k) = Sigma^x_n(-k)
    m = c1_oracle.minus
    assert np.allclose(c1_sigma_x, c1_sigma_x[m], rtol=1e-12, atol=1e-14)
