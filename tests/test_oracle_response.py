"""chi0 pins (oracle): literal Eq. chi0_matrix vs time-reversal form, Hermiticity,
negative semidefiniteness, evenness in w and the large-w tail."""
import numpy as np
import pytest

from oracle import response


@pytest.mark.parametrize("q", [0, 1, 3, 7])
def test_literal_equals_trs_form(c1_oracle, q):
    o = c1_oracle
    s = o.sys
    om = np.array([0.05, 0.7, 5.0])
    chi = o.chi0(q, omega=om)
    lit = response.chi0_literal(o.tb, s.eig, o.kpq, o.minus[q], s.n_occ, om)
    assert np.max(np.abs(lit - chi)) < 1e-13 * np.max(np.abs(chi))
    # the literal response is even in w on time-reversal-symmetric inputs
    lit_m = response.chi0_literal(o.tb, s.eig, o.kpq, o.minus[q], s.n_occ, -om)
    assert np.max(np.abs(lit_m - lit)) < 1e-13 * np.max(np.abs(chi))


@pytest.mark.parametrize("q", [0, 5])
def test_hermitian_nsd(c1_oracle, q):
    chi = c1_oracle.result["per_q"][q]["chi"]
    for c in chi:
        assert np.max(np.abs(c - c.conj().T)) <= 1e-15 * np.max(np.abs(c))
        lam = np.linalg.eigvalsh(c)
        assert lam.max() <= 1e-14 * np.abs(lam).max()


def test_large_frequency_tail(c1_oracle):
    o = c1_oracle
    s = o.sys
    q = 2
    B = o.B(q)
    # w^2 chi(w) -> -(2 s / N_k) sum D B B^H  (the -(2/w^2) sum |M|^2 D tail)
    ref = np.zeros((s.n_aux, s.n_aux), dtype=np.complex128)
    for k in range(s.n_k):
        d = (s.eig[o.kpq[k, q]][s.n_occ:][None, :] - s.eig[k][:s.n_occ][:, None]).reshape(-1)
        Bk = B[k].reshape(s.n_aux, -1)
        ref += (Bk * d[None, :]) @ Bk.conj().T
    ref *= -2.0 * 2.0 / s.n_k
    dmax = 2.8
    for w in (1e3, 1e4):
        chi = o.chi0(q, B=B, omega=np.array([w]))[0]
        rel = np.linalg.norm(w * w * chi - ref) / np.linalg.norm(ref)
        assert rel <= (dmax / w) ** 2
