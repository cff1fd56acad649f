"""Pins of the direction-averaged q -> 0 screening (oracle
`screening.screen_gamma_average`).

* The wings of Eq. dielectric_func_gamma are odd in q_hat and the head and
  body even, so eps~(-q_hat) = D eps~(q_hat) D with D = diag(-1, 1, ..., 1)
  in the Coulomb eigenbasis.  The mean over q_hat and -q_hat is therefore
  W^c built from eps~^{-1} with its wing blocks removed.  That follows from
  the block structure alone, not from the averaging code.
* Time reversal maps Sigma^c(-k) with q_hat onto Sigma^c(k) with -q_hat, so
  an average over a direction set closed under negation (the six Cartesian
  half-axes) makes Sigma^c(k) = Sigma^c(-k) on a grid with non-invariant k
  points, which a single direction does not."""
import numpy as np

from oracle import screening
from oracle.pipeline import Oracle
from synth.systems import cartesian_directions, make_custom, momentum_vectors, project_momentum


def _cell():
    return make_custom(n_atoms=2, nb_per_atom=5, naux_per_atom=7, nk=(3, 1, 2), n_occ=3, n_freq=8, qp_lo=1, n_qp=4,
                       seed=29)


def test_pair_average_removes_the_wings():
    s = _cell()
    o = Oracle(s)
    B0 = o.B(0)
    p = project_momentum(momentum_vectors(s), [[0.6, 0.0, 0.8]])[0]
    eps_l, _, _ = screening.screen_gamma(B0, s.eig, s.n_occ, p, s.omega_cell, s.V[0], o.omega)
    v, X = screening.coulomb_eigenbasis(s.V[0])
    T = X * np.sqrt(v)[None, :]
    want = np.empty_like(eps_l)
    for j in range(len(o.omega)):
        E = np.linalg.inv(eps_l[j])
        E[0, 1:] = 0.0
        E[1:, 0] = 0.0
        want[j] = T @ (E - np.eye(len(v))) @ T.conj().T
    got = screening.screen_gamma_average(B0, s.eig, s.n_occ, [p, -p], [0.5, 0.5], s.omega_cell, s.V[0], o.omega)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))
    single = screening.screen_gamma(B0, s.eig, s.n_occ, p, s.omega_cell, s.V[0], o.omega)[2]
    assert np.max(np.abs(single - want)) > 1e-6 * np.max(np.abs(want))   # the wings matter here


def test_symmetric_direction_set_restores_time_reversal():
    s = _cell()
    o = Oracle(s)
    ks = list(range(s.n_k))
    q, w = cartesian_directions()
    pd = project_momentum(momentum_vectors(s), q)
    one = o.run(ks)["sigma"]
    o.gamma_dirs = (pd, w)
    avg = o.run(ks)["sigma"]
    m = o.minus
    rel = lambda a: np.max(np.abs(a - a[m])) / np.max(np.abs(a))
    assert rel(avg) < 1e-12
    assert rel(one) > 1e-8


def test_momentum_vectors_time_reversal():
    """The synthetic Cartesian momenta obey p(-k) = -conj(p(k)) and are purely
    imaginary at the time-reversal-invariant points; the projection is linear."""
    from oracle import grids
    s = _cell()
    p3 = momentum_vectors(s)
    _, _, minus = grids.kq_tables(s.spec.nk)
    assert np.max(np.abs(p3 + np.conj(p3[:, minus]))) == 0.0
    inv = [k for k in range(s.n_k) if minus[k] == k]
    assert inv and np.max(np.abs(p3[:, inv].real)) == 0.0
    q, _ = cartesian_directions()
    pd = project_momentum(p3, q)
    assert np.array_equal(pd[0], p3[0]) and np.array_equal(pd[1], -p3[0]) and np.array_equal(pd[5], -p3[2])
