"""Pins of the learned-surrogate oracle (oracle/surrogate.py)."""
import numpy as np
import pytest

from oracle import grids, surrogate as sg
from synth.systems import bf16_round, surrogate_init, surrogate_start


def test_anchor_layout():
    # j (N-1)/(n-1) rounded half up: 31/5 * j = 0, 6.2, 12.4, 18.6, 24.8, 31
    a = sg.anchor_indices(32, 6)
    assert list(a) == [0, 6, 12, 19, 25, 31]
    assert sg.holdout_index(a) == 15
    a = sg.anchor_indices(40, 6)           # 39/5 j = 0, 7.8, 15.6, 23.4, 31.2, 39
    assert list(a) == [0, 8, 16, 23, 31, 39]
    assert sg.holdout_index(a) == 19
    t = sg.target_indices(40, a)
    assert len(t) == 34 and 19 in t and not set(t) & set(a)


def test_rule_is_identity_on_anchors():
    om, _ = grids.frequency_grid(32, 0.5)
    a = sg.anchor_indices(32, 6)
    C = sg.rule_weights(om, a, a, 0.1, 2.8)
    # in units of the anchor column norms (the scale of each anchor's values)
    n = np.linalg.norm(sg.kernel(sg.delta_family(0.1, 2.8), om[a]), axis=0)
    assert np.abs(n[:, None] * C / n[None, :] - np.eye(6)).max() < 1e-5


def test_rule_solves_regularised_normal_equations():
    # the augmented least-squares solution is the minimiser: normal equations hold
    om, _ = grids.frequency_grid(32, 0.5)
    a = sg.anchor_indices(32, 6)
    t = sg.target_indices(32, a)
    C = sg.rule_weights(om, a, t, 0.1, 2.8, ridge=1e-6)
    D = sg.delta_family(0.1, 2.8)
    G = sg.kernel(D, om[a])
    n2 = np.sum(G * G, axis=0)
    lhs = (G.T @ G + 1e-6 * np.diag(n2)) @ C
    rhs = G.T @ sg.kernel(D, om[t])
    assert np.abs(lhs - rhs).max() < 1e-8 * np.abs(rhs).max()


def test_rule_interpolates_transition_sums():
    # random positive mixtures of transitions inside the window: the rule's
    # error is small against the anchor norm, and zero-window mistakes are not
    om, _ = grids.frequency_grid(32, 0.5)
    a = sg.anchor_indices(32, 6)
    t = sg.target_indices(32, a)
    C = sg.rule_weights(om, a, t, 0.1, 2.8)
    rng = np.random.default_rng(3)
    worst = 0.0
    for _ in range(50):
        D = rng.uniform(0.1, 2.8, 200)
        w = rng.exponential(1.0, 200)
        f = (sg.kernel(D, om) * w[:, None]).sum(0)
        worst = max(worst, np.abs(f[a] @ C - f[t]).max() / np.linalg.norm(f[a]))
    assert worst < 1e-2
    # a single transition well outside the window is not reproduced
    f = sg.kernel([30.0], om)[0]
    assert np.abs(f[a] @ C - f[t]).max() / np.linalg.norm(f[a]) > worst


def test_cholesky_qr_matches_householder():
    rng = np.random.default_rng(1)
    Y = rng.normal(size=(40, 7)) + 1j * rng.normal(size=(40, 7))
    Q = sg.cholesky_qr(Y)
    assert np.abs(Q.conj().T @ Q - np.eye(7)).max() < 1e-12
    Qh, Rh = np.linalg.qr(Y)
    ph = np.diag(Rh) / np.abs(np.diag(Rh))          # make diag(R) real positive
    assert np.abs(Q - Qh * ph.conj()[None, :]).max() < 1e-12


def test_subspace_basis_finds_dominant_eigenspace():
    rng = np.random.default_rng(2)
    n, r = 60, 8
    V, _ = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
    lam = np.concatenate([np.linspace(100, 50, r), rng.uniform(0, 1, n - r)])
    chi = -(V * lam) @ V.conj().T                  # negative semidefinite like chi0
    U = sg.subspace_basis(chi, surrogate_start(n, r, 5), n_iter=4)
    assert np.abs(U.conj().T @ U - np.eye(r)).max() < 1e-12
    Vr = V[:, :r]
    assert np.linalg.norm(Vr - U @ (U.conj().T @ Vr)) < 1e-5


def test_series_round_trip():
    rng = np.random.default_rng(4)
    r = 5
    A = rng.normal(size=(3, r, r)) + 1j * rng.normal(size=(3, r, r))
    P = A + np.swapaxes(A, -1, -2).conj()
    S = sg.to_series(P)
    assert S.shape == (3, r * r)
    assert S[1, 2 * r + 3] == P[1, 2, 3].real and S[1, 3 * r + 2] == P[1, 3, 2].imag
    assert np.abs(sg.from_series(S, r) - P).max() == 0.0


def test_features_scale_and_sign():
    rng = np.random.default_rng(5)
    a = rng.normal(size=(20, 6))
    x, s = sg.features(a)
    assert np.all(x[:, 0] >= 0)
    assert np.allclose(np.linalg.norm(x, axis=1), 1.0)
    assert np.allclose(x * s[:, None], a)
    for c in (3.0, -0.25):
        x2, s2 = sg.features(c * a)
        assert np.allclose(x2, x) and np.allclose(s2, c * s)
    x0, s0 = sg.features(np.zeros((2, 6)))
    assert np.all(x0 == 0) and np.all(s0 == 0)
    # series at the rounding level of the largest one carry no shape
    b = a.copy()
    b[3] *= 1e-7
    b[4] *= 1e-5
    xb, sb = sg.features(b)
    assert sb[3] == 0 and np.all(xb[3] == 0)
    assert sb[4] != 0 and np.allclose(xb[4], x[4])


def test_network_gradient_matches_central_differences():
    n_in, H, n_out = 6, 16, 5
    theta = surrogate_init(n_in, H, n_out, 11).astype(np.float64)
    theta[np.arange(theta.size) % 7 == 0] += 0.1    # nonzero biases too
    rng = np.random.default_rng(6)
    X = rng.normal(size=(9, n_in))
    Y = rng.normal(size=(9, n_out))
    _, g = sg.loss_grad(theta, X, Y, n_in, H, n_out)
    h = 1e-5
    fd = np.zeros_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        fd[i] = (sg.loss_grad(theta + e, X, Y, n_in, H, n_out)[0] - sg.loss_grad(theta - e, X, Y, n_in, H, n_out)[0]) / (2 * h)
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-7


def test_adam_first_step_is_sign_step():
    rng = np.random.default_rng(7)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    t1, m, v = sg.adam_step(theta, np.zeros(50), np.zeros(50), g, 1, 1e-3, eps=0.0)
    assert np.allclose(t1, theta - 1e-3 * np.sign(g), rtol=0, atol=1e-15)
    # second step with the same gradient: moments unchanged after bias correction
    t2, _, _ = sg.adam_step(t1, m, v, g, 2, 1e-3, eps=0.0)
    assert np.allclose(t2, theta - 2e-3 * np.sign(g), rtol=0, atol=1e-14)


def _toy_chi(n, n_freq, seed):
    rng = np.random.default_rng(seed)
    om, _ = grids.frequency_grid(n_freq, 0.5)
    K = 300
    B = (rng.normal(size=(K, n)) + 1j * rng.normal(size=(K, n))) / np.sqrt(n)
    D = rng.uniform(0.1, 2.8, K)
    g = sg.kernel(D, om)                            # [K][N_w]
    return -np.einsum('kw,ki,kj->wij', g, B, B.conj()), om


def test_rows_vanish_when_rule_is_exact():
    n, nw = 12, 16
    chi, om = _toy_chi(n, nw, 8)
    a = sg.anchor_indices(nw, 6)
    t = sg.target_indices(nw, a)
    C = sg.rule_weights(om, a, t, 0.1, 2.8)
    chi2 = chi.copy()
    chi2[t] = np.einsum('lt,lij->tij', C, chi[a])   # responses the rule reproduces exactly
    U = sg.subspace_basis(chi2[a[0]], surrogate_start(n, 4, 1))
    x, y = sg.training_rows(chi2, a, t, C, U)
    assert x.shape == (16, 6) and y.shape == (16, len(t))
    assert np.abs(y).max() < 1e-12


def test_prediction_consistent_with_training_rows():
    # a network that returned the training targets exactly would reproduce the
    # exact response inside the subspace and the rule outside it
    n, nw, r = 14, 16, 5
    chi, om = _toy_chi(n, nw, 9)
    a = sg.anchor_indices(nw, 6)
    t = sg.target_indices(nw, a)
    C = sg.rule_weights(om, a, t, 0.1, 2.8)
    U = sg.subspace_basis(chi[a[0]], surrogate_start(n, r, 2))
    x, y = sg.training_rows(chi, a, t, C, U)
    x2, s = sg.anchor_series(chi[a], U)
    assert np.allclose(x, x2)
    pred = sg.predict_from_residual(chi[a], C, U, y, s)
    Pp = np.einsum('ia,tij,jb->tab', U.conj(), pred, U)
    Pe = np.einsum('ia,tij,jb->tab', U.conj(), chi[t], U)
    assert np.abs(Pp - Pe).max() < 1e-12 * np.abs(Pe).max()
    base = np.einsum('lt,lij->tij', C, chi[a])
    Qc = np.eye(n) - U @ U.conj().T
    assert np.abs(Qc @ (pred - base) @ Qc).max() < 1e-12 * np.abs(base).max()


def test_prediction_is_odd_and_homogeneous():
    n, nw, r, H = 10, 16, 4, 12
    chi, om = _toy_chi(n, nw, 10)
    a = sg.anchor_indices(nw, 6)
    t = sg.target_indices(nw, a)
    C = sg.rule_weights(om, a, t, 0.1, 2.8)
    U = sg.subspace_basis(chi[a[0]], surrogate_start(n, r, 3))
    theta = surrogate_init(6, H, len(t), 4).astype(np.float64) * 3.0
    p1 = sg.predict(chi[a], C, U, theta, H)
    for c in (2.5, -0.7):
        p2 = sg.predict(c * chi[a], C, U, theta, H)
        assert np.abs(p2 - c * p1).max() < 1e-12 * np.abs(c * p1).max()
    # a network with zero output layer leaves the rule alone
    th0 = theta.copy()
    th0[-(H * len(t) + len(t)):] = 0.0
    assert np.abs(sg.predict(chi[a], C, U, th0, H) - np.einsum('lt,lij->tij', C, chi[a])).max() == 0.0


def test_bf16_round_is_representable():
    v = bf16_round(np.array([1.0, 1.00390625, 1.005859375, -3.14159], dtype=np.float32))
    assert v[0] == 1.0 and v[1] == 1.0          # 1 + 2^-8 ties to even -> 1
    assert v[2] == np.float32(1.0078125)        # 1 + 1.5 * 2^-8 rounds up
    assert np.all((v.view(np.uint32) & 0xFFFF) == 0)
