"""Pade (Thiele) pins: reproduces rational functions from exact data."""
import numpy as np
import pytest

from oracle import continuation, grids


@pytest.mark.parametrize("n_poles,n_freq,n_par", [(1, 16, 4), (4, 16, 9), (4, 32, 16), (6, 48, 16)])
def test_rational_function_reproduced(n_poles, n_freq, n_par):
    rng = np.random.default_rng(11 + n_poles)
    poles = rng.uniform(-1.5, 1.5, n_poles) + 1j * rng.choice([-1, 1], n_poles) * rng.uniform(0.05, 0.5, n_poles)
    res = rng.uniform(0.1, 1.0, n_poles) * np.exp(1j * rng.uniform(0, 2 * np.pi, n_poles))
    f = lambda z: np.sum(res / (z - poles))
    omega, _ = grids.frequency_grid(n_freq, 0.5)
    idx = grids.pade_nodes(n_freq, n_par)
    z = 1j * omega[idx]
    a, n_used = continuation.thiele_coeffs(z, np.array([f(zz) for zz in z]))
    for x in np.linspace(-2, 2, 41):
        val, der = continuation.thiele_eval(z, a, x)
        assert abs(val - f(x)) < 1e-9 * max(1, abs(f(x)))
        fd = (f(x + 1e-6) - f(x - 1e-6)) / 2e-6
        assert abs(der - fd) < 1e-5 * max(1, abs(fd))


def test_interpolates_nodes():
    rng = np.random.default_rng(3)
    z = 1j * np.linspace(0.1, 5, 8)
    fv = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    a, n = continuation.thiele_coeffs(z, fv)
    assert n == 8
    for zz, ff in zip(z, fv):
        assert abs(continuation.thiele_eval(z, a, zz)[0] - ff) < 1e-10


def test_truncates_on_zero_coefficient():
    z = 1j * np.array([0.1, 0.5, 1.0, 2.0])
    a, n = continuation.thiele_coeffs(z, np.zeros(4))
    assert n == 0
    val, der = continuation.thiele_eval(z, a, 0.3)
    assert val == 0 and der == 0
    # constant function: a_2 = 0 -> truncated after the first coefficient
    a, n = continuation.thiele_coeffs(z, np.full(4, 0.7 + 0.1j))
    assert n == 1 and abs(continuation.thiele_eval(z, a, 0.3)[0] - (0.7 + 0.1j)) < 1e-15


def test_qp_no_root_reports_failure():
    # Re P(E - mu) = 5 for all E (constant): E - e - 5 = 0 -> root at e + 5, outside the +-1 Ha scan
    z = 1j * np.array([0.1, 0.5])
    a, _ = continuation.thiele_coeffs(z, np.array([5.0 + 0j, 5.0 + 0j]))
    E, Z, ok = continuation.solve_qp(0.2, 0.0, 0.0, z, a)
    # Newton solves a linear equation in one step
    assert ok and abs(E - 5.2) < 1e-12


def test_qp_ignores_pole_crossings():
    """f(E) = E - e - Re P(E) with P(z) = r/(z - p): near the pole f jumps from +inf
    to -inf (a decreasing sign change); the QP root is an increasing crossing."""
    r, pole, e0 = 0.02, 0.03, 0.0
    f = lambda zz: r / (zz - pole)
    z = 1j * np.array([0.05, 0.3, 1.0, 3.0])
    a, _ = continuation.thiele_coeffs(z, np.array([f(zz) for zz in z]))
    E, Z, ok = continuation.solve_qp(e0, 0.0, 0.0, z, a)
    assert ok
    # roots of E - r/(E - p) = 0: E = (p +- sqrt(p^2 + 4r)) / 2, both increasing crossings
    roots = [(pole - np.sqrt(pole ** 2 + 4 * r)) / 2, (pole + np.sqrt(pole ** 2 + 4 * r)) / 2]
    assert min(abs(E - x) for x in roots) < 1e-9
    fd = 1 + r / (E - pole) ** 2
    assert Z > 0 and abs(Z - 1 / fd) < 1e-9
