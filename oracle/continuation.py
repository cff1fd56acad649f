"""Analytic continuation and the quasiparticle equation (oracle; test
infrastructure).

The paper continues the imaginary-axis self-energy to the real axis
analytically (Sec. II A, citing Rojas, Godby and Needs) without printing the
scheme.  The scheme used here is the Thiele continued fraction through n_par
points (Vidberg and Serene, J. Low Temp. Phys. 29, 179 (1977)):

  P(z) = a_1 / (1 + a_2 (z - z_1) / (1 + a_3 (z - z_2) / (1 + ...)))

with inverse differences g_1(z_j) = f_j,
  g_p(z_j) = (g_{p-1}(z_{p-1}) - g_{p-1}(z_j)) / ((z_j - z_{p-1}) g_{p-1}(z_j)),
  a_p = g_p(z_p),
and evaluation by the three-term recurrence
  A_0 = 0, A_1 = a_1, B_0 = B_1 = 1,
  A_p = A_{p-1} + a_p (z - z_{p-1}) A_{p-2}  (same for B),  P = A_n / B_n.
The fit stops at the first coefficient that is zero (|a_p| < 1e-300) or not
finite; the fraction is then truncated there.

Quasiparticle equation (variable z = E - mu, as Sigma^c(i w) was defined with
i w + mu in its denominators):
  E = e_n + e_static_n + Re P_n(E - mu),   Z = 1 / (1 - Re P_n'(E - mu)).
With f(E) = E - e_n - e_static_n - Re P(E - mu): Newton from
E_0 = e_n + e_static_n, |dE| < 1e-10 Ha, at most 50 steps, abandoned as soon as
f'(E) <= 0 (a quasiparticle root has f' = 1/Z > 0; f' <= 0 means the step
crossed a pole of the continued fraction, after which Newton wanders).  Then
scan E_0 +- 1 Ha in 1 mHa steps for increasing sign changes
f(E_i) < 0 <= f(E_{i+1}) (a pole of P with positive residue gives a decreasing
change), take the one whose midpoint is closest to E_0 and bisect it to
1e-12 Ha.  Z = 1 / f'(E).
"""
from __future__ import annotations

import numpy as np

PADE_TINY = 1e-300


def thiele_coeffs(z, f):
    n = len(z)
    g = np.array(f, dtype=np.complex128)
    a = np.zeros(n, dtype=np.complex128)
    a[0] = g[0]
    n_used = n
    if not (np.isfinite(a[0]) and abs(a[0]) >= PADE_TINY):
        return a[:0], 0
    for p in range(1, n):
        gp = g.copy()
        for j in range(p, n):
            gp[j] = (g[p - 1] - g[j]) / ((z[j] - z[p - 1]) * g[j])
        g = gp
        a[p] = g[p]
        if not np.isfinite(a[p]) or abs(a[p]) < PADE_TINY:
            n_used = p
            break
    return a[:n_used], n_used


def thiele_eval(z_nodes, a, z):
    """Value and derivative d/dz of the continued fraction at z."""
    if len(a) == 0:
        return 0.0j, 0.0j
    A0, A1 = 0.0 + 0.0j, a[0]
    B0, B1 = 1.0 + 0.0j, 1.0 + 0.0j
    dA0, dA1 = 0.0j, 0.0j
    dB0, dB1 = 0.0j, 0.0j
    for p in range(1, len(a)):
        t = a[p] * (z - z_nodes[p - 1])
        A2 = A1 + t * A0
        B2 = B1 + t * B0
        dA2 = dA1 + a[p] * A0 + t * dA0
        dB2 = dB1 + a[p] * B0 + t * dB0
        A0, A1, B0, B1 = A1, A2, B1, B2
        dA0, dA1, dB0, dB1 = dA1, dA2, dB1, dB2
    val = A1 / B1
    der = (dA1 * B1 - A1 * dB1) / (B1 * B1)
    return val, der


def solve_qp(e0, e_static, mu, z_nodes, a):
    """Returns (E_qp, Z, converged)."""
    target = e0 + e_static

    def f(E):
        v, d = thiele_eval(z_nodes, a, E - mu)
        return E - target - v.real, 1.0 - d.real

    E = target
    for _ in range(50):
        fv, fd = f(E)
        if not (np.isfinite(fv) and np.isfinite(fd)) or fd <= 0.0:
            break
        dE = fv / fd
        E = E - dE
        if abs(dE) < 1e-10:
            fv, fd = f(E)
            if fd > 0.0:
                return E, 1.0 / fd, True
            break
    # bracket scan: increasing sign changes only
    grid = target + np.arange(-1000, 1001) * 1e-3
    vals = np.array([f(x)[0] for x in grid])
    best = None
    for i in range(len(grid) - 1):
        if np.isfinite(vals[i]) and np.isfinite(vals[i + 1]) and vals[i] < 0.0 <= vals[i + 1]:
            mid = 0.5 * (grid[i] + grid[i + 1])
            if best is None or abs(mid - target) < abs(best[0] - target):
                best = (mid, i)
    if best is None:
        fv, fd = f(target)
        return target, 1.0 / fd, False
    lo, hi = grid[best[1]], grid[best[1] + 1]
    for _ in range(200):
        if hi - lo < 1e-12:
            break
        mid = 0.5 * (lo + hi)
        fm = f(mid)[0]
        if fm >= 0.0:
            hi = mid
        else:
            lo = mid
    E = 0.5 * (lo + hi)
    return E, 1.0 / f(E)[1], True


def qp_energies(sigma, omega, eps_qp, e_static, mu, node_idx):
    """sigma: [N_k][N_qp][N_w] on i*omega; returns (E_qp, Z, converged) arrays."""
    n_k, nq, _ = sigma.shape
    z = 1j * omega[node_idx]
    E = np.empty((n_k, nq))
    Z = np.empty((n_k, nq))
    ok = np.empty((n_k, nq), dtype=bool)
    for k in range(n_k):
        for n in range(nq):
            a, _ = thiele_coeffs(z, sigma[k, n, node_idx])
            E[k, n], Z[k, n], ok[k, n] = solve_qp(eps_qp[k, n], e_static[k, n], mu, z, a)
    return E, Z, ok
