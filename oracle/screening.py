"""Screening: symmetrised dielectric matrix, its inverse and the correlation
part of the screened interaction (oracle; test infrastructure).

Eq. symm_dielec_func:  eps~(q,iw) = I - V^{1/2} chi~ V^{1/2}
Eq. screened_W_matr:   W(q,iw)   = V^{1/2} eps~^{-1} V^{1/2}
Correlation part:      W^c = W - V = V^{1/2} (eps~^{-1} - I) V^{1/2}
V^{1/2} is the Hermitian square root from an eigendecomposition, as the paper
writes it.  With a truncated Coulomb matrix V^cut(q) (Sec. III B), V^cut
takes the place of V in the numerator only: W^c = V^cut^{1/2} (eps~^{-1} - I)
V^cut^{1/2}, eps~ from the full V (`screen(chi, V, Vcut)`).

At q = 0 (Sec. III B, Eq. dielectric_func_gamma) the dielectric matrix is
built in the eigenbasis X, v of the truncated Coulomb matrix V^cut(0), with
lambda = 1 the eigenvector of the largest eigenvalue (the G = 0 plane-wave
like state).  For an insulator (no intraband term) with momentum elements
p_ia = p_{ia}(k).q_hat, every block of Eq. dielectric_func_gamma is one Gram
form over occupied/unoccupied pairs:

  eps~_{lam lam'} = delta + s/N_k sum_k sum_ia 2D/(D^2+w^2) y_lam conj(y_lam')
  y_1        = sqrt(4 pi / Omega) p_ia / D_ia                (head, wings)
  y_{lam>1}  = sqrt(v_lam) (X^H B_ia)_lam                     (body)

with Omega the cell volume and w_k = 1/N_k throughout (the head of the
printed equation omits the k weight and the wings carry 1/sqrt(N_k); reading
Omega as the crystal volume N_k * Omega_cell makes all three consistent).  The
body is exactly the regular formula in the eigenbasis.  The result is
transformed back with X and W^c(0) = X sqrt(v) (eps~_lam^{-1} - I) sqrt(v) X^H,
V^cut entering the numerator.  The sign of the real eigenvector X_1 is fixed
so that its largest-magnitude component is positive.

What is pinned: the head against the printed band-pair sum of the equation
(every pair with its occupation difference, Omega the crystal volume); the
body against the regular formula (p = 0); the Gram structure (eigenvalues of
eps~ >= 1) and the N_aux = 1 closed form; the wings' oddness in q_hat (a set
closed under q_hat -> -q_hat removes them).  PARITY UNPINNED for the phase of
the wings: they carry the phase of p_ia relative to the triple coefficients
B_ia(k,0), which is fixed by how the momentum elements are defined (psi_i^k
on the left, the convention that makes y_1 the q -> 0 limit of the G = 0-like
component of B(k,q)), and synthetic momentum elements carry no such relation
to B.  Two plausible errors therefore pass every pin here:
  * a wing of the wrong sign (or any constant phase on p): it changes W^c(0)
    of one direction only through the wing blocks, and the average over a
    set closed under q_hat -> -q_hat is unchanged by it;
  * conjugated momentum elements (p_ai in place of p_ia): head and body of
    eps~ are unchanged, but the wing differs in more than a phase, and W^c(0)
    moves even after the average (relative 5e-4 on the small cell), since the
    wings enter the head and body of eps~^{-1} at second order.
Both are checked to pass the pins in tests/test_oracle_screening.py.
"""
from __future__ import annotations

import numpy as np

from .response import SPIN
from .response import weight as response_weight


def sqrt_hpd(V):
    lam, U = np.linalg.eigh(V)
    if lam.min() <= 0.0:
        raise ValueError("Coulomb matrix is not positive definite")
    return (U * np.sqrt(lam)[None, :]) @ U.conj().T


def screen(chi, V, Vcut=None):
    """chi: [N_w][N][N], V: [N][N].  Returns (eps~, W^c) per frequency.

    Vcut (Sec. III B, after Eq. cut_coulomb_pot): the truncated Coulomb
    matrix V^cut(q).  It replaces V in the numerator of Eq. screened_W_matr
    (the two V^{1/2} factors) while eps~ keeps the full V:
        W^c = Vcut^{1/2} (eps~^{-1} - I) Vcut^{1/2},  eps~ = I - V^{1/2} chi V^{1/2},
    both square roots the Hermitian (principal) ones, as the equation writes
    them.  None: V in both places."""
    Vh = sqrt_hpd(V)
    Vch = Vh if Vcut is None else sqrt_hpd(Vcut)
    n = V.shape[0]
    eye = np.eye(n)
    eps = np.empty_like(chi)
    Wc = np.empty_like(chi)
    for iw in range(chi.shape[0]):
        eps[iw] = eye - Vh @ chi[iw] @ Vh
        Wc[iw] = Vch @ (np.linalg.inv(eps[iw]) - eye) @ Vch
    return eps, Wc


def coulomb_eigenbasis(Vcut0):
    """Eigenpairs of V^cut(0), descending; X_1 sign fixed (largest |component| > 0)."""
    v, X = np.linalg.eigh(Vcut0)
    order = np.argsort(v)[::-1]
    v = v[order]
    X = X[:, order].copy()
    j = np.argmax(np.abs(X[:, 0]))
    ph = X[j, 0] / abs(X[j, 0])
    X[:, 0] /= ph
    return v, X


def screen_gamma(B0, eig, n_occ, p, omega_cell, Vcut0, omega, s=SPIN, real_axis=False, eta=0.0):
    """q = 0 dielectric matrix in the Coulomb eigenbasis and W^c(0).

    B0: [N_k][N_aux][N_occ][N_unocc] = C^mu_{ia}(k,k); p: [N_k][N_occ][N_unocc].
    real_axis: real frequencies below the smallest transition, weight
    2D/(D^2 - w^2); with eta > 0 at w + i eta (as in `response.chi0_trs`).
    Returns (eps~_lambda, eps~_mu, W^c) per frequency.
    """
    n_k, n_aux = B0.shape[0], B0.shape[1]
    v, X = coulomb_eigenbasis(Vcut0)
    if v[-1] <= 0.0:
        raise ValueError("truncated Coulomb matrix is not positive definite")
    sv = np.sqrt(v)
    eye = np.eye(n_aux)
    eps_l = np.tile(eye.astype(np.complex128), (len(omega), 1, 1))
    for k in range(n_k):
        delta = (eig[k][n_occ:][None, :] - eig[k][:n_occ][:, None]).reshape(-1)
        Y = sv[:, None] * (X.conj().T @ B0[k].reshape(n_aux, -1))          # [lam][ia]
        Y[0, :] = np.sqrt(4.0 * np.pi / omega_cell) * p[k].reshape(-1) / delta
        for iw, w in enumerate(omega):
            wt = response_weight(delta, w, real_axis, eta)
            eps_l[iw] += (s / n_k) * (Y * wt[None, :]) @ Y.conj().T
    eps_mu = np.empty_like(eps_l)
    Wc = np.empty_like(eps_l)
    for iw in range(len(omega)):
        eps_mu[iw] = X @ eps_l[iw] @ X.conj().T
        Wc[iw] = (X * sv[None, :]) @ (np.linalg.inv(eps_l[iw]) - eye) @ (sv[:, None] * X.conj().T)
    return eps_l, eps_mu, Wc


def screen_gamma_average(B0, eig, n_occ, p_dirs, weights, omega_cell, Vcut0, omega, s=SPIN, real_axis=False, eta=0.0):
    """W^c(q -> 0) averaged over directions q_hat_d: sum_d w_d W^c(q_hat_d), each
    from `screen_gamma` with p_ia . q_hat_d (p_dirs: [n_dir][N_k][N_occ][N_unocc]).
    The paper notes that head and wings depend on the direction of approach
    and gives no averaging scheme; this weighted mean is the reading."""
    return sum(w * screen_gamma(B0, eig, n_occ, pd, omega_cell, Vcut0, omega, s=s, real_axis=real_axis, eta=eta)[2]
               for pd, w in zip(p_dirs, weights))

