"""Correlation self-energy on the imaginary axis (oracle; test infrastructure).

Eq. GW_selfe_element of the paper with the full W replaced by its correlation
part W^c = W - V and the BZ weight w_q = 1/N_q restored:

  Sigma^c_n(k, i w) = -1/(2 pi) sum_{m,q} w_q int dw'
        X_nm(k,q,w') / (i w - i w' + mu - e_m^{k-q}),
  X_nm(k,q,w') = sum_{mu nu} C^mu_{nm}(k,k-q) W^c_{mu nu}(q,iw') C^nu_{mn}(k-q,k).

With time-reversal symmetric inputs W^c(iw') = W^c(-iw'), so the integral over
the whole axis folds onto (0, inf):

  Sigma^c_n(k, i w_i) = -1/pi sum_q w_q sum_m sum_j g_j X_nm(k,q,w_j)
                        * a / (a^2 + w_j^2),       a = i w_i + mu - e_m^{k-q},

with (w_j, g_j) the frequency grid.  `sigma_c_unfolded` evaluates the same
integral with both signs of w' kept separately; the two must agree.

The exchange part is the bare-Coulomb term of the same equation (W_0 = V +
W^c).  V does not depend on w', and the frequency integral of the Green's
function taken with the equal-time convergence factor of the exchange term
gives 2 pi for an occupied band and 0 otherwise, so

  Sigma^x_n(k) = -sum_q w_q sum_{m occ} sum_{mu nu} C^mu_{nm}(k,k-q) V_{mu nu}(q) C^nu_{mn}(k-q,k),

static, with V(0) the truncated Coulomb matrix as in the screening (Sec. III B).
"""
from __future__ import annotations

import numpy as np


def pair_weights(x, Wc, xc=None):
    """X[k][n][m][j] = sum_{mu nu} x^mu_nm(k) W^c_{mu nu}(w_j) xc^nu_mn(k).

    x: [N_k][N_aux][N_qp][N_bands] = C^mu_{nm}(k,k-q).
    xc: the second triple coefficient C^nu_{mn}(k-q,k) in [N_k][N_aux][N_qp][N_bands]
        order (defaults to conj(x)).  Returns complex [N_k][N_qp][N_bands][N_w].
    """
    if xc is None:
        xc = np.conj(x)
    n_k, n_aux, nq, nb = x.shape
    out = np.empty((n_k, nq, nb, Wc.shape[0]), dtype=np.complex128)
    for k in range(n_k):
        xa = x[k].reshape(n_aux, -1)
        xb = xc[k].reshape(n_aux, -1)
        for j in range(Wc.shape[0]):
            out[k, :, :, j] = np.sum(xa * (Wc[j] @ xb), axis=0).reshape(nq, nb)
    return out


def sigma_c_q(X, eig, kmq, q, mu, omega, weight, n_q):
    """Folded contribution of one q; X from `pair_weights` (real part used)."""
    n_k, nq, nb, nw = X.shape
    sig = np.zeros((n_k, nq, len(omega)), dtype=np.complex128)
    for k in range(n_k):
        em = eig[kmq[k, q]]                                    # [nb]
        for i, w in enumerate(omega):
            a = 1j * w + mu - em                               # [nb]
            ker = a[:, None] / (a[:, None] ** 2 + omega[None, :] ** 2)   # [nb][nw]
            sig[k, :, i] = np.einsum("nmj,mj->n", X[k].real * weight[None, None, :], ker)
    return -(1.0 / np.pi) * sig / n_q


def sigma_c_unfolded(X, eig, kmq, q, mu, omega, weight, n_q):
    """Same integral over the whole imaginary axis, nodes +-w_j kept apart."""
    n_k, nq, nb, nw = X.shape
    sig = np.zeros((n_k, nq, len(omega)), dtype=np.complex128)
    for k in range(n_k):
        em = eig[kmq[k, q]]
        for i, w in enumerate(omega):
            for sgn in (1.0, -1.0):
                den = 1j * w - 1j * sgn * omega[None, :] + mu - em[:, None]     # [nb][nw]
                sig[k, :, i] += np.einsum("nmj,mj->n", X[k] * weight[None, None, :], 1.0 / den)
    return -(1.0 / (2.0 * np.pi)) * sig / n_q


def sigma_x_q(x_occ, V, n_q):
    """Contribution of one q to the exchange self-energy.

    x_occ: [N_k][N_aux][N_qp][N_occ] = C^mu_{nm}(k,k-q) for occupied m.
    V: [N_aux][N_aux] Coulomb matrix of this q.  Returns float64 [N_k][N_qp]:
    -(1/N_q) sum_{m occ} X_nm with X from `pair_weights` (V as its one frequency).
    """
    X = pair_weights(x_occ, V[None])[..., 0]
    return -X.real.sum(axis=2) / n_q
