"""Contour-deformation evaluation of the correlation self-energy at real
energies (oracle; test infrastructure).

The paper names contour deformation as the alternative to analytic
continuation (Sec. II A, after Eq. chi_0_realspace) and leaves the scheme to
the molecular implementation it cites (Golze et al. 2018).  Deforming the
real-axis frequency integral of G W^c onto the imaginary axis leaves the
imaginary-axis integral plus the residues of the Green-function poles that
the deformation passes over.  With the pair weights
X_nm(k,q,w) = x_nm^T W^c(q,w) conj(x_nm) of Eq. GW_selfe_element and
z = E - e_m(k-q):

  Sigma^c_n(k,E) = 1/N_q sum_q sum_m [ -(1/pi) int_0^inf dw X_nm(k,q,iw) z/(z^2+w^2)
                                       + theta_m(E) X_nm(k,q,|z|) ]

  theta_m(E) = +1 for an unoccupied m with e_m < E, -1 for an occupied m
  with e_m > E, half of that at E = e_m, 0 otherwise.

The first term is the imaginary-axis formula of `selfenergy.sigma_c_q` with
i w_i + mu replaced by the real E.  The sign of the residues follows from a
one-pole W^c, for which both sides are known in closed form.

Readings (the paper gives no scheme):
 * W^c on the real axis is needed only at the residue frequencies |z|.  They
   are taken below the smallest transition energy Delta_min, where chi0 has
   no poles: the response weight becomes 2D/(D^2 - w^2), chi~ stays
   Hermitian and eps~ positive definite.  This covers states near the band
   edges, whose residues come from levels between mu and E.  A state with a
   residue frequency beyond the real grid's top is not evaluated (NaN).
 * The imaginary-axis integral is taken on the modified Gauss-Legendre grid
   of the response with X(0) subtracted and its integral added in closed form
   (int_0^inf z/(z^2+w^2) dw = (pi/2) sgn z).  The remaining integrand
   vanishes like w^2 at 0, so the grid need not resolve the Lorentzian of
   width |z|.  X(0) is the first plane of the real grid (w = 0 lies on both
   axes).
 * X between the nodes w_r = r h (r = 0..n_r-1) of the uniform real grid is
   the 4-point Lagrange interpolant.  X is even in w, so at the left end the
   stencil reflects (X(-h) = X(h)).
 * QP energies from these values are linearised about e_n:
   E = e_n + Z (Sigma^c(e_n) + e_n^static), with Z = 1/(1 - dSigma^c/dE) from
   the central difference at e_n -+ delta.
 * Every state (residues above Delta_min): W^c is taken at the complex
   frequencies w_r + i eta of the real grid (the response weight
   2D/(D^2 - (w + i eta)^2) is complex, chi~ and eps~ are not Hermitian, the
   screening is the general inverse).  Only Re Sigma^c enters the QP
   equation, and Re X(w + i eta) is even in w (X(conj z) = conj X(z), W^c even
   in z), so the same reflection applies at w = 0; the imaginary-axis term is
   unchanged and its subtracted constant is Re X(i eta), whose closed-form
   integral is added back exactly.  eta is the broadening of the time-ordered
   W^c's poles: with a finite k grid the RPA spectrum is discrete, and eta
   smooths Sigma^c(E) over it; the grid step must resolve eta.
 * QP energies for every state: Newton steps on E - e_n - e_static - Re
   Sigma^c(E) from E_0 = e_n, the slope from the central difference at
   E -+ delta (the first step is the linearised energy).
"""
from __future__ import annotations

import numpy as np


def real_grid(n_r: int, omega_max: float):
    """Uniform real frequencies 0, h, ..., omega_max = (n_r-1) h."""
    if n_r < 4:
        raise ValueError("the 4-point interpolation needs n_r >= 4")
    return np.linspace(0.0, omega_max, n_r), omega_max / (n_r - 1)


def lagrange4(t):
    """Weights of nodes -1, 0, 1, 2 of the cubic through them, at t."""
    return np.stack([-t * (t - 1.0) * (t - 2.0) / 6.0,
                     (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0,
                     -(t + 1.0) * t * (t - 2.0) / 2.0,
                     (t + 1.0) * t * (t - 1.0) / 6.0])


def interp_real(Xr, h, w):
    """Xr[..., r] sampled at r h, interpolated at w (same leading shape as
    Xr[..., 0], 0 <= w <= (n_r-1) h)."""
    n_r = Xr.shape[-1]
    s = np.asarray(w, dtype=np.float64) / h
    i = np.minimum(np.floor(s).astype(np.int64), n_r - 3)
    L = lagrange4(s - i)
    out = np.zeros(np.shape(s), dtype=Xr.dtype)
    for o in range(4):
        node = np.abs(i - 1 + o)                       # reflection at w = 0
        out = out + L[o] * np.take_along_axis(Xr, node[..., None], axis=-1)[..., 0]
    return out


def residue_sign(z, occ):
    """theta_m(E) with z = E - e_m; occ: bool per m."""
    th = np.where(occ, -(z < 0.0).astype(np.float64), (z > 0.0).astype(np.float64))
    return np.where(z == 0.0, np.where(occ, -0.5, 0.5), th)


def sigma_cd_q(Xi, Xr, eig, kmq, q, n_occ, omega, weight, h, E, n_q):
    """Contribution of one q at real energies.

    Xi: [N_k][N_qp][N_bands][N_w] pair weights at i w_j (real part used);
    Xr: [N_k][N_qp][N_bands][n_r] pair weights at r h; kmq: rows of the k
    points in Xi; E: [n_e][N_k][N_qp].  Returns [n_e][N_k][N_qp], NaN where a
    residue frequency exceeds (n_r-1) h."""
    n_k, nq, nb, nw = Xi.shape
    top = (Xr.shape[-1] - 1) * h
    occ = np.arange(nb) < n_occ
    out = np.zeros(E.shape, dtype=np.float64)
    for k in range(n_k):
        em = eig[kmq[k, q]]
        for n in range(nq):
            X0 = Xr[k, n, :, 0].real                                        # [nb]
            Xd = Xi[k, n].real - X0[:, None]                               # [nb][nw]
            Xrn = Xr[k, n].real
            for e in range(E.shape[0]):
                z = E[e, k, n] - em                                         # [nb]
                ker = z[:, None] / (z[:, None] ** 2 + omega[None, :] ** 2)
                integ = -(1.0 / np.pi) * np.sum(Xd * weight[None, :] * ker) - 0.5 * np.sum(np.sign(z) * X0)
                th = residue_sign(z, occ)
                use = th != 0.0
                if np.any(np.abs(z[use]) > top):
                    out[e, k, n] = np.nan
                    continue
                res = np.sum(th[use] * interp_real(Xrn[use], h, np.abs(z[use])))
                out[e, k, n] = integ + res
    return out / n_q


def qp_linear(s_minus, s_0, s_plus, delta, eps, e_static):
    """Linearised QP energies and renormalisation factors from Sigma^c at
    eps - delta, eps, eps + delta."""
    Z = 1.0 / (1.0 - (s_plus - s_minus) / (2.0 * delta))
    return eps + Z * (s_0 + e_static), Z
