"""The whole imaginary-frequency path for one cell (oracle; test
infrastructure), following the flowchart of Sec. II C with the q loop outer
for both the response and the self-energy (a reordering of the finite sums):

  for q:  B(k,q) = C(k,k+q) (occ x unocc)       Eqs. AO_triple_split2, AO_MO_transform
          chi~(q, i w_j)                         Eq. chi0_matrix
          W^c(q, i w_j)                          Eqs. symm_dielec_func, screened_W_matr
                                                 (q = 0: Eq. dielectric_func_gamma)
          x(k,q) = C(k,k-q) (QP bands x all)
          Sigma^c_n(k, i w_i) += ...             Eq. GW_selfe_element
  Pade continuation and the QP equation.
The exchange self-energy (the bare-Coulomb term of Eq. GW_selfe_element) is
`sigma_x`, from the pairs of QP bands at k and occupied bands at k-q.
`sigma_cd` evaluates Sigma^c at real energies by contour deformation
(`contour`), from W^c on the imaginary grid and on a real grid below the
smallest transition energy.
"""
from __future__ import annotations

import numpy as np

from . import grids, lri, response, screening, selfenergy, continuation, contour


class Oracle:
    def __init__(self, sysm, n_par=16, per_atom=False, lri_blocks=None):
        self.sys = sysm
        sp = sysm.spec
        self.kint, self.kfrac = grids.kgrid(sp.nk)
        self.kpq, self.kmq, self.minus = grids.kq_tables(sp.nk)
        self.omega, self.weight = grids.frequency_grid(sp.n_freq, sp.x0)
        # per_atom: triples one auxiliary atom at a time (cells too large for
        # the dense AO tensor); the dense form otherwise.  lri_blocks: the
        # coefficients atom by atom when the cell does not hold them
        self.tb = lri.TripleBuilder(sysm, self.kfrac, per_atom=per_atom, blocks=lri_blocks)
        self.occ = slice(0, sp.n_occ)
        self.unocc = slice(sp.n_occ, sp.n_bands)
        self.qp = slice(sp.qp_lo, sp.qp_lo + sp.n_qp)
        self.allb = slice(0, sp.n_bands)
        self.n_par = min(n_par, sp.n_freq)
        # q -> 0 averaged over directions: (p . q_hat_d [n_dir][N_k][N_occ][N_unocc], w_d), or None
        self.gamma_dirs = None

    # ---- per-q pieces -------------------------------------------------
    def B(self, q, ks=None):
        """C^mu_{ia}(k,k+q): [len(ks)][N_aux][N_occ][N_unocc] (default every k)."""
        ks = range(self.sys.n_k) if ks is None else ks
        return np.stack([self.tb.mo(k, self.kpq[k, q], self.occ, self.unocc) for k in ks])

    def x(self, q, ks=None):
        """C^mu_{nm}(k,k-q) for QP bands n and all m: [len(ks)][N_aux][N_qp][N_bands]."""
        ks = range(self.sys.n_k) if ks is None else ks
        return np.stack([self.tb.mo(k, self.kmq[k, q], self.qp, self.allb) for k in ks])

    def x_occ(self, q, ks=None):
        """C^mu_{nm}(k,k-q) for QP bands n and occupied m: [len(ks)][N_aux][N_qp][N_occ]."""
        ks = range(self.sys.n_k) if ks is None else ks
        return np.stack([self.tb.mo(k, self.kmq[k, q], self.qp, self.occ) for k in ks])

    def sigma_x_q(self, q, ks=None):
        """Contribution of q to Sigma^x for the k points `ks` (default all)."""
        return selfenergy.sigma_x_q(self.x_occ(q, ks), self.sys.V[q], self.sys.n_k)

    def sigma_x(self, ks=None):
        """Sigma^x_n(k) [len(ks)][N_qp], summed over every q."""
        return sum(self.sigma_x_q(q, ks) for q in range(self.sys.n_k))

    def chi0(self, q, B=None, omega=None, ks=None):
        """chi~(q) at `omega` (default the grid).  ks: the k terms of the sum to
        take (B then holds those rows); the k sum over a partition of the grid
        adds up to the whole."""
        B = self.B(q, ks) if B is None else B
        om = self.omega if omega is None else omega
        return response.chi0_trs(B, self.sys.eig, self.kpq, q, self.sys.n_occ, om, ks=ks, n_k=self.sys.n_k)

    def wc(self, q, chi=None, B=None, gamma=True):
        s = self.sys
        if q == 0 and gamma:
            B = self.B(0) if B is None else B
            if self.gamma_dirs is not None:
                return screening.screen_gamma_average(B, s.eig, s.n_occ, *self.gamma_dirs, s.omega_cell, s.V[0],
                                                      self.omega)
            return screening.screen_gamma(B, s.eig, s.n_occ, s.p, s.omega_cell, s.V[0], self.omega)[2]
        chi = self.chi0(q, B) if chi is None else chi
        return screening.screen(chi, s.V[q], self._vcut(q))[1]

    def _vcut(self, q):
        """V^cut(q) of the cell for q != 0 (None: V^cut = V).  At q = 0 the
        cell's V[0] already is V^cut(0), in both places (Sec. III B)."""
        vc = getattr(self.sys, "Vcut", None)
        return None if (vc is None or q == 0) else vc[q]

    def sigma_q(self, q, Wc, ks=None):
        """Contribution of q to Sigma^c for the k points `ks` (default all)."""
        ks = list(range(self.sys.n_k)) if ks is None else list(ks)
        xq = self.x(q, ks)
        X = selfenergy.pair_weights(xq, Wc)
        kmq = self.kmq[ks]
        return selfenergy.sigma_c_q(X, self.sys.eig, kmq, q, self.sys.mu, self.omega, self.weight,
                                    self.sys.n_k), X

    # ---- real energies by contour deformation ---------------------------
    def chi0_real(self, q, omega_r, B=None, eta=0.0):
        """chi~(q, w) at real w below the smallest transition energy, or at
        w + i eta at any w (eta > 0)."""
        B = self.B(q) if B is None else B
        return response.chi0_trs(B, self.sys.eig, self.kpq, q, self.sys.n_occ, omega_r, real_axis=True, eta=eta)

    def wc_real(self, q, omega_r, chi=None, B=None, gamma=True, eta=0.0):
        s = self.sys
        if q == 0 and gamma:
            B = self.B(0) if B is None else B
            if self.gamma_dirs is not None:
                return screening.screen_gamma_average(B, s.eig, s.n_occ, *self.gamma_dirs, s.omega_cell, s.V[0],
                                                      omega_r, real_axis=True, eta=eta)
            return screening.screen_gamma(B, s.eig, s.n_occ, s.p, s.omega_cell, s.V[0], omega_r, real_axis=True,
                                          eta=eta)[2]
        chi = self.chi0_real(q, omega_r, B, eta=eta) if chi is None else chi
        return screening.screen(chi, s.V[q], self._vcut(q))[1]

    def sigma_cd_q(self, q, Wc, Wr, h, E, ks=None):
        """Contribution of q to Sigma^c at the real energies E [n_e][len(ks)][N_qp]."""
        ks = list(range(self.sys.n_k)) if ks is None else list(ks)
        xq = self.x(q, ks)
        Xi = selfenergy.pair_weights(xq, Wc)
        Xr = selfenergy.pair_weights(xq, Wr)
        return contour.sigma_cd_q(Xi, Xr, self.sys.eig, self.kmq[ks], q, self.sys.n_occ, self.omega, self.weight,
                                  h, E, self.sys.n_k)

    def sigma_cd(self, n_r, omega_max, E, ks=None, gamma=True, eta=0.0):
        """Sigma^c_n(k, E) summed over q at the real energies E (the real part,
        with the residues of the broadened W^c at w + i eta when eta > 0)."""
        omega_r, h = contour.real_grid(n_r, omega_max)
        out = np.zeros(E.shape)
        for q in range(self.sys.n_k):
            B = self.B(q)
            Wc = self.wc(q, B=B, gamma=gamma)
            Wr = self.wc_real(q, omega_r, B=B, gamma=gamma, eta=eta)
            out += self.sigma_cd_q(q, Wc, Wr, h, E, ks)
        return out

    def qp_cd(self, n_r, omega_max, eta, n_iter, delta=0.002, ks=None, gamma=True):
        """Quasiparticle energies from contour deformation: Newton steps on
        f(E) = E - e_n - e_static_n - Re Sigma^c(E) from E_0 = e_n, the slope
        from Sigma^c at E -+ delta (the first step is the linearised QP
        energy).  Returns (E [N_k][N_qp], Z, Sigma^c at the last E)."""
        s = self.sys
        ks = list(range(s.n_k)) if ks is None else list(ks)
        eps = s.eig[ks][:, self.qp]
        est = s.e_static[ks]
        E = eps.copy()
        for _ in range(n_iter):
            S3 = self.sigma_cd(n_r, omega_max, np.stack([E - delta, E, E + delta]), ks, gamma, eta)
            Z = 1.0 / (1.0 - (S3[2] - S3[0]) / (2.0 * delta))
            E = E + Z * (eps + est + S3[1] - E)
        return E, Z, S3[1]

    # ---- whole path ---------------------------------------------------
    def run(self, ks=None, gamma=True, keep=False):
        s = self.sys
        ks = list(range(s.n_k)) if ks is None else list(ks)
        sigma = np.zeros((len(ks), s.spec.n_qp, len(self.omega)), dtype=np.complex128)
        kept = {}
        for q in range(s.n_k):
            B = self.B(q)
            chi = self.chi0(q, B)
            Wc = self.wc(q, chi=chi, B=B, gamma=gamma)
            sq, X = self.sigma_q(q, Wc, ks)
            sigma += sq
            if keep:
                kept[q] = dict(chi=chi, Wc=Wc, X=X, sigma=sq)
        eps_qp = s.eig[ks][:, self.qp]
        nodes = grids.pade_nodes(len(self.omega), self.n_par)
        E, Z, ok = continuation.qp_energies(sigma, self.omega, eps_qp, s.e_static[ks], s.mu, nodes)
        return dict(sigma=sigma, E=E, Z=Z, converged=ok, per_q=kept, ks=ks)
