"""Independent-particle response on the auxiliary basis (oracle; test
infrastructure).

Eq. chi0_matrix of the paper, read with the occupation difference of the
real-space Adler-Wiser formula (Eq. chi_0_realspace, f^q_n read as f^k_n)
restored, and paired with the Coulomb matrix the way the Dyson equation in
matrix-element form requires: the dielectric matrix at q uses the response
at -q.  Writing D^mu_{mn}(k) = C^mu_{mn}(k, k+q) (the triple coefficient of
psi_m^{k*} psi_n^{k+q}), that response is

  chi~_{mu nu}(q, i w) = s/N_k sum_k sum_{mn} (f_m^k - f_n^{k+q})
                         D^mu_{mn} conj(D^nu_{mn}) / (e_m^k - e_n^{k+q} - i w).

With time-reversal symmetric inputs the two orderings of an
occupied/unoccupied pair combine into

  chi~_{mu nu}(q, i w) = -s/N_k sum_k sum_{i occ, a unocc}
                         2 D_ia/(D_ia^2 + w^2) B^mu_ia conj(B^nu_ia),
  B^mu_ia = C^mu_{ia}(k, k+q),  D_ia = e_a^{k+q} - e_i^k  (`chi0_trs`),

which is Hermitian and negative semidefinite for every real w.
`chi0_literal` evaluates Eq. chi0_matrix term by term (all band pairs, both
triple coefficients formed directly); at the paper's q = -q it must equal
`chi0_trs` at q.
s = 2 (closed shell, spin sum of the paper's formula).
"""
from __future__ import annotations

import numpy as np

SPIN = 2.0


def weight(delta, w, real_axis=False, eta=0.0):
    """The transition weight 2D/(D^2 - z^2) at z = i w (imaginary axis:
    2D/(D^2 + w^2)), at real z = w (real_axis), or at z = w + i eta
    (real_axis, eta > 0: complex)."""
    if not real_axis:
        return 2.0 * delta / (delta * delta + w * w)
    if eta == 0.0:
        return 2.0 * delta / (delta * delta - w * w)
    z = w + 1j * eta
    return 2.0 * delta / (delta * delta - z * z)


def chi0_trs(B, eig, kpq, q, n_occ, omega, s=SPIN, real_axis=False, eta=0.0, ks=None, n_k=None):
    """B: [N_k][N_aux][N_occ][N_unocc] = C^mu_{ia}(k,k+q); returns [N_w][N_aux][N_aux].
    ks / n_k: B's rows are the k points ks of a grid of n_k points (the terms
    of those k only; default every k of B).

    real_axis: the frequencies are real, w -> -i w in the denominators, so the
    weight is 2D/(D^2 - w^2); with eta = 0 meant for 0 <= w < min D, where it
    stays finite and positive (the response below the first transition).
    eta > 0: the response at the complex frequencies w + i eta, at any w: the
    complex weight makes it a sum of two Hermitian parts, Re and i Im of the
    weight, not Hermitian itself (the broadened response above the first
    transition)."""
    ks = list(range(B.shape[0])) if ks is None else list(ks)
    n_k = B.shape[0] if n_k is None else n_k
    if len(ks) != B.shape[0]:
        raise ValueError("one row of B per k in ks")
    n_aux = B.shape[1]
    cplx = real_axis and eta != 0.0
    out = np.zeros((len(omega), n_aux, n_aux), dtype=np.complex128)
    for row, k in enumerate(ks):
        kq = kpq[k, q]
        delta = eig[kq][n_occ:][None, :] - eig[k][:n_occ][:, None]     # [occ][unocc]
        Bk = B[row].reshape(n_aux, -1)
        for iw, w in enumerate(omega):
            wt = weight(delta, w, real_axis, eta).reshape(-1)
            out[iw] += (Bk * wt[None, :]) @ Bk.conj().T
    return -(s / n_k) * out


def chi0_literal(builder, eig, kpq, qp, n_occ, omega, s=SPIN):
    """Eq. chi0_matrix term by term at the paper's q = qp, with the occupation
    difference restored: s/N_k sum_k sum_{mn} (f_m^{k+qp} - f_n^k)
    C^mu_{mn}(k+qp,k) C^nu_{nm}(k,k+qp) / (e_m^{k+qp} - e_n^k - i w).
    Both triple coefficients are formed directly by `builder.mo`.
    Evaluated at qp = -q it equals chi~(q) of `chi0_trs`."""
    n_k = eig.shape[0]
    nb = eig.shape[1]
    f = np.zeros(nb)
    f[:n_occ] = 1.0
    allb = slice(0, nb)
    out = None
    for k in range(n_k):
        k1 = kpq[k, qp]
        C1 = builder.mo(k1, k, allb, allb)            # [mu][m][n]
        C2 = builder.mo(k, k1, allb, allb)            # [nu][n][m]
        n_aux = C1.shape[0]
        if out is None:
            out = np.zeros((len(omega), n_aux, n_aux), dtype=np.complex128)
        df = f[:, None] - f[None, :]                  # f_m^{k+qp} - f_n^k (T = 0, same occupations)
        de = eig[k1][:, None] - eig[k][None, :]
        A = C1.reshape(n_aux, -1)
        Bt = np.transpose(C2, (0, 2, 1)).reshape(n_aux, -1)   # [nu][m][n]
        for iw, w in enumerate(omega):
            wt = (df / (de - 1j * w)).reshape(-1)
            out[iw] += (A * wt[None, :]) @ Bt.T
    return (s / n_k) * out
