"""Localized RI triple coefficients (oracle; test infrastructure).

Sec. II C of the paper:
* Eqs. expan_coeff_FT1/2: C~_{i(0),j(k)} = sum_R exp(i k.R) C~_{i(0),j(R)}.
* Eq. AO_triple_split2: the AO triple coefficient of the Bloch product
  phi_i^{k1*} phi_j^{k2} (k1 = k+q, k2 = k in the paper) is
      C~^mu_{ij}(k1,k2) = [mu on atom(i)] C~^mu_{i(0),j(k2)}
                        + [mu on atom(j)] C~^mu_{j(0),i(-k1)}.
  (The earlier Eq. AO_triple_split has the atom labels of the two sectors
  interchanged; the split2 form is the one that follows from Eq. local_ri_FT.)
* Eq. AO_MO_transform: C^mu_{mn}(k1,k2) = sum_ij c*_{im}(k1) c_{jn}(k2) C~^mu_{ij}(k1,k2).

Here the stored real-space block of atom A, L_A(R)[mu][a][b], is the
coefficient C~^{mu(0)}_{a(0), b(R)} with mu and a on atom A.

`mo_triple` forms the dense AO triple tensor explicitly (N_aux x N_b x N_b
per Bloch pair), exactly as the equation reads.  `mo_triple_per_atom` takes
the same two equations one auxiliary atom at a time without forming the dense
tensor (for cells where it would not fit in memory): an auxiliary function on
atom A couples only to the orbital functions of A in either sector, so
    C^mu_{mn} = sum_{a in A} c*_{am}(k1) [sum_j C~^mu_{a(0),j(k2)} c_{jn}(k2)]
              + sum_{b in A} [sum_i c*_{im}(k1) C~^mu_{b(0),i(-k1)}] c_{bn}(k2).
"""
from __future__ import annotations

import numpy as np


def lri_bloch(lri_blocks, R, kfrac):
    """Eqs. expan_coeff_FT1/2 for every atom block.

    lri_blocks: list over atoms of [nR][naux_A][nb_A][N_b] float64.
    R: [nR][3] integer lattice coordinates.  kfrac: [nk][3] fractional k.
    Returns list over atoms of [nk][naux_A][nb_A][N_b] complex128.
    """
    phase = np.exp(2j * np.pi * (np.asarray(kfrac, dtype=np.float64) @ np.asarray(R, dtype=np.float64).T))
    out = []
    for blk in lri_blocks:
        nR = blk.shape[0]
        flat = blk.reshape(nR, -1)
        out.append((phase @ flat).reshape((phase.shape[0],) + blk.shape[1:]))
    return out


def ao_triple(Lk2, Lmk1, basis_off, aux_off, n_b):
    """Dense C~^mu_{ij}(k1,k2), Eq. AO_triple_split2.

    Lk2[A]  = C~_{a(0),b(k2)}  for atom A, shape [naux_A][nb_A][N_b]
    Lmk1[A] = C~_{a(0),b(-k1)} for atom A.
    Returns [N_aux][N_b][N_b] complex128.
    """
    n_atoms = len(Lk2)
    n_aux = int(aux_off[-1])
    Ct = np.zeros((n_aux, n_b, n_b), dtype=np.complex128)
    for A in range(n_atoms):
        mu = slice(int(aux_off[A]), int(aux_off[A + 1]))
        a = slice(int(basis_off[A]), int(basis_off[A + 1]))
        # mu on atom(i): i runs over atom A's functions, j over all
        Ct[mu, a, :] += Lk2[A]
        # mu on atom(j): j runs over atom A's functions, i over all
        Ct[mu, :, a] += np.transpose(Lmk1[A], (0, 2, 1))
    return Ct


def mo_triple(Ct, c1, c2):
    """Eq. AO_MO_transform: C^mu_{mn} = sum_ij c1*_{im} Ct^mu_{ij} c2_{jn}.
    c1: [N_b][M] orbitals at the first Bloch vector, c2: [N_b][N]."""
    return np.einsum("im,uij,jn->umn", c1.conj(), Ct, c2, optimize=True)


def mo_triple_per_atom(Lk2, Lmk1, basis_off, aux_off, c1, c2):
    """Eq. AO_triple_split2 followed by Eq. AO_MO_transform, one auxiliary atom
    at a time (no dense AO tensor).  Arguments as `ao_triple` and `mo_triple`;
    returns [N_aux][M][N] complex128."""
    n_aux = int(aux_off[-1])
    out = np.empty((n_aux, c1.shape[1], c2.shape[1]), dtype=np.complex128)
    for A in range(len(Lk2)):
        mu = slice(int(aux_off[A]), int(aux_off[A + 1]))
        a = slice(int(basis_off[A]), int(basis_off[A + 1]))
        # sector mu on atom(i): i = a on A, j over every function
        t1 = np.einsum("am,uaj,jn->umn", c1[a].conj(), Lk2[A], c2, optimize=True)
        # sector mu on atom(j): j = b on A, i over every function (C~_{b(0),i(-k1)})
        t2 = np.einsum("im,ubi,bn->umn", c1.conj(), Lmk1[A], c2[a], optimize=True)
        out[mu] = t1 + t2
    return out


class TripleBuilder:
    """Forms C^mu_{mn}(k1,k2) for any pair of grid points of one cell."""

    def __init__(self, sysm, kfrac, per_atom=False, blocks=None):
        """blocks: the atoms' real-space blocks in order (any iterable, taken
        one at a time); default the cell's own array."""
        self.sys = sysm
        self.per_atom = per_atom
        if blocks is None:
            blocks = (sysm.lri_block(A) for A in range(sysm.spec.n_atoms))
        self.Lk, self.Lmk = [], []
        for blk in blocks:
            self.Lk += lri_bloch([blk], sysm.R, kfrac)      # at +k
            self.Lmk += lri_bloch([blk], sysm.R, -kfrac)    # at -k (own transform)
        if len(self.Lk) != sysm.spec.n_atoms:
            raise ValueError("one block per atom expected")

    def ao(self, k1, k2):
        s = self.sys
        return ao_triple([L[k2] for L in self.Lk], [L[k1] for L in self.Lmk],
                         s.basis_off, s.aux_off, s.spec.n_b)

    def mo(self, k1, k2, rows, cols):
        """C^mu_{mn}(k1,k2) for bands m in `rows`, n in `cols` (slices/arrays)."""
        c = self.sys.evec
        if self.per_atom:
            s = self.sys
            return mo_triple_per_atom([L[k2] for L in self.Lk], [L[k1] for L in self.Lmk], s.basis_off, s.aux_off,
                                      c[k1][:, rows], c[k2][:, cols])
        return mo_triple(self.ao(k1, k2), c[k1][:, rows], c[k2][:, cols])


def fit_two_centre(T, V, n_keep):
    """Eq. two_center_coeff_determination: the two-centre coefficients of the
    orbital products of one atom pair (I in the home cell, J in cell R), from
    minimising the Coulomb self-repulsion of the expansion error:

        C~^{mu(0)}_{i(0),j(R)} = sum_{nu in {I, J(R)}} (i(0),j(R)|nu) (V^{IJ})^{-1}_{nu mu},   mu on I.

    T: [n][nrhs], (ij|nu) for the auxiliary functions nu of I (the first
    n_keep) and of J(R), one column per product (i, j); V: [n][n], the
    Coulomb matrix of those functions (symmetric positive definite; for I = J
    and R = 0 the set is I's functions alone).  Returns [n_keep][nrhs].
    """
    X = np.linalg.solve(V, T)          # (V^-1)_{nu mu} = (V^-1)_{mu nu}: the rows of V^-1 T
    return X[:n_keep]
