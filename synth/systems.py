"""Seeded synthetic G0W0 inputs.

Conventions shared by every consumer of these arrays (they are interface
conventions, not arithmetic of the method):

* k-point index.  A Gamma-centred n1 x n2 x n3 grid; the point with integer
  coordinates (i1, i2, i3), 0 <= i_d < n_d, has fractional coordinates
  i_d / n_d and index (i1 * n2 + i2) * n3 + i3.  The q-grid is the k-grid.
* Real-space LRI coefficients: amplitude a_L * N(0,1) * exp(-|R|/2 bohr) with
  a_L = 0.03 * sqrt(48 / (N_occ * N_unocc)).  The static screening per
  auxiliary function grows with the number of occupied/unoccupied pairs times
  a_L^2; this normalisation keeps every cell in the semiconductor range (eps~
  eigenvalues ~1..10 away from q = 0, |Sigma^c| ~ 0.1-0.5 Ha, Z ~ 0.8-0.9),
  where unit amplitude gives eps~ ~ 4e4 and |Sigma^c| ~ 400 Ha.  For each atom A and lattice vector R (integer
  coordinates in the primitive vectors) a block L_A(R)[mu][a][b] holds the
  two-centre coefficient of the product phi_a(0) phi_b(R) on the auxiliary
  function mu, where mu runs over the auxiliary functions of atom A, a over
  the orbital basis functions of atom A and b over all N_b orbital basis
  functions of the cell (the LRI restriction of Sec. II C: the fitting
  functions sit on the atom of the first orbital).  The flat array is the
  concatenation over atoms of [nR][naux_A][nb_A][N_b] float64 blocks.
* Eigenvectors c[k][i'][n] (complex128), eigenvalues eig[k][n] (float64,
  ascending, Hartree), all N_b bands kept.
* Coulomb matrices V[q][mu][nu] (complex128, Hermitian positive definite).
  V[0] holds the truncated Coulomb matrix at q = 0 (Sec. III B).
* Momentum matrix elements along q_hat = x: p[k][i][a] = p_{ia}(k).x for
  occupied i and unoccupied a (complex128).

Recipe (per cell, seed s): numpy.random.default_rng(s).spawn(6) gives the
sub-streams for eigenvalues, eigenvectors, LRI coefficients, Coulomb matrices
and momentum elements.  Inputs are time-reversal symmetric: quantities at -k
are complex conjugates of those at k (p is odd: p(-k) = -conj(p(k))), and
they are real (p imaginary) at time-reversal-invariant points.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

A_SI = 10.263  # bohr, Si lattice constant used for the 2-atom fcc cells


@dataclasses.dataclass(frozen=True)
class CellSpec:
    n_atoms: int
    nb_per_atom: int
    naux_per_atom: int
    nk: tuple
    n_occ: int
    n_freq: int
    qp_lo: int
    n_qp: int
    x0: float = 0.5
    rmax: int = 2
    lattice: str = "fcc"
    lri_amp: Optional[float] = None   # None: 0.03 * sqrt(48 / (N_occ * N_unocc))

    @property
    def n_b(self) -> int:
        return self.n_atoms * self.nb_per_atom

    @property
    def n_aux(self) -> int:
        return self.n_atoms * self.naux_per_atom

    @property
    def n_k(self) -> int:
        return int(np.prod(self.nk))

    @property
    def n_bands(self) -> int:
        return self.n_b

    @property
    def lri_amplitude(self) -> float:
        if self.lri_amp is not None:
            return self.lri_amp
        return 0.03 * math.sqrt(48.0 / (self.n_occ * (self.n_bands - self.n_occ)))


def _cell(n_atoms, nb, naux, nk, n_occ, n_freq, n_qp=8, qp_lo=None):
    lattice = "fcc" if n_atoms == 2 else "sc"
    if qp_lo is None:
        qp_lo = max(0, n_occ - n_qp // 2)
    return CellSpec(n_atoms=n_atoms, nb_per_atom=nb, naux_per_atom=naux, nk=tuple(nk),
                    n_occ=n_occ, n_freq=n_freq, qp_lo=qp_lo, n_qp=n_qp, lattice=lattice)


# The five workloads: (1) small FP64 case, (2) Si-like 2-atom cell,
# (3) six uneven cells, (4) 8-atom cell, (5) 16-atom cell.
CONFIGS = {
    1: [_cell(2, 8, 30, (2, 2, 2), 4, 16, n_qp=16, qp_lo=0)],
    2: [_cell(2, 39, 130, (6, 6, 6), 4, 32)],
    3: [_cell(na, 39, 130, (4, 4, 4) if na <= 4 else (3, 3, 3), 2 * na, 32)
        for na in (2, 2, 4, 4, 6, 8)],
    4: [_cell(8, 39, 130, (4, 4, 4), 16, 40)],
    5: [_cell(16, 39, 130, (3, 3, 3), 32, 48)],
}


@dataclasses.dataclass
class System:
    spec: CellSpec
    basis_off: np.ndarray      # int32 [n_atoms+1]
    aux_off: np.ndarray        # int32 [n_atoms+1]
    lattice: np.ndarray        # float64 [3][3], rows = primitive vectors (bohr)
    R: np.ndarray              # int32 [nR][3]
    lri: Optional[np.ndarray]  # float64 flat, per atom [nR][naux_A][nb_A][N_b]; None: not materialised
    lri_off: np.ndarray        # int64 [n_atoms+1] element offsets into lri
    eig: np.ndarray            # float64 [N_k][N_bands]
    evec: np.ndarray           # complex128 [N_k][N_b][N_bands]
    V: np.ndarray              # complex128 [N_q][N_aux][N_aux]; V[0] = V^cut(0)
    p: np.ndarray              # complex128 [N_k][N_occ][N_unocc]
    omega_cell: float          # cell volume (bohr^3)
    mu: float                  # chemical potential, mid-gap (Ha)
    e_static: np.ndarray       # float64 [N_k][N_qp], Sigma^x - V^xc (zero here)
    seed: int
    Vcut: Optional[np.ndarray] = None   # complex128 [N_q][N_aux][N_aux] truncated V(q), or None (V^cut = V)

    # convenience views
    @property
    def n_k(self):
        return self.spec.n_k

    @property
    def n_aux(self):
        return self.spec.n_aux

    @property
    def n_b(self):
        return self.spec.n_b

    @property
    def n_bands(self):
        return self.spec.n_bands

    @property
    def n_occ(self):
        return self.spec.n_occ

    def lri_block(self, atom: int) -> np.ndarray:
        """The [nR][naux_A][nb_A][N_b] view of atom `atom`'s coefficients."""
        s = self.spec
        if self.lri is None:
            raise ValueError("the coefficients of this cell are not materialised (use lri_blocks)")
        nR = self.R.shape[0]
        na = int(self.aux_off[atom + 1] - self.aux_off[atom])
        nb = int(self.basis_off[atom + 1] - self.basis_off[atom])
        blk = self.lri[self.lri_off[atom]:self.lri_off[atom + 1]]
        return blk.reshape(nR, na, nb, s.n_b)


def _lattice(spec: CellSpec) -> np.ndarray:
    if spec.lattice == "fcc":
        a = A_SI
        return 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    a = A_SI * (spec.n_atoms / 8.0) ** (1.0 / 3.0)
    return a * np.eye(3)


def _kint(nk):
    n1, n2, n3 = nk
    return np.array([(i1, i2, i3) for i1 in range(n1) for i2 in range(n2) for i3 in range(n3)],
                    dtype=np.int64)


def _kidx(iv, nk):
    n1, n2, n3 = nk
    return ((iv[..., 0] % n1) * n2 + (iv[..., 1] % n2)) * n3 + (iv[..., 2] % n3)


def _inscribed_radius(vectors: np.ndarray) -> float:
    vol = abs(np.linalg.det(vectors))
    r = math.inf
    for d in range(3):
        e, f = vectors[(d + 1) % 3], vectors[(d + 2) % 3]
        r = min(r, vol / np.linalg.norm(np.cross(e, f)) / 2.0)
    return r


def make_system(spec: CellSpec, seed: int, *, lri_scale: float = 1.0,
                p_scale: float = 1.0, materialize_lri: bool = True) -> System:
    """Draw one synthetic cell.  `lri_scale`/`p_scale` multiply the LRI and
    momentum arrays (0 gives the zero-coupling limits used in tests).
    materialize_lri=False leaves `lri` None (the other arrays are unchanged:
    the coefficients draw from a stream of their own); `lri_blocks` then
    yields them atom by atom."""
    rng_eig, rng_vec, rng_lri, rng_v, rng_p, _ = np.random.default_rng(seed).spawn(6)
    nk = spec.nk
    n_k, n_b, n_aux, n_occ = spec.n_k, spec.n_b, spec.n_aux, spec.n_occ
    n_bands = spec.n_bands
    n_unocc = n_bands - n_occ
    kint = _kint(nk)
    minus = _kidx(-kint, nk)
    lat = _lattice(spec)

    basis_off = np.arange(spec.n_atoms + 1, dtype=np.int32) * spec.nb_per_atom
    aux_off = np.arange(spec.n_atoms + 1, dtype=np.int32) * spec.naux_per_atom

    eig = np.empty((n_k, n_bands))
    evec = np.empty((n_k, n_b, n_bands), dtype=np.complex128)
    p = np.empty((n_k, n_occ, n_unocc), dtype=np.complex128)
    for k in range(n_k):
        mk = minus[k]
        if mk < k:  # partner already drawn
            eig[k] = eig[mk]
            evec[k] = np.conj(evec[mk])
            p[k] = -np.conj(p[mk])
            continue
        occ = np.sort(rng_eig.uniform(-0.8, -0.05, n_occ))
        unocc = np.sort(rng_eig.uniform(0.05, 2.0, n_unocc))
        eig[k] = np.concatenate([occ, unocc])
        if mk == k:  # time-reversal invariant point: real orbitals
            g = rng_vec.standard_normal((n_b, n_b))
            evec[k] = np.linalg.qr(g)[0]
            p[k] = 1j * rng_p.normal(0.0, 0.5, (n_occ, n_unocc))
        else:
            g = (rng_vec.standard_normal((n_b, n_b)) + 1j * rng_vec.standard_normal((n_b, n_b))) / math.sqrt(2.0)
            evec[k] = np.linalg.qr(g)[0]
            p[k] = (rng_p.normal(0.0, math.sqrt(0.125), (n_occ, n_unocc))
                    + 1j * rng_p.normal(0.0, math.sqrt(0.125), (n_occ, n_unocc)))
    p *= p_scale

    # real-space two-centre coefficients, |n_i| <= rmax, filled in place atom
    # by atom (the 16-atom cell's array is 50 GB)
    R = lattice_vectors(spec)
    lri_off = [0]
    for A in range(spec.n_atoms):
        lri_off.append(lri_off[-1] + R.shape[0] * spec.naux_per_atom * spec.nb_per_atom * n_b)
    lri = None
    if materialize_lri:
        lri = np.empty(lri_off[-1])
        for _ in _lri_blocks(spec, rng_lri, lat, lri_scale, lri):
            pass

    # Coulomb matrices
    recip = 2.0 * math.pi * np.linalg.inv(lat).T  # rows = reciprocal vectors
    supercell = lat * np.array(nk, dtype=np.float64)[:, None]
    r_cut = _inscribed_radius(supercell)
    h0 = 2.0 * math.pi * r_cut * r_cut
    V = np.empty((n_k, n_aux, n_aux), dtype=np.complex128)
    for q in range(n_k):
        mq = minus[q]
        if mq < q:
            V[q] = np.conj(V[mq])
            continue
        if mq == q:
            A = rng_v.standard_normal((n_aux, n_aux)) / math.sqrt(n_aux)
        else:
            A = (rng_v.standard_normal((n_aux, n_aux)) + 1j * rng_v.standard_normal((n_aux, n_aux))) \
                / math.sqrt(2.0 * n_aux)
        Vq = A @ A.conj().T + 0.1 * np.eye(n_aux)
        if q == 0:
            Vq[0, 0] += h0
        else:
            f = kint[q] / np.array(nk, dtype=np.float64)
            f = np.where(f > 0.5, f - 1.0, f)
            qc = f @ recip
            Vq[0, 0] += 4.0 * math.pi / float(qc @ qc)
        V[q] = Vq
    omega_cell = abs(float(np.linalg.det(lat)))
    mu = 0.5 * (eig[:, n_occ - 1].max() + eig[:, n_occ].min())
    e_static = np.zeros((n_k, spec.n_qp))
    return System(spec=spec, basis_off=basis_off, aux_off=aux_off, lattice=lat, R=R, lri=lri,
                  lri_off=np.array(lri_off, dtype=np.int64), eig=eig, evec=evec, V=V, p=p,
                  omega_cell=omega_cell, mu=float(mu), e_static=e_static, seed=seed)


def truncated_coulomb(sysm: System) -> np.ndarray:
    """V^cut(q) for every q, complex [N_q][N_aux][N_aux]: V(q) with the
    divergent 4 pi/|q|^2 on auxiliary function 0 replaced by the Fourier
    transform of the Coulomb operator cut off at R_cut (the inscribed radius
    of the Born-von Karman supercell), 4 pi (1 - cos(|q| R_cut))/|q|^2, whose
    q -> 0 limit 2 pi R_cut^2 is the value V[0] already carries.  Positive
    definite (the added term is >= 0); V^cut(-q) = conj V^cut(q)."""
    sp = sysm.spec
    nk = sp.nk
    kint = _kint(nk)
    recip = 2.0 * math.pi * np.linalg.inv(sysm.lattice).T
    r_cut = _inscribed_radius(sysm.lattice * np.array(nk, dtype=np.float64)[:, None])
    minus = _kidx(-kint, nk)
    Vc = sysm.V.copy()
    for q in range(1, sysm.n_k):
        if minus[q] < q:   # the partner's |q| is the one V(q) = conj V(-q) carries
            Vc[q] = np.conj(Vc[minus[q]])
            continue
        f = kint[q] / np.array(nk, dtype=np.float64)
        f = np.where(f > 0.5, f - 1.0, f)
        qc = f @ recip
        q2 = float(qc @ qc)
        Vc[q, 0, 0] -= 4.0 * math.pi * math.cos(math.sqrt(q2) * r_cut) / q2
    return Vc


def lattice_vectors(spec: CellSpec) -> np.ndarray:
    """The R of the two-centre coefficients, integer [nR][3], |n_i| <= rmax."""
    rr = range(-spec.rmax, spec.rmax + 1)
    return np.array([(a, b, c) for a in rr for b in rr for c in rr], dtype=np.int32)


def _lri_blocks(spec: CellSpec, rng, lat, lri_scale=1.0, out=None):
    """Yield atom A's block [nR][naux_A][nb_A][N_b] of the real-space
    coefficients in generator order (into `out`, the flat array, if given)."""
    R = lattice_vectors(spec)
    nR = R.shape[0]
    amp = np.exp(-np.linalg.norm(R @ lat, axis=1) / 2.0) * (spec.lri_amplitude * lri_scale)
    shape = (nR, spec.naux_per_atom, spec.nb_per_atom, spec.n_b)
    size = int(np.prod(shape))
    for A in range(spec.n_atoms):
        blk = out[A * size:(A + 1) * size].reshape(shape) if out is not None else np.empty(shape)
        rng.standard_normal(out=blk)
        blk *= amp[:, None, None, None]
        yield blk


def lri_blocks(spec: CellSpec, seed: int, lri_scale: float = 1.0):
    """Atom by atom, the real-space coefficient blocks make_system(spec, seed)
    draws, without holding the others (the same generator stream)."""
    rng_lri = np.random.default_rng(seed).spawn(6)[2]
    yield from _lri_blocks(spec, rng_lri, _lattice(spec), lri_scale)


def momentum_vectors(sysm: System) -> np.ndarray:
    """Cartesian momentum matrix elements p_ia(k), complex [3][N_k][N_occ][N_unocc],
    for averaging the q -> 0 treatment over directions.  Drawn like
    `System.p` (time reversal: p(-k) = -conj(p(k)), purely imaginary at the
    invariant points), from a generator of their own seeded by the cell's seed."""
    rng = np.random.default_rng([sysm.seed, 3])
    sp = sysm.spec
    n_k, n_occ, n_un = sysm.n_k, sp.n_occ, sp.n_bands - sp.n_occ
    minus = _kidx(-_kint(sp.nk), sp.nk)
    p3 = np.empty((3, n_k, n_occ, n_un), dtype=np.complex128)
    for k in range(n_k):
        mk = minus[k]
        if mk < k:
            p3[:, k] = -np.conj(p3[:, mk])
        elif mk == k:
            p3[:, k] = 1j * rng.normal(0.0, 0.5, (3, n_occ, n_un))
        else:
            p3[:, k] = (rng.normal(0.0, math.sqrt(0.125), (3, n_occ, n_un))
                        + 1j * rng.normal(0.0, math.sqrt(0.125), (3, n_occ, n_un)))
    return p3


def cartesian_directions():
    """The six half-axes +-x, +-y, +-z, equal weights."""
    q = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.float64)
    return q, np.full(6, 1.0 / 6.0)


def project_momentum(p3, qhat) -> np.ndarray:
    """p_ia(k) . q_hat for each direction: complex [n_dir][N_k][N_occ][N_unocc]."""
    return np.einsum("c...,dc->d...", p3, np.asarray(qhat, dtype=np.float64))


def eigenvalues_of(spec: CellSpec, seed: int) -> np.ndarray:
    """The eigenvalues make_system(spec, seed) draws, [N_k][N_bands], from the
    same generator stream (without drawing the other arrays)."""
    rng_eig = np.random.default_rng(seed).spawn(6)[0]
    kint = _kint(spec.nk)
    minus = _kidx(-kint, spec.nk)
    n_unocc = spec.n_bands - spec.n_occ
    eig = np.empty((spec.n_k, spec.n_bands))
    for k in range(spec.n_k):
        if minus[k] < k:
            eig[k] = eig[minus[k]]
            continue
        occ = np.sort(rng_eig.uniform(-0.8, -0.05, spec.n_occ))
        unocc = np.sort(rng_eig.uniform(0.05, 2.0, n_unocc))
        eig[k] = np.concatenate([occ, unocc])
    return eig


def window_of(eig: np.ndarray, n_occ: int) -> tuple:
    """transition_window from eigenvalues alone."""
    return float(eig[:, n_occ:].min() - eig[:, :n_occ].max()), float(eig[:, n_occ:].max() - eig[:, :n_occ].min())


def training_cells(config: int, n: int, **kw) -> List[System]:
    """n further seeded cells of workload `config`'s (first) shape, cells
    1..n of the seed convention (seed = 1000 * config + cell)."""
    return [make_system(CONFIGS[config][0], 1000 * config + 1 + i, **kw) for i in range(n)]


def make_config(config: int, cell: int = 0, **kw) -> System:
    """Cell `cell` of workload `config`; seed = 1000 * config + cell."""
    return make_system(CONFIGS[config][cell], 1000 * config + cell, **kw)


def make_custom(n_atoms=2, nb_per_atom=4, naux_per_atom=6, nk=(2, 1, 1), n_occ=2, n_freq=8,
                qp_lo=0, n_qp=None, seed=7, **kw) -> System:
    """A small cell of any shape (tests: ragged tiles, degenerate sizes)."""
    n_b = n_atoms * nb_per_atom
    if n_qp is None:
        n_qp = n_b
    spec = CellSpec(n_atoms=n_atoms, nb_per_atom=nb_per_atom, naux_per_atom=naux_per_atom,
                    nk=tuple(nk), n_occ=n_occ, n_freq=n_freq, qp_lo=qp_lo, n_qp=n_qp,
                    lattice="fcc" if n_atoms == 2 else "sc")
    return make_system(spec, seed, **kw)


def all_cells(config: int) -> List[System]:
    return [make_config(config, c) for c in range(len(CONFIGS[config]))]


# ---------------------------------------------------------------- surrogate inputs
# Random draws of the learned-surrogate form, made here and passed to both the
# library and the oracle: initial network parameters (values representable in
# BF16, so that both sides start from the same weights), the start block of
# the subspace iteration and the order in which training rows are visited.

def bf16_round(a) -> np.ndarray:
    """Round float values to the nearest BF16 value (ties to even), as float32."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def surrogate_init(n_in: int, hidden: int, n_out: int, seed: int, out_scale: float = 1.0) -> np.ndarray:
    """Flat parameters W1 [n_in][H], b1, W2 [H][H], b2, W3 [H][n_out], b3:
    weights uniform in +-sqrt(6/(fan_in+fan_out)) (W3 times out_scale; the
    targets are small residuals), biases zero, BF16 values."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (fi, fo) in enumerate(((n_in, hidden), (hidden, hidden), (hidden, n_out))):
        lim = math.sqrt(6.0 / (fi + fo)) * (out_scale if li == 2 else 1.0)
        parts.append(rng.uniform(-lim, lim, fi * fo))
        parts.append(np.zeros(fo))
    return bf16_round(np.concatenate(parts))


def surrogate_start(n_aux: int, rank: int, seed: int) -> np.ndarray:
    """Start block of the subspace iteration: float64 [n_aux][rank], U(-1,1)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (n_aux, rank))


def surrogate_order(n_rows: int, n_visits: int, seed: int) -> np.ndarray:
    """Row visiting order for training: concatenated permutations, int32."""
    rng = np.random.default_rng(seed)
    reps = (n_visits + n_rows - 1) // n_rows
    return np.concatenate([rng.permutation(n_rows) for _ in range(reps)])[:n_visits].astype(np.int32)


def transition_window(sysm: "System") -> tuple:
    """Smallest and largest occupied -> unoccupied energy difference over all
    k, k' (the band gap and the width of the transition spectrum), Ha."""
    occ = sysm.eig[:, :sysm.n_occ]
    unocc = sysm.eig[:, sysm.n_occ:]
    return float(unocc.min() - occ.max()), float(unocc.max() - occ.min())
