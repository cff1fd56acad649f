"""RI-exact discrete periodic rig: pins the oracle's LRI transform, chi0,
screening and Sigma^c against brute-force real-space evaluation.

A 1D crystal is sampled on a periodic grid (N_k cells of G points, the
Born-von Karman supercell).  Each cell holds two atoms carrying a few real,
localised orbital basis functions.  The auxiliary functions of the two atoms
together span every product of two orbital functions, so
the two-centre expansion of Sec. II C (Eq. realspace_expan1) is exact and the
LRI pipeline must reproduce the real-space formulas of Sec. II A to rounding:

  (1) psi_m^{k1*} psi_n^{k2} = sum_mu C^mu_{mn}(k1,k2) P_mu^{(k1-k2)*}   (Eq. KSproduct_expan)
  (2) chi0(x,x') from Eq. chi_0_realspace (f^q_n read as f^k_n)
  (3) W^c = (1 - v chi0)^-1 v - v, its Bloch matrix elements
  (4) Sigma^c_n(k, i w) from Eqs. gw_selfenergy_realspace / green_function_realspace
      on the same frequency grid.

The coefficients are the minimum-norm fit of each product on the union of the
two atoms' auxiliary functions; for an on-site product both sectors use the
same functions and the fit splits the coefficient evenly between them.
Grid sums carry unit measure; Bloch functions are normalised per cell.
"""
import numpy as np
import pytest

from oracle import grids
from oracle.pipeline import Oracle
from synth.systems import CellSpec, System

NK = 4          # cells in the supercell (k points)
G = 20          # grid points per cell
TAU = (5, 15)   # atom positions in a cell
W = 6           # orbital half-width (grid points)
NB_ATOM = 3
N_OCC = 2
NF = 10
S_SPIN = 2.0


def _place(vals, center, n_tot):
    out = np.zeros(n_tot)
    for o, v in zip(range(-W, W + 1), vals):
        out[(center + o) % n_tot] += v
    return out


@pytest.fixture(scope="module")
def rig():
    return build_rig()


def build_rig():
    rng = np.random.default_rng(2024)
    n_tot = NK * G
    n_b = 2 * NB_ATOM
    phi = rng.standard_normal((2, NB_ATOM, 2 * W + 1)) * np.hanning(2 * W + 3)[1:-1][None, None, :]
    Rs = (-1, 0, 1)

    def orb(A, a, cell):
        return _place(phi[A, a], TAU[A] + G * cell, n_tot)

    # auxiliary functions: orthonormal basis of the on-site products of atom A and
    # of its products with the functions of the other atom (B > A), so that every
    # product lies in the span of one atom's functions and the union of all
    # auxiliary functions stays linearly independent (V positive definite)
    abf_win = []
    for A in range(2):
        prods = [orb(A, a, 0) * orb(B, b, R) for a in range(NB_ATOM) for B in range(A, 2)
                 for b in range(NB_ATOM) for R in Rs]
        Pm = np.array(prods).T
        U, sv, _ = np.linalg.svd(Pm, full_matrices=False)
        U = U[:, sv > 1e-10 * sv[0]]
        win = np.array([[U[(TAU[A] + o) % n_tot, m] for o in range(-W, W + 1)] for m in range(U.shape[1])])
        abf_win.append(win)                      # [naux_A][2W+1]
    naux = [w.shape[0] for w in abf_win]
    aux_off = np.array([0, naux[0], naux[0] + naux[1]], dtype=np.int32)
    basis_off = np.array([0, NB_ATOM, 2 * NB_ATOM], dtype=np.int32)

    def abf(A, m, cell):
        return _place(abf_win[A][m], TAU[A] + G * cell, n_tot)

    # two-centre coefficients by minimum-norm fit on the union of both atoms' ABFs
    lri_blocks = [np.zeros((len(Rs), naux[A], NB_ATOM, n_b)) for A in range(2)]
    other = {}
    for A in range(2):
        for a in range(NB_ATOM):
            for B in range(2):
                for b in range(NB_ATOM):
                    for ir, R in enumerate(Rs):
                        p = orb(A, a, 0) * orb(B, b, R)
                        Umat = np.array([abf(A, m, 0) for m in range(naux[A])]
                                        + [abf(B, m, R) for m in range(naux[B])]).T
                        coef = np.linalg.pinv(Umat, rcond=1e-12) @ p
                        assert np.linalg.norm(Umat @ coef - p) < 1e-12
                        lri_blocks[A][ir, :, a, basis_off[B] + b] = coef[:naux[A]]
                        other[(A, a, B, b, R)] = coef[naux[A]:]
    # translation consistency of the second sector: coefficient on P_B(R) equals L_B(-R)[b, a]
    for (A, a, B, b, R), c in other.items():
        ir = Rs.index(-R)
        assert np.max(np.abs(lri_blocks[B][ir, :, b, basis_off[A] + a] - c)) < 1e-10

    kfrac = np.array([[n / NK, 0.0, 0.0] for n in range(NK)])
    minus = np.array([(-n) % NK for n in range(NK)])

    def bloch(f_cell, kf):
        return sum(f_cell(c) * np.exp(2j * np.pi * kf * c) for c in range(NK))

    # overlap, TRS eigenvectors normalised per cell (c^H S c = I), eigenvalues with a gap
    evec = np.zeros((NK, n_b, n_b), dtype=np.complex128)
    eig = np.zeros((NK, n_b))
    phik = np.zeros((NK, n_b, n_tot), dtype=np.complex128)
    for k in range(NK):
        for i in range(n_b):
            A, a = divmod(i, NB_ATOM)
            phik[k, i] = bloch(lambda c: orb(A, a, c), kfrac[k, 0])
    for k in range(NK):
        mk = minus[k]
        Sk = phik[k].conj() @ phik[k].T / NK
        lam, Us = np.linalg.eigh(Sk)
        Sih = (Us / np.sqrt(lam)[None, :]) @ Us.conj().T
        if mk < k:
            evec[k] = np.conj(evec[mk])
            eig[k] = eig[mk]
            continue
        if mk == k:
            Q = np.linalg.qr(rng.standard_normal((n_b, n_b)))[0]
        else:
            Q = np.linalg.qr(rng.standard_normal((n_b, n_b)) + 1j * rng.standard_normal((n_b, n_b)))[0]
        evec[k] = Sih @ Q
        eig[k] = np.concatenate([np.sort(rng.uniform(-0.7, -0.1, N_OCC)), np.sort(rng.uniform(0.15, 1.8, n_b - N_OCC))])
    psi = np.einsum("kin,kix->knx", evec, phik)           # [k][n][x]
    assert np.allclose(np.einsum("knx,kmx->knm", psi.conj(), psi) / NK, np.eye(n_b)[None], atol=1e-12)

    # circulant positive-definite Coulomb kernel on the supercell grid
    nn = np.fft.fftfreq(n_tot) * n_tot
    vhat = 4 * np.pi / (0.3 + (2 * np.pi * nn / n_tot) ** 2)
    F = np.exp(-2j * np.pi * np.outer(np.arange(n_tot), np.arange(n_tot)) / n_tot)
    v = (F.conj().T @ np.diag(vhat) @ F / n_tot).real

    # Bloch-summed ABFs P^q_mu(x) = sum_R P_mu(x - R - tau) e^{i q R}
    Pq = np.zeros((NK, aux_off[-1], n_tot), dtype=np.complex128)
    for q in range(NK):
        for A in range(2):
            for m in range(naux[A]):
                Pq[q, aux_off[A] + m] = bloch(lambda c: abf(A, m, c), kfrac[q, 0])
    Vq = np.einsum("qux,xy,qvy->quv", Pq.conj(), v, Pq) / NK

    spec = CellSpec(n_atoms=2, nb_per_atom=NB_ATOM, naux_per_atom=0, nk=(NK, 1, 1), n_occ=N_OCC,
                    n_freq=NF, qp_lo=0, n_qp=n_b)
    lri_flat = np.concatenate([b.reshape(-1) for b in lri_blocks])
    lri_off = np.array([0, lri_blocks[0].size, lri_flat.size], dtype=np.int64)
    R = np.array([[r, 0, 0] for r in Rs], dtype=np.int32)
    mu = 0.5 * (eig[:, N_OCC - 1].max() + eig[:, N_OCC].min())
    sysm = System(spec=spec, basis_off=basis_off, aux_off=aux_off, lattice=np.eye(3), R=R, lri=lri_flat,
                  lri_off=lri_off, eig=eig, evec=evec, V=Vq, p=np.zeros((NK, N_OCC, n_b - N_OCC), complex),
                  omega_cell=1.0, mu=mu, e_static=np.zeros((NK, n_b)), seed=0)
    return dict(sys=sysm, psi=psi, v=v, Pq=Pq, kfrac=kfrac, n_tot=n_tot, naux=int(aux_off[-1]), orb=orb, abf=abf,
                naux_atoms=naux, lri_blocks=lri_blocks, Rs=Rs, basis_off=basis_off)


def _oracle(rig):
    s = rig["sys"]
    # the rig's atoms carry different numbers of auxiliary functions, so the
    # oracle is assembled from its parts rather than from CellSpec counts
    o = Oracle.__new__(Oracle)
    sp = s.spec
    o.sys = s
    o.kint, o.kfrac = grids.kgrid(sp.nk)
    o.kpq, o.kmq, o.minus = grids.kq_tables(sp.nk)
    o.omega, o.weight = grids.frequency_grid(sp.n_freq, sp.x0)
    from oracle import lri
    o.tb = lri.TripleBuilder(s, o.kfrac)
    o.occ, o.unocc = slice(0, N_OCC), slice(N_OCC, sp.n_bands)
    o.qp, o.allb = slice(0, sp.n_bands), slice(0, sp.n_bands)
    o.n_par = min(16, sp.n_freq)
    return o


def test_product_expansion_exact(rig):
    o = _oracle(rig)
    psi, Pq = rig["psi"], rig["Pq"]
    nb = psi.shape[1]
    for k1 in range(NK):
        for k2 in range(NK):
            C = o.tb.mo(k1, k2, slice(0, nb), slice(0, nb))               # [mu][m][n]
            q = (k1 - k2) % NK
            lhs = psi[k1].conj()[:, None, :] * psi[k2][None, :, :]          # [m][n][x]
            rhs = np.einsum("umn,ux->mnx", C, Pq[q].conj())
            assert np.max(np.abs(lhs - rhs)) < 1e-13


def _brute_chi0(rig, omega):
    s = rig["sys"]
    psi = rig["psi"]
    nb = psi.shape[1]
    f = np.zeros(nb)
    f[:N_OCC] = 1
    n_tot = rig["n_tot"]
    chi = np.zeros((len(omega), n_tot, n_tot), dtype=np.complex128)
    for k in range(NK):
        for q in range(NK):
            kq = (k + q) % NK
            for m in range(nb):
                for n in range(nb):
                    df = f[m] - f[n]
                    if df == 0:
                        continue
                    a = psi[kq, m].conj() * psi[k, n]
                    for iw, w in enumerate(omega):
                        chi[iw] += S_SPIN * df / (s.eig[kq, m] - s.eig[k, n] - 1j * w) / NK / NK * np.outer(a, a.conj())
    return chi


def test_chi0_and_wc_match_real_space(rig):
    o = _oracle(rig)
    s = rig["sys"]
    Pq, v = rig["Pq"], rig["v"]
    chi_bf = _brute_chi0(rig, o.omega)
    chi_q = [o.chi0(q) for q in range(NK)]
    # chi0(x,x') = sum_q w_q P^q(x) chi~(q) P^{q*}(x')
    rec = sum(np.einsum("ux,wuv,vy->wxy", Pq[q], chi_q[q], Pq[q].conj()) for q in range(NK)) / NK
    assert np.max(np.abs(rec - chi_bf)) < 1e-13 * np.max(np.abs(chi_bf))
    n_tot = rig["n_tot"]
    for q in range(NK):
        Wc = o.wc(q, chi=chi_q[q], gamma=False)
        for iw in range(len(o.omega)):
            Wbf = np.linalg.solve(np.eye(n_tot) - v @ chi_bf[iw], v) - v
            ref = Pq[q].conj() @ Wbf @ Pq[q].T / NK
            assert np.max(np.abs(Wc[iw] - ref)) < 1e-11 * np.max(np.abs(ref))


def test_sigma_matches_real_space(rig):
    o = _oracle(rig)
    s = rig["sys"]
    psi, v = rig["psi"], rig["v"]
    nb = psi.shape[1]
    n_tot = rig["n_tot"]
    r = o.run(gamma=False)
    chi_bf = _brute_chi0(rig, o.omega)
    Wbf = [np.linalg.solve(np.eye(n_tot) - v @ chi_bf[j], v) - v for j in range(len(o.omega))]
    for k in (0, 1):
        for n in (0, N_OCC, nb - 1):
            for i in (0, 4, 9):
                tot = 0.0j
                for kp in range(NK):
                    for m in range(nb):
                        a = psi[k, n].conj() * psi[kp, m]           # psi_n^{k*}(x) psi_m^{k'}(x)
                        for j, wj in enumerate(o.omega):
                            z = 1j * o.omega[i] + s.mu - s.eig[kp, m]
                            ker = z / (z * z + wj * wj)
                            tot += -(1 / np.pi) * o.weight[j] * ker / NK * (a @ Wbf[j] @ a.conj())
                tot /= NK   # per-cell normalised diagonal element
                assert abs(r["sigma"][k, n, i] - tot) < 1e-12 * max(1.0, abs(tot))


def test_rig_detects_swapped_sectors(rig, monkeypatch):
    """Eq. AO_triple_split as printed (atom labels of the two sectors interchanged)
    must break the exact product expansion; the rig is sensitive to it."""
    from oracle import lri

    def swapped(Lk2, Lmk1, basis_off, aux_off, n_b):
        n_aux = int(aux_off[-1])
        Ct = np.zeros((n_aux, n_b, n_b), dtype=np.complex128)
        for A in range(len(Lk2)):
            mu = slice(int(aux_off[A]), int(aux_off[A + 1]))
            a = slice(int(basis_off[A]), int(basis_off[A + 1]))
            Ct[mu, :, a] += np.transpose(Lk2[A], (0, 2, 1))
            Ct[mu, a, :] += Lmk1[A]
        return Ct

    monkeypatch.setattr(lri, "ao_triple", swapped)
    o = _oracle(rig)
    psi, Pq = rig["psi"], rig["Pq"]
    nb = psi.shape[1]
    C = o.tb.mo(1, 0, slice(0, nb), slice(0, nb))
    lhs = psi[1].conj()[:, None, :] * psi[0][None, :, :]
    rhs = np.einsum("umn,ux->mnx", C, Pq[1].conj())
    assert np.max(np.abs(lhs - rhs)) > 1e-3


def test_coulomb_metric_fit_recovers_rig_coefficients(rig):
    """Eq. two_center_coeff_determination on the rig: every orbital product lies
    in the span of its pair's auxiliary functions, so the Coulomb-metric fit
    must return the rig's exact coefficients (those of its minimum-norm fit);
    for an on-site pair the fit on I's functions alone gives twice the stored
    block (the two sectors share one coefficient)."""
    from oracle import lri
    v, orb, abf = rig["v"], rig["orb"], rig["abf"]
    naux, blocks, Rs, boff = rig["naux_atoms"], rig["lri_blocks"], rig["Rs"], rig["basis_off"]
    for A in range(2):
        for B in range(2):
            for ir, R in enumerate(Rs):
                onsite = A == B and R == 0
                funcs = [abf(A, m, 0) for m in range(naux[A])]
                if not onsite:
                    funcs += [abf(B, m, R) for m in range(naux[B])]
                P = np.array(funcs)                               # [n][x]
                Vm = P @ v @ P.T
                prods = np.array([orb(A, a, 0) * orb(B, b, R) for a in range(NB_ATOM) for b in range(NB_ATOM)])
                T = P @ v @ prods.T                               # [n][(a, b)]
                C = lri.fit_two_centre(T, Vm, naux[A]).reshape(naux[A], NB_ATOM, NB_ATOM)
                stored = blocks[A][ir][:, :, boff[B]:boff[B] + NB_ATOM]
                want = 2.0 * stored if onsite else stored
                assert np.max(np.abs(C - want)) < 1e-9 * max(1.0, np.max(np.abs(want))), (A, B, R)


def test_sigma_x_matches_real_space(rig):
    """Sigma^x (the bare-Coulomb term of Eq. GW_selfe_element, occupied sum,
    w_q = 1/N_q) against the brute-force real-space exchange on the
    supercell grid:
        Sigma^x_n(k) = -(1/N_k) sum_{k'} sum_{m occ} <psi_n^k psi_m^{k'}| v |psi_m^{k'} psi_n^k>
    (Bloch functions normalised per cell, grid sums of unit measure, a per-cell
    diagonal element, no spin factor).  A factor 2, a missing 1/N_q or the
    empty bands in the sum each miss it by far more than rounding."""
    o = _oracle(rig)
    s = rig["sys"]
    psi, v = rig["psi"], rig["v"]
    nb = psi.shape[1]
    sx = o.sigma_x()
    ref = np.zeros((NK, nb))
    all_bands = np.zeros((NK, nb))
    for k in range(NK):
        for n in range(nb):
            for kp in range(NK):
                for m in range(nb):
                    a = psi[k, n].conj() * psi[kp, m]
                    val = -(a @ v @ a.conj()).real / NK / NK
                    all_bands[k, n] += val
                    if m < N_OCC:
                        ref[k, n] += val
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(sx - ref)) < 1e-13 * scale
    # the variants a magnitude error would give are far outside that bound
    assert np.max(np.abs(sx - 2.0 * ref)) > 0.1 * scale
    assert np.max(np.abs(sx - NK * ref)) > 0.1 * scale
    assert np.max(np.abs(sx - all_bands)) > 0.1 * scale
