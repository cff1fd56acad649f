"""LRI pins (oracle): Bloch transform, AO triple symmetry, gauge and relabelling
invariance of the whole path, zero coupling, time-reversal symmetry."""
import dataclasses

import numpy as np
import pytest

from oracle import lri, grids
from oracle.pipeline import Oracle
from synth.systems import make_config, make_custom


def test_bloch_transform_direct_loop(c1_system):
    s = c1_system
    _, kfrac = grids.kgrid(s.spec.nk)
    blk = s.lri_block(1)
    Lk = lri.lri_bloch([blk], s.R, kfrac)[0]
    k = 5
    ref = np.zeros(blk.shape[1:], dtype=np.complex128)
    for r in range(s.R.shape[0]):
        ref += np.exp(2j * np.pi * np.dot(kfrac[k], s.R[r])) * blk[r]
    assert np.max(np.abs(Lk[k] - ref)) < 1e-13
    # real coefficients: C~(-k) = conj C~(k); periodic in reciprocal lattice vectors
    Lm = lri.lri_bloch([blk], s.R, -kfrac)[0]
    assert np.max(np.abs(Lm - Lk.conj())) < 1e-13
    Lg = lri.lri_bloch([blk], s.R, kfrac + np.array([1.0, -2.0, 3.0]))[0]
    assert np.max(np.abs(Lg - Lk)) < 1e-12


def test_product_hermiticity(c1_oracle):
    # psi_m^{k1*} psi_n^{k2} = conj(psi_n^{k2*} psi_m^{k1}): C^mu_{mn}(k1,k2) = conj C^mu_{nm}(k2,k1)
    tb = c1_oracle.tb
    allb = slice(0, 16)
    for k1, k2 in [(0, 3), (2, 7), (5, 5)]:
        a = tb.mo(k1, k2, allb, allb)
        b = tb.mo(k2, k1, allb, allb)
        assert np.max(np.abs(a - np.transpose(b, (0, 2, 1)).conj())) < 1e-13


def _run(sysm):
    o = Oracle(sysm)
    return o, o.run(keep=True)


def test_gauge_invariance(c1_oracle):
    base = c1_oracle.result
    s = c1_oracle.sys
    rng = np.random.default_rng(5)
    ev = s.evec.copy()
    # independent phase per (k, n), consistent with time reversal (c(-k) = conj c(k))
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, ev.shape[::2]))
    kpq, kmq, minus = grids.kq_tables(s.spec.nk)
    for k in range(s.n_k):
        if minus[k] == k:
            ph[k] = np.sign(np.cos(np.angle(ph[k]))) + 0j  # real orbitals stay real
        elif minus[k] < k:
            ph[k] = np.conj(ph[minus[k]])
    ev = ev * ph[:, None, :]
    no = s.n_occ
    p = s.p * np.conj(ph[:, :no])[:, :, None] * ph[:, no:][:, None, :]   # p_ia = <psi_i|p|psi_a>
    s2 = dataclasses.replace(s, evec=ev, p=p)
    _, r = _run(s2)
    for q in (0, 3):
        assert np.max(np.abs(r["per_q"][q]["chi"] - base["per_q"][q]["chi"])) < 1e-12
        assert np.max(np.abs(r["per_q"][q]["Wc"] - base["per_q"][q]["Wc"])) < 1e-11
    assert np.max(np.abs(r["sigma"] - base["sigma"])) < 1e-12
    assert np.max(np.abs(r["E"] - base["E"])) < 1e-10


def test_atom_relabelling(c1_oracle):
    s = c1_oracle.sys
    base = c1_oracle.result
    nb, na = s.spec.nb_per_atom, s.spec.naux_per_atom
    perm_b = np.concatenate([np.arange(nb, 2 * nb), np.arange(0, nb)])
    perm_a = np.concatenate([np.arange(na, 2 * na), np.arange(0, na)])
    blocks = [s.lri_block(1), s.lri_block(0)]
    blocks = [b[:, :, :, perm_b] for b in blocks]
    lri_new = np.concatenate([b.reshape(-1) for b in blocks])
    s2 = dataclasses.replace(s, lri=lri_new, evec=s.evec[:, perm_b, :], V=s.V[:, perm_a][:, :, perm_a])
    _, r = _run(s2)
    for q in (1, 6):
        c_new = r["per_q"][q]["chi"]
        c_old = base["per_q"][q]["chi"][:, perm_a][:, :, perm_a]
        assert np.max(np.abs(c_new - c_old)) < 1e-12
    assert np.max(np.abs(r["sigma"] - base["sigma"])) < 1e-12


def test_zero_coupling():
    s = make_config(1, lri_scale=0.0)
    _, r = _run(s)
    assert np.max(np.abs(r["per_q"][2]["chi"])) == 0.0
    assert np.max(np.abs(r["per_q"][2]["Wc"])) == 0.0
    assert np.max(np.abs(r["sigma"])) == 0.0
    assert np.max(np.abs(r["E"] - s.eig[:, :16])) == 0.0


def test_time_reversal_of_outputs():
    # Away from the Gamma head/wings, Sigma_n(k) = Sigma_n(-k) on time-reversal-symmetric
    # inputs.  The q -> 0 wings are odd in q_hat (p.q_hat changes sign), so with p != 0 the
    # partner relation is Sigma_n(-k; q_hat) = Sigma_n(k; -q_hat).
    s = make_custom(n_atoms=2, nb_per_atom=3, naux_per_atom=5, nk=(3, 3, 1), n_occ=2, n_freq=12, seed=9,
                    p_scale=0.0)
    o, r = _run(s)
    for k in range(s.n_k):
        mk = o.minus[k]
        assert np.max(np.abs(r["sigma"][k] - r["sigma"][mk])) < 1e-13
        assert np.max(np.abs(r["E"][k] - r["E"][mk])) < 1e-9
    s1 = make_custom(n_atoms=2, nb_per_atom=3, naux_per_atom=5, nk=(3, 3, 1), n_occ=2, n_freq=12, seed=9)
    s2 = dataclasses.replace(s1, p=-s1.p)
    o1, r1 = _run(s1)
    _, r2 = _run(s2)
    assert np.max(np.abs(r1["sigma"][1] - r1["sigma"][o1.minus[1]])) > 1e-8   # wings break k <-> -k
    for k in range(s1.n_k):
        assert np.max(np.abs(r1["sigma"][k] - r2["sigma"][o1.minus[k]])) < 1e-13


@pytest.mark.parametrize("cell", ["c1", "ragged", "nontrim"])
def test_per_atom_triples_equal_dense(c1_system, cell):
    """The per-atom evaluation of Eqs. AO_triple_split2 / AO_MO_transform (no
    dense AO tensor; the form the oracle uses for large cells) against the
    dense tensor, every Bloch pair and band block."""
    if cell == "c1":
        s = c1_system
    elif cell == "ragged":
        s = make_custom(n_atoms=3, nb_per_atom=5, naux_per_atom=7, nk=(2, 2, 1), n_occ=3, n_freq=6, seed=41)
    else:
        s = make_custom(n_atoms=2, nb_per_atom=4, naux_per_atom=9, nk=(3, 1, 2), n_occ=2, n_freq=6, seed=43)
    _, kfrac = grids.kgrid(s.spec.nk)
    dense = lri.TripleBuilder(s, kfrac)
    pa = lri.TripleBuilder(s, kfrac, per_atom=True)
    nb, no = s.spec.n_bands, s.spec.n_occ
    blocks = [(slice(0, no), slice(no, nb)), (slice(0, nb), slice(0, nb)), (np.array([no - 1, no]), slice(0, no))]
    for k1 in range(s.n_k):
        for k2 in range(s.n_k):
            for rows, cols in blocks:
                a = dense.mo(k1, k2, rows, cols)
                b = pa.mo(k1, k2, rows, cols)
                assert np.max(np.abs(a - b)) < 1e-14 * max(1.0, np.max(np.abs(a)))


def test_per_atom_triples_expand_rig_products_exactly():
    """On the real-space rig (atoms with different numbers of auxiliary
    functions), the per-atom triples reproduce every Bloch product exactly."""
    from tests.test_oracle_rig import NK, build_rig
    rig = build_rig()
    s = rig["sys"]
    pa = lri.TripleBuilder(s, rig["kfrac"], per_atom=True)
    psi, Pq = rig["psi"], rig["Pq"]
    nb = psi.shape[1]
    for k1 in range(NK):
        for k2 in range(NK):
            C = pa.mo(k1, k2, slice(0, nb), slice(0, nb))
            lhs = psi[k1].conj()[:, None, :] * psi[k2][None, :, :]
            rhs = np.einsum("umn,ux->mnx", C, Pq[(k1 - k2) % NK].conj())
            assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_streamed_blocks_and_k_partition():
    """An oracle fed the coefficients atom by atom (the cell not holding them)
    forms the same triples; chi~ summed over a partition of the k grid is the
    whole k sum."""
    from synth.systems import lri_blocks, make_system
    s = make_custom(n_atoms=2, nb_per_atom=5, naux_per_atom=9, nk=(3, 1, 2), n_occ=3, n_freq=6, seed=17)
    bare = make_system(s.spec, s.seed, materialize_lri=False)
    o = Oracle(s, per_atom=True)
    ob = Oracle(bare, per_atom=True, lri_blocks=lri_blocks(s.spec, s.seed))
    for q in (0, 4):
        B = o.B(q)
        assert np.array_equal(B, ob.B(q))
        full = o.chi0(q, B)
        parts = [[0, 3], [1, 4, 5], [2]]
        tot = sum(ob.chi0(q, ks=ks) for ks in parts)
        assert np.max(np.abs(tot - full)) < 1e-14 * np.max(np.abs(full))
        sub = ob.chi0(q, omega=o.omega[[1, 4]], ks=[1, 2])
        ref = o.chi0(q, B[[1, 2]], omega=o.omega[[1, 4]], ks=[1, 2])
        assert np.array_equal(sub, ref)
    with pytest.raises(ValueError):
        Oracle(bare)
