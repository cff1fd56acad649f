"""GPU parity of the two-centre LRI coefficient fit (lrigw_lri_fit, Eq.
two_center_coeff_determination) against the oracle's fit, and on the
real-space rig, where the fit is exact."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import lri
from synth.systems import make_config


def _ctx():
    from paper_2011_01400_amd import lrigw as L
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    return L, L.Context.from_system(make_config(1), precision="fp64")


def _spd_batch(rng, batch, n):
    A = rng.standard_normal((batch, n, n)) / np.sqrt(n)
    return np.einsum("bij,bkj->bik", A, A) + 0.5 * np.eye(n)[None]


@pytest.mark.parametrize("batch,n,n_keep,nrhs", [(1, 1, 1, 1), (4, 19, 19, 5), (1, 60, 30, 9), (3, 74, 37, 49),
                                               (5, 135, 45, 36), (2, 260, 130, 1521)])
def test_fit_matches_oracle(batch, n, n_keep, nrhs):
    L, ctx = _ctx()
    rng = np.random.default_rng(1000 + n)
    V = _spd_batch(rng, batch, n)
    T = rng.standard_normal((batch, n, nrhs))
    C = torch.full((batch, n_keep, nrhs), np.nan, dtype=torch.float64, device="cuda")
    print(f"\n[gpu fit] batch {batch} n {n} keep {n_keep} rhs {nrhs}", flush=True)
    ctx.lri_fit(torch.from_numpy(V).cuda(), torch.from_numpy(T).cuda(), n_keep, C, scale=0.5)
    got = C.cpu().numpy()
    for b in range(batch):
        ref = 0.5 * lri.fit_two_centre(T[b], V[b], n_keep)
        assert np.linalg.norm(got[b] - ref) / np.linalg.norm(ref) < 1e-12, b


def test_fit_not_positive_definite_reports_pair():
    L, ctx = _ctx()
    rng = np.random.default_rng(5)
    V = _spd_batch(rng, 4, 70)
    V[2, 10, 10] = -5.0
    T = rng.standard_normal((4, 70, 8))
    C = torch.zeros((4, 35, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(L.LrigwError) as e:
        ctx.lri_fit(torch.from_numpy(V).cuda(), torch.from_numpy(T).cuda(), 35, C)
    assert e.value.code == L.LRIGW_ERR_NOT_HPD


def test_fit_on_rig_recovers_coefficients():
    """The rig's products lie in their pair's auxiliary span: the device fit
    must return the rig's coefficients (half of the fit for on-site pairs)."""
    from tests.test_oracle_rig import NB_ATOM, build_rig
    L, ctx = _ctx()
    rig = build_rig()
    v, orb, abf = rig["v"], rig["orb"], rig["abf"]
    naux, blocks, Rs, boff = rig["naux_atoms"], rig["lri_blocks"], rig["Rs"], rig["basis_off"]
    for A in range(2):
        for B in range(2):
            for ir, R in enumerate(Rs):
                onsite = A == B and R == 0
                funcs = [abf(A, m, 0) for m in range(naux[A])]
                if not onsite:
                    funcs += [abf(B, m, R) for m in range(naux[B])]
                P = np.array(funcs)
                Vm = P @ v @ P.T
                prods = np.array([orb(A, a, 0) * orb(B, b, R) for a in range(NB_ATOM) for b in range(NB_ATOM)])
                T = P @ v @ prods.T
                C = torch.zeros((1, naux[A], NB_ATOM * NB_ATOM), dtype=torch.float64, device="cuda")
                ctx.lri_fit(torch.from_numpy(Vm[None]).cuda(), torch.from_numpy(T[None]).cuda(), naux[A], C,
                            scale=0.5 if onsite else 1.0)
                got = C.cpu().numpy()[0].reshape(naux[A], NB_ATOM, NB_ATOM)
                want = blocks[A][ir][:, :, boff[B]:boff[B] + NB_ATOM]
                assert np.max(np.abs(got - want)) < 1e-9 * max(1.0, np.max(np.abs(want))), (A, B, R)
