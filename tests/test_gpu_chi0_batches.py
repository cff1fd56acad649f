"""GPU: K splits beyond what the partial-tile buffer holds (at most 3 GiB) run
in batches whose reductions add up in the output.  A cell with a large
auxiliary basis and many frequencies (N_aux 1040, 48 frequencies: 240 MB of
partial tiles per split in the complex64 forms, 481 MB in FP64) and K = 1024
rows, with 16 splits set explicitly: 13 + 3 splits per batch in the FP32 and
split forms, 6 + 6 + 4 in FP64.  chi~ of one q against the oracle and
against the unbatched single-split result."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.pipeline import Oracle
from synth.systems import make_custom


def relf(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def cell():
    from paper_2011_01400_amd import lrigw as L
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    s = make_custom(n_atoms=8, nb_per_atom=5, naux_per_atom=130, nk=(2, 2, 1), n_occ=8, n_freq=48, seed=29)
    assert s.n_k * s.n_occ * (s.n_bands - s.n_occ) == 1024
    print(f"\n[gpu chi0 batches] N_aux {s.n_aux}, K 1024, {s.spec.n_freq} frequencies", flush=True)
    o = Oracle(s)
    q = 1
    ref = o.chi0(q)
    return L, s, L.device_inputs(s), q, ref


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("split_f16", 1e-5), ("split_bf16", 1e-5)])
def test_batched_splits(cell, precision, tol):
    L, s, dev, q, ref = cell
    ctx = L.Context.from_system(s, precision=precision)
    H, M, chi = ctx.empty("H"), ctx.empty("M"), ctx.empty("W")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    ctx.build_M(q, 0, H, dev["evec"], M)
    nw, _, pad, var = ctx.tiles
    got = {}
    for splits in (1, 16):
        ctx.set_tiles(nw, splits, pad, var)
        chi.zero_()
        ctx.chi0(q, M, dev["eig"], chi)
        got[splits] = chi.cpu().numpy().reshape(ref.shape).astype(np.complex128)
    e1, e16 = relf(got[1], ref), relf(got[16], ref)
    d = relf(got[16], got[1])
    print(f"  {precision}: vs oracle {e1:.2e} (1 split), {e16:.2e} (16 splits in batches); between them {d:.2e}",
          flush=True)
    assert e1 < tol and e16 < tol
    assert np.max(np.abs(got[16] - got[16].conj().transpose(0, 2, 1))) == 0.0
    ctx.close()
