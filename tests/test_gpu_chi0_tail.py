"""GPU: the response kernels at the auxiliary-basis sizes that decide how the
last 64-row tile row runs.  With at most 16 rows left in it, the eight-wave
kernel takes that row's tiles with rows and columns swapped (its 16 rows
weighted, sixteen frequencies per workgroup, the tile stored conjugated and
transposed); with 17 or more it takes them like every other tile.  N_aux 12
(a single tile row, all swapped), 79 and 80 (15 and 16 rows left), 81 (17
left), with 19 frequencies (a partial group of sixteen and of four), in every
split form, for the eight-wave and the four-wave kernels, with one K split and
with four (K 288 in splits of 96 rows, the last of them empty): chi~ of one q
against the oracle, and exactly Hermitian."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.pipeline import Oracle
from synth.systems import make_custom


def relf(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module", params=[12, 79, 80, 81])
def cell(request):
    from paper_2011_01400_amd import lrigw as L
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    s = make_custom(n_atoms=1, nb_per_atom=22, naux_per_atom=request.param, nk=(2, 2, 1), n_occ=4, n_freq=19,
                    qp_lo=0, n_qp=2, seed=61)
    assert s.n_aux == request.param and s.n_k * s.n_occ * (s.n_bands - s.n_occ) == 288
    print(f"\n[gpu chi0 tail] N_aux {s.n_aux} ({s.n_aux - 64 * ((s.n_aux - 1) // 64)} rows in the last tile row), "
          f"K 288, {s.spec.n_freq} frequencies", flush=True)
    q = 1
    return L, s, L.device_inputs(s), q, Oracle(s).chi0(q)


@pytest.mark.parametrize("precision", ["split_f16", "split_bf16", "split3_bf16", "split_mixed"])
def test_last_tile_row(cell, precision):
    L, s, dev, q, ref = cell
    ctx = L.Context.from_system(s, precision=precision)
    H, M, chi = ctx.empty("H"), ctx.empty("M"), ctx.empty("W")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    ctx.build_M(q, 0, H, dev["evec"], M)
    _, _, pad, var = ctx.tiles
    for nw in (4, 2):
        for splits in (1, 4):
            ctx.set_tiles(nw, splits, pad, var)
            chi.zero_()
            ctx.chi0(q, M, dev["eig"], chi)
            c = chi.cpu().numpy().reshape(ref.shape).astype(np.complex128)
            e = relf(c, ref)
            print(f"  {precision} nw {nw} splits {splits}: vs oracle {e:.2e}", flush=True)
            assert e < 1e-5, (nw, splits)
            assert np.max(np.abs(c - c.conj().transpose(0, 2, 1))) == 0.0
    ctx.close()
