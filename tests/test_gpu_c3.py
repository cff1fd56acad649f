"""GPU, full size: the six uneven Si-like cells (2, 2, 4, 4, 6, 8 atoms; N_aux
260 to 1040; 4x4x4 and 3x3x3 k; 32 frequencies) in one captured hipGraph,
FP16 form with the tile autotuner, as `bench.py --workload batched` runs them.
Checked: every cell's status; each cell's batched result equals its own
lrigw_g0w0 on the same tuned context; on the smallest cell one q's Sigma^c
contribution at sampled k points equals the FP64 oracle's; and on the
largest cell two q against the oracle's sampled values (golden file).

Sigma^c(k) = Sigma^c(-k) does not hold with one direction q_hat. The q -> 0
head and wings are taken along q_hat, and the wings are odd in p.q_hat. These
inputs have no crystal symmetry to cancel them, so W^c(0) is complex and the
q = 0 term differs between k and -k: by 1e-4 relative in the FP64 oracle as
well, while without the Gamma correction the oracle is symmetric to rounding.
With the six Cartesian half-axes set on every context, the second graph of
the last test restores the symmetry."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.pipeline import Oracle
from synth.systems import all_cells


def _lib():
    from paper_2011_01400_amd import lrigw as L
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    return L


@pytest.fixture(scope="module")
def batched():
    L = _lib()
    t0 = time.perf_counter()
    cells = all_cells(3)
    print(f"\n[gpu c3] inputs of {len(cells)} cells in {time.perf_counter() - t0:.1f} s", flush=True)
    stream = torch.cuda.Stream()
    items = []
    with torch.cuda.stream(stream):
        for s in cells:
            dev = L.device_inputs(s)
            ctx = L.Context.from_system(s, precision="split_f16")
            H = ctx.empty("H")
            ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
            sp = s.spec
            items.append(dict(ctx=ctx, H=H, evec=dev["evec"], eig=dev["eig"], V=dev["V"], p=dev["p"],
                              omega_cell=s.omega_cell, e_static=dev["e_static"], n_par=16,
                              sigma=torch.zeros((s.n_k, sp.n_qp, sp.n_freq), dtype=torch.complex128, device="cuda"),
                              e_qp=torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda"),
                              z=torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")))
    torch.cuda.synchronize()
    b = L.Batch(items, autotune=True, stream=stream)
    for rep in range(2):
        b.run()
        st = b.status()
        print(f"[gpu c3] graph replay {rep}: status {st}", flush=True)
    torch.cuda.synchronize()
    return L, cells, items, b, st


def test_status(batched):
    L, cells, items, b, st = batched
    for i, (s, it) in enumerate(zip(cells, items)):
        assert st[i][0] == -1 and st[i][1] == 0, (i, st[i])
        assert np.all(np.isfinite(it["sigma"].cpu().numpy()))
        assert np.all(np.isfinite(it["e_qp"].cpu().numpy()))
        z = it["z"].cpu().numpy()
        print(f"  cell {i} ({s.spec.n_atoms} atoms, N_aux {s.n_aux}, {s.n_k} k): Z in [{z.min():.3f}, {z.max():.3f}]",
              flush=True)


def test_batched_equals_per_cell_pass(batched):
    L, cells, items, b, st = batched
    for i, (s, it) in enumerate(zip(cells, items)):
        sp = s.spec
        sg = torch.zeros_like(it["sigma"])
        e = torch.zeros_like(it["e_qp"])
        z = torch.zeros_like(it["z"])
        it["ctx"].g0w0(it["H"], it["evec"], it["eig"], it["V"], it["p"], it["omega_cell"], it["e_static"], 16, sg, e, z)
        torch.cuda.synchronize()
        ds = np.max(np.abs(sg.cpu().numpy() - it["sigma"].cpu().numpy()))
        de = np.max(np.abs(e.cpu().numpy() - it["e_qp"].cpu().numpy())) * 27211.386
        print(f"  cell {i}: batched vs own pass max|dSigma| {ds:.1e} Ha, max|dE| {de:.1e} meV", flush=True)
        assert ds < 1e-12 and de < 1e-6


def test_smallest_cell_one_q_against_oracle(batched):
    L, cells, items, b, st = batched
    i = min(range(len(cells)), key=lambda j: cells[j].n_aux * cells[j].n_k)
    s, it = cells[i], items[i]
    sp = s.spec
    ctx = it["ctx"]
    q = 1
    dev = L.device_inputs(s)
    torch.cuda.synchronize()
    M, x, chi, W = ctx.empty("M"), ctx.empty("x"), ctx.empty("W"), ctx.empty("W")
    ctx.build_M(q, 0, it["H"], it["evec"], M)
    ctx.chi0(q, M, it["eig"], chi)
    ctx.screen(q, chi, dev["V"][q], W)
    ctx.build_M(q, 1, it["H"], it["evec"], x)
    sg = torch.zeros((s.n_k, sp.n_qp, sp.n_freq), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()            # the context launches on the batch's stream
    ctx.sigma_c(q, x, W, it["eig"], sg)
    torch.cuda.synchronize()
    ks = [0, 5, s.n_k - 1]
    t0 = time.perf_counter()
    o = Oracle(s)
    ref, _ = o.sigma_q(q, o.wc(q, gamma=False), ks)
    got = sg.cpu().numpy()[ks]
    e = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"  cell {i} (N_aux {s.n_aux}, {s.n_k} k) q={q}: sampled Sigma^c rel {e:.1e} "
          f"(oracle {time.perf_counter() - t0:.1f} s)", flush=True)
    assert e < 2e-5


def test_largest_cell_sampled_q_against_oracle(batched):
    """The largest cell (8 atoms, N_aux 1040, the streaming self-energy kernel
    and the multi-block Cholesky) with its tuned FP16 tiles, and the plain FP64
    path, against the oracle's values for two q (q = 0 with the Gamma
    treatment) written by tests/golden/make_c3_golden.py: chi0 and W^c rows at
    three frequencies, and the Sigma^c contribution at three k.  Its batched
    result equals its own pass (test_batched_equals_per_cell_pass)."""
    import os
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_cell5_sampled.npz")
    if not os.path.exists(gold):
        pytest.skip("c3_cell5_sampled.npz not written")
    L, cells, items, b, st = batched
    g = np.load(gold)
    i = int(g["CELL"])
    s, it = cells[i], items[i]
    assert int(g["seed"]) == s.seed
    sp = s.spec
    n = s.n_aux
    rows = int(g["ROWS"])
    widx, kidx = g["W_IDX"], g["K_IDX"]
    dev = L.device_inputs(s)
    torch.cuda.synchronize()

    def relf(a, b_):
        return np.linalg.norm(a - b_) / np.linalg.norm(b_)

    for precision, tol in (("split_f16", 1e-5), ("fp64", 1e-10)):
        if precision == "split_f16":
            ctx, H = it["ctx"], it["H"]
        else:
            ctx = L.Context.from_system(s, precision="fp64")
            H = ctx.empty("H")
            ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
        ctx.gamma_prepare(dev["V"][0], dev["p"], s.omega_cell)
        M, x, chi, W = ctx.empty("M"), ctx.empty("x"), ctx.empty("W"), ctx.empty("W")
        for q in g["Q"]:
            q = int(q)
            # the batched contexts launch on the batch's stream, the copies
            # below run on the default one: the device is synchronised first
            ctx.build_M(q, 0, H, dev["evec"], M)
            ctx.chi0(q, M, dev["eig"], chi)
            torch.cuda.synchronize()
            ec = relf(chi.cpu().numpy().reshape(-1, n, n)[widx, :rows], g[f"chi_q{q}"])
            if q == 0:
                ctx.chi0(0, M, dev["eig"], chi, apply_gamma=True)
            ctx.screen(q, chi, dev["V"][q], W)
            torch.cuda.synchronize()
            ew = relf(W.cpu().numpy().reshape(-1, n, n)[widx, :rows], g[f"wc_q{q}"])
            ctx.build_M(q, 1, H, dev["evec"], x)
            sig = torch.zeros((s.n_k, sp.n_qp, sp.n_freq), dtype=torch.complex128, device="cuda")
            torch.cuda.synchronize()
            ctx.sigma_c(q, x, W, dev["eig"], sig)
            torch.cuda.synchronize()
            ref = g[f"sigma_q{q}"]
            es = np.max(np.abs(sig.cpu().numpy()[kidx] - ref)) / np.max(np.abs(ref))
            print(f"  cell {i} q={q} {precision} (tiles {ctx.tiles}): chi {ec:.2e}  Wc {ew:.2e}  Sigma_q {es:.2e}",
                  flush=True)
            assert ec < tol and ew < 10 * tol and es < 10 * tol
        del M, x, chi, W
        if precision == "fp64":
            ctx.close()


def test_batched_with_directions_restores_time_reversal(batched):
    """The six Cartesian half-axes set on every cell's context and the cells
    captured in a second graph: each cell's Sigma^c(k) equals Sigma^c(-k) to
    the form's rounding, and equals its own direction-averaged pass."""
    from oracle import grids as og
    from synth.systems import cartesian_directions, momentum_vectors, project_momentum
    L, cells, items, b, st = batched
    q, w = cartesian_directions()
    items2 = []
    for s, it in zip(cells, items):
        pd = torch.from_numpy(project_momentum(momentum_vectors(s), q)).cuda()
        it["ctx"].set_gamma_directions(pd, w)
        items2.append(dict(it, sigma=torch.zeros_like(it["sigma"]), e_qp=torch.zeros_like(it["e_qp"]),
                           z=torch.zeros_like(it["z"])))
    try:
        b2 = L.Batch(items2, autotune=False, stream=b.stream)
        b2.run()
        torch.cuda.synchronize()
        st2 = b2.status()
        for i, (s, it) in enumerate(zip(cells, items2)):
            assert st2[i][0] == -1 and st2[i][1] == 0, (i, st2[i])
            minus = og.kq_tables(s.spec.nk)[2]
            a = it["sigma"].cpu().numpy()
            trs = np.max(np.abs(a - a[minus])) / np.max(np.abs(a))
            sg, e, z = torch.zeros_like(it["sigma"]), torch.zeros_like(it["e_qp"]), torch.zeros_like(it["z"])
            it["ctx"].g0w0(it["H"], it["evec"], it["eig"], it["V"], it["p"], it["omega_cell"], it["e_static"], 16, sg, e, z)
            torch.cuda.synchronize()
            ds = np.max(np.abs(sg.cpu().numpy() - a))
            print(f"  cell {i} with directions: |Sigma(k) - Sigma(-k)| rel {trs:.1e}, batched vs own pass {ds:.1e} Ha",
                  flush=True)
            assert trs < 1e-6 and ds < 1e-12
    finally:
        for it in items:
            it["ctx"].set_gamma_directions(None, None)
