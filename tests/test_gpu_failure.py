"""Failure paths of the hot-path calls, each forced from the host with inputs
the kernels handle normally (status words and host checks, no fault):

* lrigw_screen with a Coulomb matrix that is not positive definite:
  ERR_NOT_HPD with info = -2; the whole pass names the failing q;
* lrigw_chi0 with an occupied level above an unoccupied one: ERR_ARG, also
  when new eigenvalues are written into a buffer that was checked before;
* lrigw_qp on a self-energy whose continuation gives no root: WARN_QP_NOCONV
  with the count of such states, E = e + e_static there (as the oracle's
  solver decides);
* lrigw_qp on an all-zero self-energy: WARN_PADE_TRUNC, E = e, Z = 1.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def c1():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_01400_amd import lrigw as L
    from synth.systems import make_config
    L.load()
    s = make_config(1)
    return dict(L=L, s=s, dev=L.device_inputs(s))


def _ctx(c1, precision="fp64"):
    return c1["L"].Context.from_system(c1["s"], precision=precision)


def test_screen_rejects_non_positive_definite_V(c1):
    L, s, dev = c1["L"], c1["s"], c1["dev"]
    print("\n[gpu failure] screen with V = -I", flush=True)
    ctx = _ctx(c1)
    n = s.n_aux
    chi = torch.zeros(int(ctx.sizes.w_elems), dtype=torch.complex128, device="cuda")
    W = ctx.empty("W")
    V = -torch.eye(n, dtype=torch.complex128, device="cuda")
    with pytest.raises(L.LrigwError) as e:
        ctx.screen(1, chi, V, W)
    assert e.value.code == L.LRIGW_ERR_NOT_HPD
    assert e.value.info == -2
    # a good V afterwards still screens (the failed call left no state behind)
    ctx.screen(1, chi, dev["V"][1], W)
    assert torch.all(W == 0)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "split_f16"])
def test_whole_pass_names_failing_q(c1, precision):
    L, s, dev = c1["L"], c1["s"], c1["dev"]
    print(f"\n[gpu failure] whole pass with V(q=3) = -V(q=3), {precision}", flush=True)
    ctx = _ctx(c1, precision)
    sp = s.spec
    H = ctx.empty("H")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    V = dev["V"].clone()
    V[3] = -V[3]
    sigma = torch.zeros((s.n_k, sp.n_qp, sp.n_freq), dtype=torch.complex128, device="cuda")
    e = torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    z = torch.zeros_like(e)
    with pytest.raises(L.LrigwError) as err:
        ctx.g0w0(H, dev["evec"], dev["eig"], V, dev["p"], s.omega_cell, dev["e_static"], 16, sigma, e, z)
    assert err.value.code == L.LRIGW_ERR_NOT_HPD
    ctx.close()


def test_chi0_rejects_overlapping_levels_in_a_reused_buffer(c1):
    L, s, dev = c1["L"], c1["s"], c1["dev"]
    print("\n[gpu failure] chi0 with an occupied level above an unoccupied one", flush=True)
    ctx = _ctx(c1)
    H = ctx.empty("H")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    M, chi = ctx.empty("M"), ctx.empty("W")
    ctx.build_M(1, 0, H, dev["evec"], M)
    eig = dev["eig"].clone()
    ctx.chi0(1, M, eig, chi)          # a good spectrum: accepted
    good = chi.clone()
    no = s.n_occ
    # same buffer, new contents: the highest occupied level of k = 2 above the
    # lowest unoccupied level of every k
    eig[2, no - 1] = float(s.eig[:, no:].min()) + 0.05
    with pytest.raises(L.LrigwError) as e:
        ctx.chi0(1, M, eig, chi)
    assert e.value.code == L.LRIGW_ERR_ARG
    # a non-finite level is refused as well
    eig.copy_(dev["eig"])
    eig[0, 0] = float("nan")
    with pytest.raises(L.LrigwError) as e:
        ctx.chi0(1, M, eig, chi)
    assert e.value.code == L.LRIGW_ERR_ARG
    # the original levels again: accepted, same result
    eig.copy_(dev["eig"])
    ctx.chi0(1, M, eig, chi)
    assert torch.equal(chi, good)
    ctx.close()


def test_qp_without_root_warns(c1):
    """Sigma(i w) = 2 i w continues to P(z) = 2z, so E - e - Re P(E - mu) =
    2 mu - e - E decreases everywhere: Newton stops at once (f' < 0) and the
    scan finds no increasing sign change.  Those states return E = e (no
    static term here), flagged; the others solve normally."""
    from oracle import continuation, grids
    L, s, dev = c1["L"], c1["s"], c1["dev"]
    print("\n[gpu failure] QP equation without a root", flush=True)
    ctx = _ctx(c1)
    sp = s.spec
    omega = grids.frequency_grid(sp.n_freq, sp.x0)[0]
    rng = np.random.default_rng(3)
    # a regular self-energy: a sum of two poles of positive residue
    sig = np.zeros((s.n_k, sp.n_qp, sp.n_freq), dtype=np.complex128)
    z = 1j * omega
    for k in range(s.n_k):
        for n in range(sp.n_qp):
            a1, a2 = 0.05 + 0.05 * rng.random(2)
            sig[k, n] = a1 / (z + s.mu - (-0.9)) + a2 / (z + s.mu - 2.5)
    bad = [(0, 0), (3, 5), (7, sp.n_qp - 1)]
    for k, n in bad:
        sig[k, n] = 2.0 * z
    eps = s.eig[:, sp.qp_lo:sp.qp_lo + sp.n_qp]
    e_st = np.zeros_like(eps)
    E = torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    Z = torch.zeros_like(E)
    rc, info = ctx.qp(torch.from_numpy(sig).cuda(), torch.from_numpy(np.ascontiguousarray(eps)).cuda(),
                      torch.from_numpy(e_st).cuda(), 16, E, Z)
    assert rc == L.LRIGW_WARN_QP_NOCONV
    assert info == len(bad)
    nodes = grids.pade_nodes(sp.n_freq, 16)
    Eo, Zo, ok = continuation.qp_energies(sig, omega, eps, e_st, s.mu, nodes)
    assert sorted(zip(*np.nonzero(~ok))) == sorted(bad)
    Eg = E.cpu().numpy()
    for k, n in bad:
        assert Eg[k, n] == eps[k, n]
    assert np.max(np.abs(Eg - Eo)) < 1e-9
    ctx.close()


def test_qp_zero_sigma_warns_truncation(c1):
    L, s, dev = c1["L"], c1["s"], c1["dev"]
    print("\n[gpu failure] Pade fit of an all-zero self-energy", flush=True)
    ctx = _ctx(c1)
    sp = s.spec
    sig = torch.zeros((s.n_k, sp.n_qp, sp.n_freq), dtype=torch.complex128, device="cuda")
    eps = np.ascontiguousarray(s.eig[:, sp.qp_lo:sp.qp_lo + sp.n_qp])
    E = torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    Z = torch.zeros_like(E)
    rc, info = ctx.qp(sig, torch.from_numpy(eps).cuda(), None, 16, E, Z)
    assert rc == L.LRIGW_WARN_PADE_TRUNC
    assert info == 0
    assert np.array_equal(E.cpu().numpy(), eps)
    assert np.all(Z.cpu().numpy() == 1.0)
    ctx.close()
