"""GPU parity of the contour-deformation path (lrigw_set_real_grid,
lrigw_chi0_real, lrigw_screen_real, lrigw_sigma_cd, lrigw_sigma_cd_pass,
lrigw_g0w0_cd) against the FP64 oracle on the same seeded inputs, its error
and warning paths, and sampled k points of the Si-like cell.

Energies are drawn inside [VBM - 0.45 D_min, CBM + 0.45 D_min] and the real
grid reaches 0.6 D_min, so every residue frequency lies on the grid; the
linearised QP step evaluates at e_n -+ delta, where states far from the band
edges have residues beyond the grid and give NaN on both sides alike."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import contour, continuation, grids
from oracle.pipeline import Oracle
from synth.systems import make_config, make_custom

HA_MEV = 27211.386


def _lib():
    from paper_2011_01400_amd import lrigw as L
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    return L


def relf(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = {
    "c1": lambda: make_config(1),
    "ragged": lambda: make_custom(n_atoms=2, nb_per_atom=7, naux_per_atom=37, nk=(3, 1, 2), n_occ=5, n_freq=10,
                                  qp_lo=2, n_qp=6, seed=17),
    "three_atoms": lambda: make_custom(n_atoms=3, nb_per_atom=6, naux_per_atom=45, nk=(1, 1, 1), n_occ=4, n_freq=8,
                                       qp_lo=1, n_qp=7, seed=23),
    "edge": lambda: make_custom(n_atoms=1, nb_per_atom=5, naux_per_atom=19, nk=(1, 1, 1), n_occ=1, n_freq=7,
                                qp_lo=0, n_qp=1, seed=41),
}
# chi~ and W^c on the real grid; Sigma^c(E) relative to its largest value
TOL_CHI = {"fp64": 1e-10, "fp32": 1e-5, "split_bf16": 1e-5, "split3_bf16": 1e-5, "split_mixed": 1e-5, "split_f16": 1e-5}
TOL_SIG = {"fp64": 1e-10, "fp32": 2e-5, "split_f16": 2e-5}


def _window(s):
    vbm, cbm = s.eig[:, :s.n_occ].max(), s.eig[:, s.n_occ:].min()
    return vbm, cbm, cbm - vbm


def _grid(s):
    n_r = min(12, s.spec.n_freq)
    return n_r, 0.6 * _window(s)[2]


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    L = _lib()
    print(f"\n[gpu contour] case={request.param}", flush=True)
    s = CASES[request.param]()
    o = Oracle(s)
    vbm, cbm, dmin = _window(s)
    E = np.random.default_rng(7).uniform(vbm - 0.45 * dmin, cbm + 0.45 * dmin, (3, s.n_k, s.spec.n_qp))
    return dict(name=request.param, sys=s, o=o, dev=L.device_inputs(s), L=L, E=E)


def _ctx(case, precision):
    s = case["sys"]
    ctx = case["L"].Context.from_system(s, precision=precision)
    ctx.set_real_grid(*_grid(s))
    H = ctx.empty("H")
    ctx.lri_ft(case["dev"]["lri"], s.R, case["dev"]["evec"], H)
    return ctx, H


@pytest.mark.parametrize("precision", list(TOL_CHI))
def test_real_axis_response_and_screening(case, precision):
    s, o, dev = case["sys"], case["o"], case["dev"]
    tol = TOL_CHI[precision]
    ctx, H = _ctx(case, precision)
    n_r, wmax = _grid(s)
    omr, h = contour.real_grid(n_r, wmax)
    n = s.n_aux
    M, chi, W = ctx.empty("M"), ctx.empty_real(), ctx.empty_real()
    ctx.gamma_prepare(dev["V"][0], dev["p"], s.omega_cell)
    for q in sorted({0, 1 % s.n_k, s.n_k - 1}):
        B = o.B(q)
        ctx.build_M(q, 0, H, dev["evec"], M)
        for g in ((False, True) if q == 0 else (False,)):
            ctx.chi0_real(q, M, dev["eig"], chi, apply_gamma=g)
            ctx.screen_real(q, chi, dev["V"][q], W)
            w = W.cpu().numpy().reshape(n_r, n, n)
            refw = o.wc_real(q, omr, B=B, gamma=g)
            ew = relf(w, refw)
            if not g:
                c = chi.cpu().numpy().reshape(n_r, n, n)
                ec = relf(c, o.chi0_real(q, omr, B))
                print(f"  {case['name']} {precision} q={q}: chi~(w_r) {ec:.1e}, W^c(w_r) {ew:.1e}", flush=True)
                assert ec < tol, (q, ec)
            else:
                print(f"  {case['name']} {precision} q=0 with Gamma: W^c(w_r) {ew:.1e}", flush=True)
            assert ew < 10 * tol, (q, g, ew)


@pytest.mark.parametrize("precision", list(TOL_SIG))
def test_sigma_cd_per_q_and_pass(case, precision):
    s, o, dev = case["sys"], case["o"], case["dev"]
    sp = s.spec
    tol = TOL_SIG[precision]
    ctx, H = _ctx(case, precision)
    n_r, wmax = _grid(s)
    omr, h = contour.real_grid(n_r, wmax)
    E = case["E"]
    Ed = torch.from_numpy(E).cuda()
    M, x = ctx.empty("M"), ctx.empty("x")
    chi, W, chir, Wr = ctx.empty("W"), ctx.empty("W"), ctx.empty_real(), ctx.empty_real()
    for q in sorted({1 % s.n_k, s.n_k - 1}):
        B = o.B(q)
        ctx.build_M(q, 0, H, dev["evec"], M)
        ctx.chi0(q, M, dev["eig"], chi)
        ctx.screen(q, chi, dev["V"][q], W)
        ctx.chi0_real(q, M, dev["eig"], chir)
        ctx.screen_real(q, chir, dev["V"][q], Wr)
        ctx.build_M(q, 1, H, dev["evec"], x)
        acc = torch.full((3, s.n_k, sp.n_qp), 0.25, dtype=torch.float64, device="cuda")   # accumulated onto
        ctx.sigma_cd(q, x, W, Wr, dev["eig"], Ed, acc)
        ref = o.sigma_cd_q(q, o.wc(q, B=B, gamma=False), o.wc_real(q, omr, B=B, gamma=False), h, E)
        got = acc.cpu().numpy() - 0.25
        e = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"  {case['name']} {precision} q={q}: Sigma^c(E) rel {e:.1e}", flush=True)
        assert e < tol, (q, e)
    out = torch.full((3, s.n_k, sp.n_qp), 9.0, dtype=torch.float64, device="cuda")   # set, not accumulated
    rc, bad = ctx.sigma_cd_pass(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, Ed, out)
    ref = o.sigma_cd(n_r, wmax, E)
    e = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(np.abs(ref))
    print(f"  {case['name']} {precision}: pass Sigma^c(E) rel {e:.1e} (rc {rc}, NaN {bad})", flush=True)
    assert rc == 0 and bad == 0
    assert e < tol


@pytest.mark.parametrize("var", [7, 8, 9, 10, 13])
def test_sigma_cd_resident_variants(case, var):
    """The FP16 form's resident-tile self-energy kernel (8 and 4 waves per
    workgroup; 13: 8 waves with the frequencies in four sets) on both plane
    sets: the imaginary grid and the real grid, which has item lists of its
    own."""
    s, o, dev = case["sys"], case["o"], case["dev"]
    sp = s.spec
    ctx, H = _ctx(case, "split_f16")
    ctx.set_tiles(4, 1, 8, var)
    n_r, wmax = _grid(s)
    omr, h = contour.real_grid(n_r, wmax)
    E = case["E"]
    Ed = torch.from_numpy(E).cuda()
    q = 1 % s.n_k
    B = o.B(q)
    M, x = ctx.empty("M"), ctx.empty("x")
    chi, W, chir, Wr = ctx.empty("W"), ctx.empty("W"), ctx.empty_real(), ctx.empty_real()
    ctx.build_M(q, 0, H, dev["evec"], M)
    ctx.chi0(q, M, dev["eig"], chi)
    ctx.screen(q, chi, dev["V"][q], W)
    ctx.chi0_real(q, M, dev["eig"], chir)
    ctx.screen_real(q, chir, dev["V"][q], Wr)
    ctx.build_M(q, 1, H, dev["evec"], x)
    acc = torch.zeros((3, s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    ctx.sigma_cd(q, x, W, Wr, dev["eig"], Ed, acc)
    ref = o.sigma_cd_q(q, o.wc(q, B=B, gamma=False), o.wc_real(q, omr, B=B, gamma=False), h, E)
    e = np.max(np.abs(acc.cpu().numpy() - ref)) / np.max(np.abs(ref))
    out = torch.zeros((3, s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    rc, bad = ctx.sigma_cd_pass(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, Ed, out)
    refp = o.sigma_cd(n_r, wmax, E)
    ep = np.max(np.abs(out.cpu().numpy() - refp)) / np.max(np.abs(refp))
    print(f"  {case['name']} variant {var}: q={q} Sigma^c(E) rel {e:.1e}, pass rel {ep:.1e}", flush=True)
    assert e < 2e-5 and ep < 2e-5 and rc == 0 and bad == 0


@pytest.mark.parametrize("precision,tol_mev", [("fp64", 1e-5), ("split_f16", 1.0)])
def test_linearised_qp(case, precision, tol_mev):
    s, o, dev = case["sys"], case["o"], case["dev"]
    sp = s.spec
    ctx, H = _ctx(case, precision)
    n_r, wmax = _grid(s)
    delta = 0.002
    e_qp = torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    z = torch.zeros_like(e_qp)
    S3 = torch.zeros((3, s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    rc, bad = ctx.g0w0_cd(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, dev["e_static"], delta, e_qp, z,
                          sigma3=S3)
    eps = s.eig[:, o.qp]
    E3 = eps[None] + np.array([-delta, 0.0, delta])[:, None, None]
    Sref = o.sigma_cd(n_r, wmax, E3)
    Eref, Zref = contour.qp_linear(Sref[0], Sref[1], Sref[2], delta, eps, s.e_static)
    got_s, got_e, got_z = S3.cpu().numpy(), e_qp.cpu().numpy(), z.cpu().numpy()
    assert np.array_equal(np.isnan(got_s), np.isnan(Sref))
    assert bad == int(np.isnan(Sref).sum())
    assert rc == (3 if bad else 0)
    ok = ~np.isnan(Eref)
    print(f"  {case['name']} {precision}: {ok.sum()} of {ok.size} states evaluated", flush=True)
    if ok.sum():
        de = np.max(np.abs(got_e[ok] - Eref[ok])) * HA_MEV
        dz = np.max(np.abs(got_z[ok] - Zref[ok]))
        print(f"    max|dE| {de:.2e} meV, max|dZ| {dz:.1e}", flush=True)
        assert de < tol_mev and dz < (1e-8 if precision == "fp64" else 1e-3)
    assert np.all(np.isnan(got_e[~ok]))


def test_errors_and_range_warning():
    L = _lib()
    s = make_config(1)
    dev = L.device_inputs(s)
    sp = s.spec
    ctx = L.Context.from_system(s, precision="fp64")
    for bad_n in (3, sp.n_freq + 1):
        with pytest.raises(L.LrigwError) as e:
            ctx.set_real_grid(bad_n, 0.01)
        assert e.value.code == L.LRIGW_ERR_ARG
    vbm, cbm, dmin = _window(s)
    H = ctx.empty("H")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    M, chir = ctx.empty("M"), None
    ctx.set_real_grid(8, 1.01 * dmin)   # reaches the first transition: the response has a pole
    chir = ctx.empty_real()
    ctx.build_M(1, 0, H, dev["evec"], M)
    with pytest.raises(L.LrigwError) as e:
        ctx.chi0_real(1, M, dev["eig"], chir)
    assert e.value.code == L.LRIGW_ERR_ARG
    ctx.set_real_grid(8, 0.5 * dmin)
    # energies below every occupied level: residues from all of them, most beyond the grid
    E = np.full((1, s.n_k, sp.n_qp), s.eig[:, :s.n_occ].min() - 0.01)
    out = torch.zeros((1, s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    rc, bad = ctx.sigma_cd_pass(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell,
                                torch.from_numpy(E).cuda(), out)
    assert rc == L.LRIGW_WARN_CD_RANGE and bad == out.numel()
    assert np.all(np.isnan(out.cpu().numpy()))


def test_si_like_sampled():
    """Si-like cell (N_aux 260, 6x6x6 k, 32 frequencies), default FP16 form:
    one q's contribution at sampled k points against the oracle."""
    L = _lib()
    s = make_config(2)
    sp = s.spec
    dev = L.device_inputs(s)
    o = Oracle(s)
    ctx = L.Context.from_system(s, precision="split_f16")
    n_r, wmax = 16, 0.6 * _window(s)[2]
    ctx.set_real_grid(n_r, wmax)
    omr, h = contour.real_grid(n_r, wmax)
    H = ctx.empty("H")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    vbm, cbm, dmin = _window(s)
    E = np.random.default_rng(3).uniform(vbm - 0.45 * dmin, cbm + 0.45 * dmin, (2, s.n_k, sp.n_qp))
    q = 95
    M, x = ctx.empty("M"), ctx.empty("x")
    chi, W, chir, Wr = ctx.empty("W"), ctx.empty("W"), ctx.empty_real(), ctx.empty_real()
    ctx.build_M(q, 0, H, dev["evec"], M)
    ctx.chi0(q, M, dev["eig"], chi)
    ctx.screen(q, chi, dev["V"][q], W)
    ctx.chi0_real(q, M, dev["eig"], chir)
    ctx.screen_real(q, chir, dev["V"][q], Wr)
    ctx.build_M(q, 1, H, dev["evec"], x)
    acc = torch.zeros((2, s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    ctx.sigma_cd(q, x, W, Wr, dev["eig"], torch.from_numpy(E).cuda(), acc)
    ks = [0, 37, 150]
    B = o.B(q)
    ref = o.sigma_cd_q(q, o.wc(q, B=B, gamma=False), o.wc_real(q, omr, B=B, gamma=False), h, E[:, ks], ks)
    got = acc.cpu().numpy()[:, ks]
    e = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"  si-like q={q}: sampled Sigma^c(E) rel {e:.1e}", flush=True)
    assert e < 2e-5


def test_si_like_against_pade_continuation():
    """Si-like cell, FP16 form: Sigma^c at e_n of the band-edge states from
    contour deformation against the Pade continuation (the library's node
    choice, continued fraction evaluated on the host) of the same path's
    imaginary-axis Sigma^c.  They agree to the continuation's error (0.1 meV
    at most on this cell, against |Sigma^c| up to 20 eV)."""
    L = _lib()
    s = make_config(2)
    sp = s.spec
    dev = L.device_inputs(s)
    ctx = L.Context.from_system(s, precision="split_f16")
    H = ctx.empty("H")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    sig = torch.zeros((s.n_k, sp.n_qp, sp.n_freq), dtype=torch.complex128, device="cuda")
    e = torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    z = torch.zeros_like(e)
    ctx.g0w0(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, dev["e_static"], 16, sig, e, z)
    ctx.set_real_grid(16, 0.6 * _window(s)[2])
    S3 = torch.zeros((3, s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    ecd, zcd = torch.zeros_like(e), torch.zeros_like(e)
    ctx.g0w0_cd(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, dev["e_static"], 0.002, ecd, zcd, sigma3=S3)
    cd = S3.cpu().numpy()[1]
    # the library's own continuation at e_n
    Ed = torch.from_numpy(s.eig[None, :, sp.qp_lo:sp.qp_lo + sp.n_qp].copy()).cuda()
    pv = torch.zeros((1, s.n_k, sp.n_qp), dtype=torch.complex128, device="cuda")
    ctx.pade_eval(sig, 16, Ed, pv)
    pdev = pv.cpu().numpy()[0].real
    sg = sig.cpu().numpy()
    nodes = grids.pade_nodes(sp.n_freq, 16)
    om, _ = grids.frequency_grid(sp.n_freq, sp.x0)
    zn = 1j * om[nodes]
    eps = s.eig[:, sp.qp_lo:sp.qp_lo + sp.n_qp]
    ok = np.isfinite(cd)
    d = []
    for k, n in zip(*np.nonzero(ok)):
        a, _ = continuation.thiele_coeffs(zn, sg[k, n, nodes])
        d.append(abs(continuation.thiele_eval(zn, a, eps[k, n] - s.mu)[0].real - cd[k, n]))
    d = np.array(d) * HA_MEV
    dd = np.abs(pdev[ok] - cd[ok]) * HA_MEV
    print(f"  si-like: {ok.sum()} band-edge states, |Sigma_CD(e) - Sigma_Pade(e)| median {np.median(d):.2f} meV, "
          f"max {d.max():.2f} meV (lrigw_pade_eval: max {dd.max():.2f} meV); |Sigma^c(e)| up to "
          f"{np.abs(cd[ok]).max() * HA_MEV:.0f} meV", flush=True)
    assert ok.sum() > 0 and d.max() < 2.0 and dd.max() < 2.0


# ---- every state: the broadened real grid (W^c at w_r + i eta)
ETA = 0.05


def _broad_grid(s, E):
    # every |E - e_m| lies below this
    top = max(float(E.max() - s.eig.min()), float(s.eig.max() - E.min())) + 0.02
    h = ETA / 4
    n_r = int(np.ceil(top / h)) + 1
    return n_r, (n_r - 1) * h


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("split_f16", 2e-5), ("fp32", 2e-5)])
def test_broadened_pass_every_state(case, precision, tol):
    """Sigma^c at energies across every band (residues far above the first
    transition), whole pass with the broadened grid, against the oracle's
    contour deformation on the same grid."""
    s, o, dev, L = case["sys"], case["o"], case["dev"], case["L"]
    if s.spec.n_freq < 2:
        pytest.skip("n_freq < 2")
    E = np.random.default_rng(8).uniform(s.eig.min() - 0.05, s.eig.max() + 0.05, (2, s.n_k, s.spec.n_qp))
    n_r, wmax = _broad_grid(s, E)
    print(f"  {case['name']} {precision}: broadened grid {n_r} nodes to {wmax:.3f} Ha", flush=True)
    ctx = L.Context.from_system(s, precision=precision)
    ctx.set_real_grid(n_r, wmax, ETA)
    H = ctx.empty("H")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    Ed = torch.from_numpy(np.ascontiguousarray(E)).cuda()
    out = torch.zeros_like(Ed)
    rc, bad = ctx.sigma_cd_pass(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, Ed, out)
    assert rc == L.LRIGW_OK and bad == 0
    got = out.cpu().numpy()
    ref = o.sigma_cd(n_r, wmax, E, eta=ETA)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"    Sigma^c(E) rel. {err:.2e}", flush=True)
    assert np.all(np.isfinite(got)) and err < tol
    ctx.close()


def test_broadened_qp_newton(case):
    """lrigw_qp_cd (three Newton steps, broadened grid) against the oracle's
    Newton steps, every state evaluated (FP64)."""
    s, o, dev, L = case["sys"], case["o"], case["dev"], case["L"]
    if s.spec.n_freq < 2:
        pytest.skip("n_freq < 2")
    # the Newton iterates stay within 0.6 Ha of the band range
    span = np.array([s.eig.min() - 0.6, s.eig.max() + 0.6])
    n_r, wmax = _broad_grid(s, span)
    ctx = L.Context.from_system(s, precision="fp64")
    ctx.set_real_grid(n_r, wmax, ETA)
    H = ctx.empty("H")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    e = torch.zeros((s.n_k, s.spec.n_qp), dtype=torch.float64, device="cuda")
    z = torch.zeros_like(e)
    rc, bad = ctx.qp_cd(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, dev["e_static"], 0.002, 3, e, z)
    assert rc == L.LRIGW_OK and bad == 0
    Eo, Zo, _ = o.qp_cd(n_r, wmax, ETA, 3, delta=0.002)
    # one step, then two more continuing from its energies: the same iterates
    e1, z1 = torch.zeros_like(e), torch.zeros_like(e)
    assert ctx.qp_cd(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, dev["e_static"], 0.002, 1, e1,
                     z1)[0] == L.LRIGW_OK
    assert ctx.qp_cd(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, dev["e_static"], 0.002, 2, e1, z1,
                     warm=True)[0] == L.LRIGW_OK
    assert torch.equal(e1, e) and torch.equal(z1, z)
    d = np.abs(e.cpu().numpy() - Eo) * HA_MEV
    print(f"  {case['name']}: QP by Newton on the broadened grid, max {d.max():.2e} meV from the oracle; "
          f"shifts {np.abs(Eo - s.eig[:, s.spec.qp_lo:s.spec.qp_lo + s.spec.n_qp]).max():.3f} Ha", flush=True)
    assert np.all(np.isfinite(e.cpu().numpy())) and d.max() < 1e-4
    assert np.max(np.abs(z.cpu().numpy() - Zo)) < 1e-8
    ctx.close()
