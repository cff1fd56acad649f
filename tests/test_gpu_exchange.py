"""GPU parity of the exchange self-energy (lrigw_build_M slice 2,
lrigw_sigma_x, lrigw_sigma_x_pass) against the FP64 oracle on the same seeded
inputs, and on the Si-like cell at sampled k points."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.pipeline import Oracle
from synth.systems import make_config, make_custom


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
    # ragged N_aux = 74, non-TRIM 3x1x2 grid (complex V(q))
    "ragged": lambda: make_custom(n_atoms=2, nb_per_atom=7, naux_per_atom=37, nk=(3, 1, 2), n_occ=5, n_freq=10,
                                  qp_lo=2, n_qp=6, seed=17),
    "three_atoms": lambda: make_custom(n_atoms=3, nb_per_atom=6, naux_per_atom=45, nk=(1, 1, 1), n_occ=4, n_freq=8,
                                       qp_lo=1, n_qp=7, seed=23),
    # one occupied band, N_aux below one tile, a single QP band
    "edge": lambda: make_custom(n_atoms=1, nb_per_atom=5, naux_per_atom=19, nk=(1, 1, 1), n_occ=1, n_freq=7,
                                qp_lo=0, n_qp=1, seed=41),
}
# FP64: rounding only; reduced-precision forms: the pairs are FP32 (relative
# 6e-8 per element), the quadratic form is taken in FP64
TOL = {"fp64": (1e-12, 1e-11), "fp32": (2e-6, 1e-6), "split_f16": (2e-6, 1e-6)}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    L = _lib()
    print(f"\n[gpu exchange] case={request.param}", flush=True)
    s = CASES[request.param]()
    return dict(name=request.param, sys=s, o=Oracle(s), dev=L.device_inputs(s), L=L)


@pytest.mark.parametrize("precision", list(TOL))
def test_exchange_per_q_and_pass(case, precision):
    s, o, dev, L = case["sys"], case["o"], case["dev"], case["L"]
    tol_x, tol_s = TOL[precision]
    ctx = L.Context.from_system(s, precision=precision)
    sp = s.spec
    H = ctx.empty("H")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    xo = ctx.empty("xo")
    sx = torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    for q in sorted({0, 1 % s.n_k, s.n_k - 1}):
        ctx.build_M(q, 2, H, dev["evec"], xo)
        X = xo.cpu().numpy().reshape(s.n_k, sp.n_qp, s.n_occ, s.n_aux)
        ref = np.transpose(o.x_occ(q), (0, 2, 3, 1))
        assert relf(X, ref) < tol_x, (q, relf(X, ref))
        sx.zero_()
        ctx.sigma_x(q, xo, dev["V"][q], sx)
        refq = o.sigma_x_q(q)
        e = relf(sx.cpu().numpy(), refq)
        print(f"  {case['name']} {precision} q={q}: pairs {relf(X, ref):.1e}, Sigma^x {e:.1e}", flush=True)
        assert e < tol_s, (q, e)
    allq = torch.full((s.n_k, sp.n_qp), 7.0, dtype=torch.float64, device="cuda")   # overwritten, not accumulated
    ctx.sigma_x_pass(H, dev["evec"], dev["V"], allq)
    ref = o.sigma_x()
    e = relf(allq.cpu().numpy(), ref)
    print(f"  {case['name']} {precision}: pass Sigma^x rel {e:.1e}", flush=True)
    assert e < tol_s
    assert np.all(allq.cpu().numpy() < 0.0)


def test_exchange_si_like_sampled():
    """Si-like cell (N_aux 260, 6x6x6 k): the whole pass in the default FP16 form
    is negative and time-reversal symmetric everywhere; two q's contributions
    at sampled k points match the oracle."""
    L = _lib()
    s = make_config(2)
    sp = s.spec
    dev = L.device_inputs(s)
    o = Oracle(s)
    ctx = L.Context.from_system(s, precision="split_f16")
    H = ctx.empty("H")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    allq = torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    ctx.sigma_x_pass(H, dev["evec"], dev["V"], allq)
    a = allq.cpu().numpy()
    assert np.all(a < 0.0)
    assert np.max(np.abs(a - a[o.minus])) < 1e-9 * np.max(np.abs(a))
    xo = ctx.empty("xo")
    ks = [0, 37, 150]
    for q in (0, 95):
        ctx.build_M(q, 2, H, dev["evec"], xo)
        sx = torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
        ctx.sigma_x(q, xo, dev["V"][q], sx)
        got = sx.cpu().numpy()[ks]
        ref = o.sigma_x_q(q, ks)
        print(f"  si-like q={q}: sampled Sigma^x rel {relf(got, ref):.1e}", flush=True)
        assert relf(got, ref) < 1e-6
