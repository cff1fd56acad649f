"""Throughput of the imaginary-frequency LRI-G0W0 path on one MI355X.

One step = the whole path over the Si-like 2-atom cell (N_b = 78, N_aux = 260,
6x6x6 k grid, 4 occupied bands, 32 frequencies): LRI Bloch/half transform,
then for every q the response build, chi0, screening to W^c and the Sigma^c
contribution of every (k, QP band), then Pade + QP.  value = (q, w) pairs per
second = N_q * N_w * steps / seconds.

Prints one JSON line.  The FP64 oracle is timed on a bounded sample on the
host cores (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X dense matrix peaks (the split forms run BF16 or FP16 MFMA)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "split_bf16": 2500.0, "split3_bf16": 2500.0, "split_mixed": 2500.0,
               "split_f16": 2500.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "split_bf16": "bf16", "split3_bf16": "bf16", "split_mixed": "bf16",
         "split_f16": "f16"}
STAGES = ("lri_ft", "build_M", "chi0", "chi0_split", "chi0_mfma", "screen", "sigma_c", "sigma_split", "sigma_mfma", "qp")
HA_MEV = 27211.386


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--precision", default="split_f16", choices=list(PEAK_TFLOPS))
    ap.add_argument("--no-tune", action="store_true", help="skip the response-kernel tile autotuner")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain FP64 path")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the exchange, coefficient-fit and contour-deformation legs (kernel profiles of the metric)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--n-par", type=int, default=16)
    ap.add_argument("--cd-eta", type=float, default=0.05, help="broadening (Ha) of the cd_every_state workload")
    ap.add_argument("--workload", default="cell", choices=["cell", "batched", "surrogate", "cd_every_state"],
                    help="cell: one cell (--config); batched: the six uneven cells of config 3 in one captured graph; "
                         "surrogate: the learned frequency surrogate on the 8-atom cell against its exact pass; "
                         "cd_every_state: every QP state of the Si-like cell by contour deformation on the "
                         "broadened real grid (Newton steps), against the Pade roots")
    return ap.parse_args()


class Run:
    """All device state of one precision form on one cell."""

    def __init__(self, L, sysm, dev, precision, n_par):
        import torch
        self.torch = torch
        self.sysm, self.dev, self.n_par = sysm, dev, n_par
        self.ctx = L.Context.from_system(sysm, precision=precision)
        sp = sysm.spec
        self.H = self.ctx.empty("H")
        self.sigma = torch.zeros((sysm.n_k, sp.n_qp, sp.n_freq), dtype=torch.complex128, device="cuda")
        self.e_qp = torch.zeros((sysm.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
        self.z = torch.zeros_like(self.e_qp)

    def step(self):
        s, d = self.sysm, self.dev
        self.ctx.lri_ft(d["lri"], s.R, d["evec"], self.H)
        return self.ctx.g0w0(self.H, d["evec"], d["eig"], d["V"], d["p"], s.omega_cell, d["e_static"], self.n_par,
                             self.sigma, self.e_qp, self.z)

    def timed(self, steps, warmup):
        """Time `steps` passes with HIP events around the two MFMA kernel stages
        only (their launches over the timed region give the roofline figures),
        then record every stage over one further, untimed pass for the stage
        breakdown.  Returns (seconds, kernel stages, breakdown of one pass)."""
        torch = self.torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        self.ctx.reset_timing()
        self.ctx.set_timing(True, kernels_only=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kern = self._stages()
        self.ctx.reset_timing()
        self.ctx.set_timing(True)
        self.step()
        torch.cuda.synchronize()
        breakdown = self._stages()
        self.ctx.set_timing(False)
        return dt, kern, breakdown

    def _stages(self):
        out = {}
        for name in STAGES:
            ms, n = self.ctx.stage_ms(name)
            if n:
                out[name] = (ms, n)
        return out


def algorithmic_flops(sysm):
    """Real flops of each MFMA kernel stage for one q (all frequencies):
    chi0: 8 N_aux^2 K per (q, w) pair, K = N_k N_occ N_unocc (full Hermitian
    count); Sigma^c: 8 N_aux^2 N_k N_qp N_bands per pair.  One q is one launch
    unless its K splits run in batches (one launch per batch)."""
    sp = sysm.spec
    n_aux, n_k, nw = sysm.n_aux, sysm.n_k, sp.n_freq
    K = n_k * sp.n_occ * (sp.n_bands - sp.n_occ)
    return {"chi0_mfma": 8.0 * n_aux * n_aux * K * nw,
            "sigma_mfma": 8.0 * n_aux * n_aux * n_k * sp.n_qp * sp.n_bands * nw}


def traffic_for(kernel, precision, config):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    r = rec.get(f"{kernel}:{precision}:c{config}")
    if not r:
        return None
    src = os.path.join(ROOT, "paper_2011_01400_amd", "csrc", r["source"])
    try:
        with open(src, "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None
    return r["bytes_per_launch"] if h == r["source_sha256_16"] else None


def roofline(sysm, stages, precision, config, n_q):
    """Dominant MFMA kernel: algorithmic flops per launch / average launch
    time, over the n_q q of the recorded passes (flops per launch = their
    flops over the launches, so K splits run in batches count right)."""
    flops = algorithmic_flops(sysm)
    best = None
    for name, f in flops.items():
        if name not in stages:
            continue
        ms, n = stages[name]
        if best is None or ms > best[1]:
            best = (name, ms, n, f)
    name, ms, n, f = best
    fl = f * n_q / n
    achieved = fl / (ms / n / 1e3) / 1e12
    peak = PEAK_TFLOPS[precision]
    return {"bound": "mfma", "kernel": name, "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic_for(name, precision, config),
            "avg_launch_ms": round(ms / n, 4), "launches_per_q": round(n / n_q, 3), "flops_per_launch": fl}


def mfma_sustained():
    """The sustained dense FP16 matrix-core rate of this device, from the
    calibration program built beside the library (eight independent
    16x16x32 FP16 MFMA chains per wave on every SIMD, zero and then random
    operands, with the mean shader clock of each), run in a child process
    after the timed steps.  With random operands the clock drops below its
    peak, so the published peak is not reachable with the data the kernels
    see; the fractions against this rate are reported beside those against
    the published peak."""
    exe = os.path.join(ROOT, "paper_2011_01400_amd", "mfma_rate")
    if not os.path.exists(exe):
        return {"error": "calibration program not built"}
    try:
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        d = json.loads(r.stdout.strip().splitlines()[-1])
    except (subprocess.TimeoutExpired, ValueError, IndexError) as e:
        return {"error": str(e)}
    if r.returncode != 0 and "error" not in d:
        d["error"] = f"exit status {r.returncode}"
    return d


def other_kernel(sysm, stages, precision, rl, n_q):
    """The same figures for the other MFMA kernel."""
    flops = algorithmic_flops(sysm)
    out = {}
    for name, f in flops.items():
        if name == rl["kernel"] or name not in stages:
            continue
        ms, n = stages[name]
        a = f * n_q / (ms / 1e3) / 1e12
        out[name] = {"achieved": round(a, 2), "peak": PEAK_TFLOPS[precision], "frac": round(a / PEAK_TFLOPS[precision], 4),
                     "avg_launch_ms": round(ms / n, 4), "launches_per_q": round(n / n_q, 3)}
    return out


def sigma_x_timing(run, sysm, dev, reps=3):
    """Exchange self-energy over every q (lrigw_sigma_x_pass: the exchange
    pairs of each q and their FP64 quadratic form with V(q)), outside the timed
    region of the metric.  Algorithmic flops per pass: 8 N_aux^2 per pair,
    N_k N_qp N_occ pairs per q, on the FP64 MFMA GEMM."""
    torch = run.torch
    sp = sysm.spec
    sx = torch.zeros((sysm.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    run.ctx.sigma_x_pass(run.H, dev["evec"], dev["V"], sx)   # first call allocates its workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run.ctx.sigma_x_pass(run.H, dev["evec"], dev["V"], sx)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    flops = 8.0 * sysm.n_aux ** 2 * sysm.n_k * sp.n_qp * sp.n_occ * sysm.n_k
    a = flops / dt / 1e12
    v = sx.cpu().numpy()
    return {"ms_per_pass": round(dt * 1e3, 3), "bound": "mfma", "achieved": round(a, 2), "peak": PEAK_TFLOPS["fp64"],
            "unit": "TFLOP/s", "frac": round(a / PEAK_TFLOPS["fp64"], 4), "flops_per_pass": flops,
            "range_ha": [round(float(v.min()), 6), round(float(v.max()), 6)]}


def contour_timing(run, sysm, dev, n_r=16, reps=1):
    """Quasiparticle energies by contour deformation (lrigw_g0w0_cd) on the
    same cell and form, outside the timed region of the metric: per q the
    response and W^c on the imaginary grid and on n_r real frequencies up to
    0.6 of the smallest transition energy, Sigma^c at e_n and e_n -+ 2 mHa,
    then the linearised QP step.  States whose residue frequencies pass the
    real grid (those far from the band edges) come back as NaN."""
    torch = run.torch
    sp = sysm.spec
    occ, un = sysm.eig[:, :sysm.n_occ], sysm.eig[:, sysm.n_occ:]
    dmin = float(un.min() - occ.max())
    wmax = 0.6 * dmin
    run.ctx.set_real_grid(n_r, wmax)
    e = torch.zeros((sysm.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    z = torch.zeros_like(e)
    S3 = torch.zeros((3, sysm.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    args = (run.H, dev["evec"], dev["eig"], dev["V"], dev["p"], sysm.omega_cell, dev["e_static"], 0.002, e, z, S3)
    run.ctx.g0w0_cd(*args)   # first call allocates its workspaces
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        rc, bad = run.ctx.g0w0_cd(*args)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ev = e.cpu().numpy()
    ok = np.isfinite(ev)
    # Sigma^c(e_n) against the Pade continuation of the timed steps' Sigma^c(i w)
    # (lrigw_pade_eval), on the states contour deformation evaluated
    Ee = torch.from_numpy(np.ascontiguousarray(sysm.eig[None, :, sp.qp_lo:sp.qp_lo + sp.n_qp])).cuda()
    pv = torch.zeros((1, sysm.n_k, sp.n_qp), dtype=torch.complex128, device="cuda")
    run.ctx.pade_eval(run.sigma, run.n_par, Ee, pv)
    s0 = S3.cpu().numpy()[1]
    m = np.isfinite(s0)
    dp = np.abs(pv.cpu().numpy()[0].real[m] - s0[m]) * 27211.386
    return {"ms_per_pass": round(dt * 1e3, 3), "n_real": n_r, "omega_max_ha": round(wmax, 6),
            "sigma_vs_pade_mev": {"states": int(m.sum()), "median": round(float(np.median(dp)), 4),
                                  "max": round(float(dp.max()), 4)} if m.any() else None,
            "pairs_per_s": round(sysm.n_k * (sp.n_freq + n_r) / dt, 1),
            "states_evaluated": int(ok.sum()), "states": int(ok.size), "nan_outputs": int(bad),
            "z_range": [round(float(z.cpu().numpy()[ok].min()), 4), round(float(z.cpu().numpy()[ok].max()), 4)]
            if ok.any() else None}


def cd_every_state(args, eta=0.05, max_iter=8, tol_mev=0.1, delta=0.002):
    """Every QP state of the Si-like cell by contour deformation: W^c at
    w_r + i eta on a uniform real grid of step eta/4 reaching every residue
    of energies within 0.6 Ha of the band range, Newton steps on the QP
    equation with Re Sigma^c(E) (lrigw_qp_cd, one step per call continuing
    from the previous energies, each step one pass over every q) until no
    state moves by more than tol_mev (at most max_iter steps), against the
    roots of the Pade continuation of the same form's Sigma^c(i w)
    (lrigw_g0w0) and, when on file, the oracle's Pade roots."""
    import torch
    from paper_2011_01400_amd import lrigw as L
    from synth.systems import make_config
    L.load()
    t_start = time.perf_counter()
    s = make_config(2)
    sp = s.spec
    dev = L.device_inputs(s)
    run = Run(L, s, dev, args.precision, args.n_par)
    run.ctx.lri_ft(dev["lri"], s.R, dev["evec"], run.H)
    tuned = run.ctx.tune(run.H, dev["evec"], dev["eig"])
    run.step()
    torch.cuda.synchronize()
    e_pade, z_pade = run.e_qp.cpu().numpy(), run.z.cpu().numpy()
    lo, hi = float(s.eig.min()) - 0.6, float(s.eig.max()) + 0.6
    h = eta / 4.0
    top = max(hi - float(s.eig.min()), float(s.eig.max()) - lo) + 0.02
    n_r = int(np.ceil(top / h)) + 1
    run.ctx.set_real_grid(n_r, (n_r - 1) * h, eta)
    print(f"# bench cd_every_state: broadened grid of {n_r} nodes to {(n_r - 1) * h:.3f} Ha (eta {eta} Ha)",
          file=sys.stderr, flush=True)
    e = torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    z = torch.zeros_like(e)
    S3 = torch.zeros((3, s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    steps, times = [], []
    prev = s.eig[:, sp.qp_lo:sp.qp_lo + sp.n_qp].copy()
    rc, bad = 0, 0
    for it in range(max_iter):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, bad = run.ctx.qp_cd(run.H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, dev["e_static"],
                                delta, 1, e, z, sigma3=S3, warm=it > 0)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        ev = e.cpu().numpy()
        st = np.abs(ev - prev) * HA_MEV
        prev = ev.copy()
        fin = np.isfinite(st)
        steps.append((float(np.median(st[fin])) if fin.any() else None, float(st[fin].max()) if fin.any() else None,
                      int((~np.isfinite(ev)).sum())))
        print(f"# bench cd_every_state: Newton step {it + 1}: {times[-1]:.1f} s, |step| median {steps[-1][0]:.3f} "
              f"max {steps[-1][1]:.3f} meV, {steps[-1][2]} states off the grid", file=sys.stderr, flush=True)
        if fin.all() and st.max() <= tol_mev:
            break
    ev, zv = e.cpu().numpy(), z.cpu().numpy()
    ok = np.isfinite(ev)
    d = np.abs(ev - e_pade) * HA_MEV
    reg = ok & (z_pade >= 0.5) & (z_pade <= 1.0) & (zv >= 0.5) & (zv <= 1.0)
    dt = float(np.sum(times))
    out = {"metric": "contour-deformation QP states per second", "value": round(float(ok.sum()) / dt, 2),
           "unit": "states/s", "n_gpus": 1, "higher_is_better": True, "dtype": DTYPE[args.precision],
           "data": "synthetic",
           "config": {"workload": f"Si-like 2-atom cell: N_aux={s.n_aux}, k grid {'x'.join(map(str, sp.nk))}, every "
                                  f"QP state; broadened real grid eta={eta} Ha, step eta/4, {n_r} nodes; Newton steps "
                                  f"(delta {delta} Ha) until no state moves by more than {tol_mev} meV",
                      "precision_form": args.precision},
           "seconds": round(dt, 2), "seconds_per_newton_pass": round(dt / len(times), 2), "rc": int(rc),
           "newton_steps": len(times),
           "step_mev_median_max_offgrid": [[None if v is None else round(v, 4) for v in st[:2]] + [st[2]] for st in steps],
           "states_evaluated": int(ok.sum()), "states": int(ok.size), "nan_outputs": int(bad),
           "vs_pade_mev": {"all_median": round(float(np.median(d[ok])), 3), "all_max": round(float(d[ok].max()), 3),
                           "quasiparticle_like_states": int(reg.sum()),
                           "quasiparticle_like_median": round(float(np.median(d[reg])), 3) if reg.any() else None,
                           "quasiparticle_like_max": round(float(d[reg].max()), 3) if reg.any() else None},
           "z_range": [round(float(zv[ok].min()), 4), round(float(zv[ok].max()), 4)] if ok.any() else None,
           "tuned": list(tuned), "wall_s": round(time.perf_counter() - t_start, 1)}
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "c2_qp.npz")
    if os.path.exists(gold):
        g = np.load(gold, allow_pickle=False)
        do = np.abs(ev - g["E"]) * HA_MEV
        out["vs_oracle_pade_mev"] = {"median": round(float(np.median(do[ok])), 3), "max": round(float(do[ok].max()), 3)}
    print(json.dumps(out))


def lri_fit_timing(run, sysm, reps=2):
    """Two-centre coefficient fit (lrigw_lri_fit) at the Si-like cell's shape:
    every off-site pair (I, J(R)) of its 2 atoms and 125 lattice vectors,
    n = 2 x 130 auxiliary functions, 130 kept, 39 x 39 products, on seeded
    synthetic SPD Coulomb blocks.  Algorithmic FP64 flops per pair: the
    Cholesky factor (n^3/3) and two triangular solves (2 n^2 nrhs)."""
    torch = run.torch
    n_at, n_r = sysm.spec.n_atoms, int(sysm.R.shape[0])
    nb = sysm.n_b // n_at
    na = sysm.n_aux // n_at
    batch, n, keep, nrhs = n_at * n_at * n_r, 2 * na, na, nb * nb
    g = torch.Generator(device="cuda").manual_seed(2011)
    A = torch.randn((batch, n, n), generator=g, dtype=torch.float64, device="cuda") / n ** 0.5
    V = torch.bmm(A, A.transpose(1, 2).contiguous()) + 0.5 * torch.eye(n, dtype=torch.float64, device="cuda")
    del A
    T = torch.randn((batch, n, nrhs), generator=g, dtype=torch.float64, device="cuda")
    C = torch.empty((batch, keep, nrhs), dtype=torch.float64, device="cuda")
    run.ctx.lri_fit(V, T, keep, C)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run.ctx.lri_fit(V, T, keep, C)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    flops = batch * (n ** 3 / 3.0 + 2.0 * n * n * nrhs)
    a = flops / dt / 1e12
    del V, T, C
    return {"ms": round(dt * 1e3, 3), "pairs": batch, "n": n, "kept": keep, "products": nrhs, "bound": "mfma",
            "achieved": round(a, 2), "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s", "frac": round(a / PEAK_TFLOPS["fp64"], 4),
            "flops": flops}


def cpu_baseline(sysm):
    """FP64 oracle as it stands on a bounded sample of the same workload: one q
    (q = 1), all N_w frequencies, all k points, through the oracle's own
    functions (triples, chi0, screening, pair weights, Sigma^c).  cores: the
    host threads this process may run on (its affinity mask), which NumPy's
    BLAS uses."""
    from oracle.pipeline import Oracle
    from oracle import screening, selfenergy, response
    cores = len(os.sched_getaffinity(0))
    o = Oracle(sysm)
    s = sysm
    q = 1
    ks = list(range(0, s.n_k, 1))
    scale = s.n_k / len(ks)
    t0 = time.perf_counter()
    B = o.B(q)
    t_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    chi = response.chi0_trs(B, s.eig, o.kpq, q, s.n_occ, o.omega)
    t_chi = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, Wc = screening.screen(chi, s.V[q])
    t_scr = time.perf_counter() - t0
    t0 = time.perf_counter()
    x = o.x(q, ks)
    t_x = time.perf_counter() - t0
    t0 = time.perf_counter()
    X = selfenergy.pair_weights(x, Wc)
    selfenergy.sigma_c_q(X, s.eig, o.kmq[ks], q, s.mu, o.omega, o.weight, s.n_k)
    t_X = time.perf_counter() - t0
    nw = len(o.omega)
    per_q = scale * (t_b + t_chi + t_x + t_X) + t_scr
    total = t_b + t_chi + t_scr + t_x + t_X
    return {"value": round(nw / per_q, 4), "unit": "(q,w)-pairs/s", "cores": int(cores), "kind": "oracle",
            "sample": f"one q (q=1) of {s.n_k}, all {nw} frequencies, all {len(ks)} k points: {nw} of "
                      f"{s.n_k * nw} (q,w) pairs; {total:.1f} s of CPU work"}


def qp_against_oracle(sysm, config, e_form, e_plain):
    """QP energies of the timed form (and of the plain FP64 path) against the
    FP64 oracle's whole pass over the same seeded cell, per state, when that
    pass is on file (tests/golden/c2_qp.npz, written by an oracle-only script)."""
    path = os.path.join(ROOT, "tests", "golden", f"c{config}_qp.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    if int(g["seed"]) != sysm.seed:
        return None
    E, Z = g["E"], g["Z"]
    reg = (Z >= 0.5) & (Z <= 1.0)   # quasiparticle-like in the oracle's pass
    out = {"states": int(E.size), "quasiparticle_like_states": int(reg.sum())}
    for name, e in (("form", e_form), ("plain_fp64", e_plain)):
        if e is None:
            continue
        d = np.abs(e - E) * HA_MEV
        out[name] = {"max_mev": round(float(d.max()), 4), "median_mev": round(float(np.median(d)), 5),
                     "within_1_mev": bool(d.max() <= 1.0), "states_over_1_mev": int((d > 1.0).sum()),
                     "max_mev_quasiparticle_like": round(float(d[reg].max()), 4)}
    return out


def batched(args):
    """Six uneven Si-like cells (2 to 8 atoms) in one captured hipGraph: value = total
    (q, w) pairs of all cells per second; compared with the same cells run one
    after the other through lrigw_g0w0."""
    import torch
    from paper_2011_01400_amd import lrigw as L
    from synth.systems import all_cells
    L.load()
    cells = all_cells(3)
    stream = torch.cuda.Stream()
    items, runs = [], []
    pairs = 0
    with torch.cuda.stream(stream):
        for s in cells:
            dev = L.device_inputs(s)
            r = Run(L, s, dev, args.precision, args.n_par)
            r.ctx.lri_ft(dev["lri"], s.R, dev["evec"], r.H)
            runs.append(r)
            items.append(dict(ctx=r.ctx, H=r.H, evec=dev["evec"], eig=dev["eig"], V=dev["V"], p=dev["p"],
                              omega_cell=s.omega_cell, e_static=dev["e_static"], n_par=args.n_par, sigma=r.sigma,
                              e_qp=r.e_qp, z=r.z))
            pairs += s.n_k * s.spec.n_freq
            print(f"# bench: cell {s.spec.n_atoms} atoms, N_aux {s.n_aux}, {s.n_k} k ready", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    b = L.Batch(items, autotune=not args.no_tune, stream=stream)
    for _ in range(args.warmup):
        b.run()
    b.status()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    st = b.status()
    dt = time.perf_counter() - t0
    value = pairs * args.steps / dt
    print(f"# bench: batched {value:.1f} pairs/s", file=sys.stderr, flush=True)
    # the same cells one after the other, no graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in runs:
        r.ctx.g0w0(r.H, r.dev["evec"], r.dev["eig"], r.dev["V"], r.dev["p"], r.sysm.omega_cell, r.dev["e_static"],
                   args.n_par, r.sigma, r.e_qp, r.z)
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    out = {"metric": "chi0+Sigma^c (q,w)-pairs/s", "value": round(value, 2), "unit": "(q,w)-pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision],
           "data": "synthetic",
           "config": {"workload": "six uneven Si-like cells: " + ", ".join(
               f"{s.spec.n_atoms} atoms/N_aux {s.n_aux}/{'x'.join(map(str, s.spec.nk))} k" for s in cells)
               + f", {cells[0].spec.n_freq} frequencies, one captured hipGraph", "precision_form": args.precision,
               "pairs_per_step": pairs},
           "graph_nodes": b.graph_nodes(), "status": st,
           "tuning": [b.tuning(i) for i in range(len(cells))],
           "sequential_uncaptured": {"value": round(pairs / dt_seq, 2), "ms": round(dt_seq * 1e3, 3)},
           "speedup_vs_sequential": round(value / (pairs / dt_seq), 3)}
    print(json.dumps(out))


def kernel_rank(omega, d_lo, d_hi, rel=1e-6):
    """Numerical rank of the transition kernel 2D/(D^2 + w^2) over the
    transition window on the frequency grid: singular values of the
    [256 log-spaced D][N_w] matrix above rel times the largest."""
    D = d_lo * (d_hi / d_lo) ** (np.arange(256) / 255.0)
    G = 2.0 * D[:, None] / (D[:, None] ** 2 + np.asarray(omega)[None, :] ** 2)
    s = np.linalg.svd(G, compute_uv=False)
    return int((s > rel * s[0]).sum())


def surrogate_leg(args):
    """Learned frequency surrogate on the 8-atom cell (N_aux 1040, 4x4x4 k,
    40 frequencies): rank-48 projection, network 3 x 256, anchors = the
    numerical rank of the transition kernel at 1e-6 (plus the held-out index),
    trained on 13 q of each of 4 further seeded cells of the same shape
    (2080 (q, w) samples), judged on the workload cell against its exact pass
    in the same precision form (the method without the surrogate): time,
    share of q that keep the prediction, frequencies computed exactly, QP
    energies against the exact pass; the same with the network's output
    switched off (the interpolation rule alone)."""
    import torch
    from paper_2011_01400_amd import lrigw as L
    from synth.systems import (CONFIGS, eigenvalues_of, make_config, make_system, surrogate_init, surrogate_order,
                               surrogate_start, transition_window, window_of)
    L.load()
    t_start = time.perf_counter()
    cfg = 4
    print("# bench surrogate: generating the 8-atom cell", file=sys.stderr, flush=True)
    s = make_config(cfg)
    sp = s.spec
    rank, hidden = 48, 256
    # the training cells (seeds 1000 config + 1..4), one at a time: their
    # transition windows first (eigenvalues only), then the rows
    train_seeds = [1000 * cfg + 1 + i for i in range(4)]
    wins = [transition_window(s)] + [window_of(eigenvalues_of(CONFIGS[cfg][0], sd), sp.n_occ) for sd in train_seeds]
    lo, hi = min(w[0] for w in wins), max(w[1] for w in wins)
    ctx = L.Context.from_system(s, precision=args.precision)
    omega = ctx.grids()[0].cpu().numpy()
    n_anchor = min(16, kernel_rank(omega, lo, hi))
    n_out = sp.n_freq - n_anchor
    qs_train = [1 + (i * (s.n_k - 1)) // 13 for i in range(13)]
    th = surrogate_init(n_anchor, hidden, n_out, 41, out_scale=0.01)
    sg = L.Surrogate(ctx, torch.from_numpy(th).cuda(),
                     torch.from_numpy(surrogate_start(s.n_aux, rank, 2)).cuda(), rank=rank, n_anchor=n_anchor,
                     hidden=hidden, d_lo=lo, d_hi=hi, row_capacity=len(train) * len(qs_train) * rank * rank)
    for i, sd in enumerate(train_seeds):
        print(f"# bench surrogate: generating training cell seed {sd}", file=sys.stderr, flush=True)
        c = make_system(CONFIGS[cfg][0], sd)
        cx = L.Context.from_system(c, precision=args.precision)
        dv = L.device_inputs(c)
        H = cx.empty("H")
        cx.lri_ft(dv["lri"], c.R, dv["evec"], H)
        M, chi = cx.empty("M"), cx.empty("W")
        for q in qs_train:
            cx.build_M(q, 0, H, dv["evec"], M)
            cx.chi0(q, M, dv["eig"], chi)
            sg.add(cx, chi)
        cx.close()
        del dv, H, M, chi, c
        torch.cuda.empty_cache()
        print(f"# bench surrogate: training cell {i + 1} added ({sg.n_rows()} rows)", file=sys.stderr, flush=True)
    n_rows = sg.n_rows()
    batch = 512
    t0 = time.perf_counter()
    hist = []
    for lr, steps, seed in ((1e-3, 3000, 7), (3e-4, 1500, 8)):
        order = torch.from_numpy(surrogate_order(n_rows, steps * batch, seed)).cuda()
        h = torch.zeros(steps, dtype=torch.float32, device="cuda")
        sg.train(steps, batch, lr, order, h)
        hist.append(h.cpu().numpy())
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    h = np.concatenate(hist)
    x, y = sg.rows()
    r_rule = float(torch.sqrt((y ** 2).mean()))
    r_net = float(torch.sqrt(((sg.forward(x) - y) ** 2).mean()))
    trained = sg.params().clone()
    print(f"# bench surrogate: trained {len(h)} steps in {t_train:.1f} s, loss {h[:20].mean():.3e} -> "
          f"{h[-100:].mean():.3e}; training-series rms rule {r_rule:.3e} network {r_net:.3e}",
          file=sys.stderr, flush=True)

    dev = L.device_inputs(s)
    run = Run(L, s, dev, args.precision, args.n_par)
    run.ctx.close()
    run.ctx = ctx
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], run.H)
    tuned = ctx.tune(run.H, dev["evec"], dev["eig"])
    pairs = s.n_k * sp.n_freq

    def timed_pass():
        run.step()
        torch.cuda.synchronize()
        t = time.perf_counter()
        run.step()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    ctx.set_surrogate(None)
    dt_exact = timed_pass()
    e_exact = run.e_qp.cpu().numpy().copy()
    print(f"# bench surrogate: exact pass {dt_exact * 1e3:.0f} ms", file=sys.stderr, flush=True)
    legs = []
    for name, params in (("network", trained), ("rule", torch.zeros_like(trained))):
        sg.params(set_to=params)
        for thr in (1e-5, 3e-5, 1e-4):
            ctx.set_surrogate(sg, thr)
            sg.reset_stats()
            dt = timed_pass()
            n_calls, n_fb, errs = sg.stats(4 * s.n_k)
            d = np.abs(run.e_qp.cpu().numpy() - e_exact) * HA_MEV
            # the two timed_pass steps each call the surrogate once per q
            per_pass_fb = n_fb / 2.0
            kept = s.n_k - per_pass_fb
            exact_planes = kept * (n_anchor + 1) + per_pass_fb * sp.n_freq
            legs.append({"params": name, "threshold": thr, "ms_per_pass": round(dt * 1e3, 1),
                         "pairs_per_s": round(pairs / dt, 1), "speedup_vs_exact": round(dt_exact / dt, 3),
                         "q_keeping_prediction": f"{kept:.0f} of {s.n_k}",
                         "exact_frequency_planes": f"{exact_planes:.0f} of {pairs}",
                         "heldout_error_median": float(np.median(errs)) if errs else None,
                         "heldout_error_max": float(np.max(errs)) if errs else None,
                         "qp_max_err_mev_vs_exact": round(float(d.max()), 4),
                         "qp_median_err_mev_vs_exact": round(float(np.median(d)), 5),
                         "within_1_mev": bool(d.max() <= 1.0)})
            print(f"# bench surrogate: {legs[-1]}", file=sys.stderr, flush=True)
    ctx.set_surrogate(None)
    ok = [g for g in legs if g["params"] == "network" and g["within_1_mev"]]
    best = max(ok, key=lambda g: g["pairs_per_s"]) if ok else None
    out = {"metric": "chi0+Sigma^c (q,w)-pairs/s", "value": best["pairs_per_s"] if best else round(pairs / dt_exact, 1),
           "unit": "(q,w)-pairs/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": best["ms_per_pass"] if best else round(dt_exact * 1e3, 1), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision], "data": "synthetic",
           "config": {"workload": f"8-atom cell: N_b={s.n_b}, N_aux={s.n_aux}, k grid {'x'.join(map(str, sp.nk))}, "
                                  f"N_occ={sp.n_occ}, {sp.n_bands} bands, {sp.n_freq} frequencies; learned surrogate, "
                                  f"rank {rank}, network 3x{hidden}, {n_anchor} anchors + 1 held-out",
                      "precision_form": args.precision, "pairs_per_step": pairs},
           "exact_pass": {"ms": round(dt_exact * 1e3, 1), "pairs_per_s": round(pairs / dt_exact, 1), "tuned": tuned},
           "training": {"cells": 4, "seeds": train_seeds, "q_per_cell": len(qs_train), "samples": 4 * len(qs_train) * sp.n_freq,
                        "rows": n_rows, "steps": int(len(h)), "seconds": round(t_train, 1),
                        "loss_first": float(h[:20].mean()), "loss_last": float(h[-100:].mean()),
                        "series_rms_rule": r_rule, "series_rms_network": r_net},
           "transition_window_ha": [round(lo, 4), round(hi, 4)], "kernel_rank_1e-6": kernel_rank(omega, lo, hi),
           "legs": legs, "chosen": best, "wall_s": round(time.perf_counter() - t_start, 1)}
    sg.close()
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is described in DESIGN.md",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "batched":
        batched(args)
        return
    if args.workload == "surrogate":
        surrogate_leg(args)
        return
    if args.workload == "cd_every_state":
        cd_every_state(args, eta=args.cd_eta)
        return
    import torch
    from paper_2011_01400_amd import lrigw as L
    from synth.systems import make_config
    L.load()
    sysm = make_config(args.config)
    dev = L.device_inputs(sysm)
    sp = sysm.spec
    pairs = sysm.n_k * sp.n_freq

    run = Run(L, sysm, dev, args.precision, args.n_par)
    tuned = None
    if not args.no_tune:
        run.ctx.lri_ft(dev["lri"], sysm.R, dev["evec"], run.H)
        nw, sp_, sv, ms = run.ctx.tune(run.H, dev["evec"], dev["eig"])
        tuned = {"chi0_freq_per_workgroup": nw, "chi0_k_splits": sp_, "sigma_variant": sv, "chi0_ms_one_q": round(ms, 3)}
        print(f"# bench: tuned chi0 tiles {tuned}", file=sys.stderr, flush=True)
    print(f"# bench: config {args.config} precision {args.precision}: warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    dt, kern, stages = run.timed(args.steps, args.warmup)
    value = pairs * args.steps / dt
    e_form = run.e_qp.cpu().numpy()
    print(f"# bench: {value:.1f} pairs/s, {dt / args.steps * 1e3:.1f} ms/step", file=sys.stderr, flush=True)

    plain = None
    if not args.no_plain and args.precision != "fp64":
        prun = Run(L, sysm, dev, "fp64", args.n_par)
        pdt, pkern, pstages = prun.timed(1, 1)
        e_plain = prun.e_qp.cpu().numpy()
        z_plain = prun.z.cpu().numpy()
        reg = (z_plain >= 0.5) & (z_plain <= 1.0)
        d = np.abs(e_form - e_plain) * HA_MEV
        plain = {"value": round(pairs / pdt, 2), "ms_per_step": round(pdt * 1e3, 2),
                 "qp_max_err_mev_all_states": float(d.max()),
                 "within_1_mev": bool(d.max() <= 1.0),
                 "qp_max_err_mev_quasiparticle_like": float(d[reg].max()),
                 "quasiparticle_like_states": f"{int(reg.sum())} of {reg.size} (0.5 <= Z <= 1 in the plain path)",
                 "within_1_mev_quasiparticle_like": bool(d[reg].max() <= 1.0),
                 "stages_ms_per_step": {k: round(v[0], 3) for k, v in pstages.items()},
                 "roofline": roofline(sysm, pkern, "fp64", args.config, sysm.n_k)}
        print(f"# bench: plain fp64 {plain['value']} pairs/s, QP diff {plain['qp_max_err_mev_quasiparticle_like']:.3f} meV "
              f"(quasiparticle-like), {plain['qp_max_err_mev_all_states']:.3f} meV (all)", file=sys.stderr, flush=True)
        prun.ctx.close()
        del prun
    oracle_qp = qp_against_oracle(sysm, args.config, e_form, e_plain if plain else None)

    rl = roofline(sysm, kern, args.precision, args.config, args.steps * sysm.n_k)
    out = {
        "metric": "chi0+Sigma^c (q,w)-pairs/s", "value": round(value, 2), "unit": "(q,w)-pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"Si-like 2-atom cell: N_b={sysm.n_b}, N_aux={sysm.n_aux}, "
                               f"k grid {'x'.join(map(str, sp.nk))}, N_occ={sp.n_occ}, {sp.n_bands} bands, "
                               f"{sp.n_freq} modified Gauss-Legendre frequencies, QP bands {sp.qp_lo}..{sp.qp_lo + sp.n_qp - 1}, "
                               f"LRI amplitude a_L={sp.lri_amplitude:.4g} x N(0,1) exp(-|R|/2 bohr)",
                   "precision_form": args.precision, "pairs_per_step": pairs},
        "stages_ms_per_step": {k: round(v[0], 3) for k, v in stages.items()},
        "roofline": rl,
        "other_kernel": other_kernel(sysm, kern, args.precision, rl, args.steps * sysm.n_k),
    }
    if tuned:
        out["tuned"] = tuned
    if args.precision == "split_f16":
        sus = mfma_sustained()
        out["mfma_sustained"] = sus
        if "random" in sus and sus["random"]["pflops"] > 0:
            ref = sus["random"]["pflops"] * 1e3
            rl["frac_of_sustained_fp16"] = round(rl["achieved"] / ref, 4)
            for v in out["other_kernel"].values():
                v["frac_of_sustained_fp16"] = round(v["achieved"] / ref, 4)
        print(f"# bench: sustained FP16 MFMA {sus}", file=sys.stderr, flush=True)
    if not args.no_extras:
        out["sigma_x"] = sigma_x_timing(run, sysm, dev)
        out["lri_fit"] = lri_fit_timing(run, sysm)
        print("# bench: contour-deformation pass", file=sys.stderr, flush=True)
        out["contour_deformation"] = contour_timing(run, sysm, dev)
    if plain:
        out["plain_fp64"] = plain
        out["speedup_vs_plain"] = round(value / plain["value"], 3)
    if oracle_qp:
        out["qp_vs_oracle"] = oracle_qp
    if not args.no_cpu:
        print("# bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sysm)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
