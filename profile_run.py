"""Short workload for hardware-counter runs (run under rocprofv3).

Runs (1) a plain device-to-device copy of a known size, the calibration for
the FETCH_SIZE / WRITE_SIZE counters, then (2) the tile tuner and one q of the
path on the Si-like cell in the chosen precision form (the per-launch traffic
of every kernel is the same for every q except q = 0).  `summarize` turns the
counter CSVs of two such runs into bytes per launch, taking for each kernel
family its last dispatch (the pass's; the tuner's trials come first).

  rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -- python3 profile_run.py
  python3 profile_run.py --summarize <fetch dir> <write dir>
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30          # calibration copy: 1 GiB read + 1 GiB written
# the main kernel of each stage (all its variants) and its source file
FAMILIES = {"sigma_mfma": (("k_sigma_res", "k_sigma_split", "k_sigma_splitq", "k_sigma_mfma"), "k_sigma.hip"),
            "chi0_mfma": (("k_chi0_split", "k_chi0_split8", "k_chi0_mfma"), "k_chi0.hip")}


def run(precision: str, config: int, q: int, chi0_nw: int = 0):
    import torch
    sys.path.insert(0, ROOT)
    from paper_2011_01400_amd import lrigw as L
    from synth.systems import make_config
    L.load()
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    b.copy_(a)                     # the calibration dispatch
    torch.cuda.synchronize()
    del a, b
    s = make_config(config)
    dev = L.device_inputs(s)
    sp = s.spec
    ctx = L.Context.from_system(s, precision=precision)
    H = ctx.empty("H")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    ctx.tune(H, dev["evec"], dev["eig"])           # the kernel variants bench.py runs
    if chi0_nw:
        # the tuner's choice between the two response kernels is a near-tie
        # that varies by run: hold the one asked for (tuned splits and padding)
        nw, sp_, pad, var = ctx.tiles
        ctx.set_tiles(chi0_nw, sp_, pad, var)
    sigma = torch.zeros((s.n_k, sp.n_qp, sp.n_freq), dtype=torch.complex128, device="cuda")
    e = torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    z = torch.zeros_like(e)
    ctx.g0w0(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, dev["e_static"], 16, sigma, e, z,
             q_first=q, q_last=q + 1)
    torch.cuda.synchronize()
    print(f"profile_run: {precision} config {config} q {q} done", flush=True)


def run_contour(precision: str, config: int, n_r: int = 16):
    """The tile tuner, then one whole contour-deformation pass (lrigw_g0w0_cd,
    n_r real frequencies up to 0.6 of the smallest transition energy), the
    workload of bench.py's contour-deformation figures."""
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    from paper_2011_01400_amd import lrigw as L
    from synth.systems import make_config
    L.load()
    s = make_config(config)
    dev = L.device_inputs(s)
    sp = s.spec
    ctx = L.Context.from_system(s, precision=precision)
    H = ctx.empty("H")
    ctx.lri_ft(dev["lri"], s.R, dev["evec"], H)
    ctx.tune(H, dev["evec"], dev["eig"])
    dmin = float(s.eig[:, s.n_occ:].min() - s.eig[:, :s.n_occ].max())
    ctx.set_real_grid(n_r, 0.6 * dmin)
    e = torch.zeros((s.n_k, sp.n_qp), dtype=torch.float64, device="cuda")
    z = torch.zeros_like(e)
    rc, bad = ctx.g0w0_cd(H, dev["evec"], dev["eig"], dev["V"], dev["p"], s.omega_cell, dev["e_static"], 0.002, e, z)
    torch.cuda.synchronize()
    print(f"profile_run: contour pass {precision} config {config}: rc {rc}, "
          f"{int(np.isfinite(e.cpu().numpy()).sum())} states evaluated", flush=True)


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    out = []
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            out.append(r)
    return out


def _per_kernel(rows):
    """{kernel name: [(dispatch id, value)]} (counter value in KiB, summed over the dispatch)."""
    acc = {}
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("KernelName") or ""
        val = float(r.get("Counter_Value") or r.get("Counter-Value") or 0.0)
        disp = int(r.get("Dispatch_Id") or r.get("Dispatch-Id") or r.get("Correlation_Id") or 0)
        acc.setdefault(name, {}).setdefault(disp, 0.0)
        acc[name][disp] += val
    return {k: sorted(v.items()) for k, v in acc.items()}


def summarize(fetch_dir, write_dir, precision, config, out_path):
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        per = _per_kernel(_rows(d))
        copy = [v for k, lst in per.items() if "copy" in k.lower() for _, v in lst]
        copy = max(copy, default=None)
        scale = COPY_BYTES / (copy * 1024.0) if copy else None
        res[counter] = {"copy_kib": copy, "scale": scale, "kernels": {}}
        last = {}
        for k, lst in per.items():
            name = k.split("(")[0].replace("void ", "").strip()
            base = name.split("<")[0].strip()
            for fam, (members, _) in FAMILIES.items():
                if base in members and (fam not in last or lst[-1][0] > last[fam][0]):
                    last[fam] = (lst[-1][0], lst[-1][1], name)
        for fam, (_, v, name) in last.items():
            res[counter]["kernels"][fam] = (v, name)
    out = {}
    try:
        with open(out_path) as f:
            out = json.load(f)
    except (OSError, ValueError):
        pass
    for fam, (_, src) in FAMILIES.items():
        fr = res["FETCH_SIZE"]["kernels"].get(fam)
        wr = res["WRITE_SIZE"]["kernels"].get(fam)
        if fr is None or wr is None:
            continue
        (f, kname), (w, _) = fr, wr
        sf, sw = res["FETCH_SIZE"]["scale"], res["WRITE_SIZE"]["scale"]
        with open(os.path.join(ROOT, "paper_2011_01400_amd", "csrc", src), "rb") as fh:
            h = hashlib.sha256(fh.read()).hexdigest()[:16]
        key = f"{fam}:{precision}:c{config}"
        out[key] = {"kernel": kname, "source": src, "source_sha256_16": h,
                    "fetch_kib_per_launch": f, "write_kib_per_launch": w,
                    "copy_calibration": {"fetch_scale": sf, "write_scale": sw, "copy_bytes": COPY_BYTES},
                    "bytes_per_launch": (f * 1024.0 * (sf or 1.0)) + (w * 1024.0 * (sw or 1.0))}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def _per_kernel_counters(rows):
    """{kernel name: {dispatch id: {counter: value}}} from one counter CSV."""
    acc = {}
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("KernelName") or ""
        cname = r.get("Counter_Name") or r.get("Counter-Name") or ""
        val = float(r.get("Counter_Value") or r.get("Counter-Value") or 0.0)
        disp = int(r.get("Dispatch_Id") or r.get("Dispatch-Id") or r.get("Correlation_Id") or 0)
        d = acc.setdefault(name, {}).setdefault(disp, {})
        d[cname] = d.get(cname, 0.0) + val
    return acc


def summarize_counters(dirs, title):
    """Markdown table of every counter in the given runs for the last dispatch
    of each kernel family (the pass's launch; the tuner's trials come first),
    with MFMA busy as a share of the SIMD cycles of the dispatch."""
    vals = {}
    names = {}
    for d in dirs:
        per = _per_kernel_counters(_rows(d))
        for k, disp in per.items():
            base = k.split("(")[0].replace("void ", "").strip().split("<")[0].strip()
            for fam, (members, _) in FAMILIES.items():
                if base in members:
                    last = max(disp)
                    if fam not in names or last >= names[fam][0]:
                        names[fam] = (last, k.split("(")[0].replace("void ", "").strip())
                        vals.setdefault(fam, {}).update(disp[last])
    lines = [f"## {title}", "", "| counter | " + " | ".join(f"{fam} (`{names[fam][1]}`)" for fam in vals) + " |",
             "|---|" + "---:|" * len(vals)]
    counters = sorted({c for v in vals.values() for c in v})
    for c in counters:
        lines.append(f"| {c} | " + " | ".join(f"{vals[f].get(c, float('nan')):.6g}" for f in vals) + " |")
    derived = []
    for f, v in vals.items():
        if "SQ_INSTS_MFMA" in v and "SQ_INSTS_VALU" in v and v["SQ_INSTS_MFMA"] > 0:
            derived.append(f"- {f}: VALU instructions per MFMA instruction "
                           f"{(v['SQ_INSTS_VALU'] - v['SQ_INSTS_MFMA']) / v['SQ_INSTS_MFMA']:.3f} "
                           "(SQ_INSTS_VALU counts the MFMA instructions too)")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in v and "GRBM_GUI_ACTIVE" in v and v["GRBM_GUI_ACTIVE"] > 0:
            derived.append(f"- {f}: MFMA busy {100.0 * v['SQ_VALU_MFMA_BUSY_CYCLES'] / (v['GRBM_GUI_ACTIVE'] / 8 * 256 * 4):.1f}% "
                           "of SIMD cycles (SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 XCDs x 256 CUs x 4 SIMDs))")
        if "SQ_LDS_BANK_CONFLICT" in v and "SQ_LDS_IDX_ACTIVE" in v and v["SQ_LDS_IDX_ACTIVE"] > 0:
            derived.append(f"- {f}: LDS bank-conflict cycles per LDS-active cycle "
                           f"{v['SQ_LDS_BANK_CONFLICT'] / v['SQ_LDS_IDX_ACTIVE']:.3f}")
    if derived:
        lines += ["", *derived]
    print("\n".join(lines))


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", default="split_f16")
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--q", type=int, default=1)
    ap.add_argument("--summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--counters", nargs="+", metavar="PMC_DIR", help="markdown table of the counters of these runs")
    ap.add_argument("--contour", action="store_true", help="one contour-deformation pass instead of one q")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--chi0-nw", type=int, default=0, help="hold the response kernel at this many frequencies per "
                    "workgroup after tuning (2 or 4; 0: the tuner's choice)")
    a = ap.parse_args()
    if a.counters:
        summarize_counters(a.counters, f"{a.precision}, config {a.config}")
    elif a.summarize:
        summarize(a.summarize[0], a.summarize[1], a.precision, a.config, a.out)
    elif a.contour:
        run_contour(a.precision, a.config)
    else:
        run(a.precision, a.config, a.q, a.chi0_nw)
