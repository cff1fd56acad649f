"""GPU: the calibration program for the sustained dense FP16 matrix-core rate
(built beside the library) runs and reports figures inside what the device
can do: at most the published 2.5 PFLOP/s dense FP16 peak (at most 2.4 GHz
shader clock), and random operands no faster than zero operands."""
import json
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2011_01400_amd", "mfma_rate")


def test_sustained_rate_is_plausible():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        pytest.fail("mfma_rate not built (run __graft_entry__.build())")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    d = json.loads(r.stdout.strip().splitlines()[-1])
    print(f"\n[gpu mfma rate] {d}", flush=True)
    z, x = d["zeros"], d["random"]
    for m in (z, x):
        assert 0.2 < m["pflops"] <= 2.5 * 1.02
        assert 300 < m["mhz"] <= 2400 * 1.02
    assert x["pflops"] <= z["pflops"] * 1.02
    # the rate follows the clock: one 16x16x32 MFMA per 16 cycles per SIMD
    for m in (z, x):
        assert abs(m["pflops"] / (1024 * m["mhz"] * 1e6 * 1024 / 1e15) - 1.0) < 0.15
