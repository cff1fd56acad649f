"""The C-ABI library loads on the host and exports every symbol the header
declares (no compute calls: this container has no GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lrigw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lrigw_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_matches_binding_list():
    from paper_2011_01400_amd import lrigw as L
    assert sorted(L.EXPORTS) == _declared()


def test_library_exports_every_symbol():
    from paper_2011_01400_amd import lrigw as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("liblrigw.so not built (run __graft_entry__.build())")
    lib = L.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.lrigw_strerror(-4).decode() == "matrix not Hermitian positive definite"
    assert lib.lrigw_strerror(0).decode() == "ok"


def test_binding_has_no_host_fallback():
    """The binding forwards to the library and nothing else: it imports neither
    the oracle nor numpy linear algebra for compute."""
    src = open(os.path.join(ROOT, "paper_2011_01400_amd", "lrigw.py")).read()
    assert "oracle" not in src
    assert "linalg" not in src


def test_bench_runs_on_one_gpu_only():
    """bench.py with more than one GPU exits with status 2 and says so in its
    JSON line, before it touches a device."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    d = json.loads(r.stdout.strip().splitlines()[-1])
    assert d["n_gpus"] == 2 and "one GPU" in d["error"]


def test_calibration_program_built_beside_the_library():
    """The build step also compiles the sustained matrix-core rate program that
    bench.py runs after its timed steps."""
    from paper_2011_01400_amd import build, lrigw as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("liblrigw.so not built (run __graft_entry__.build())")
    assert os.path.isfile(build.RATE_BIN) and os.access(build.RATE_BIN, os.X_OK)
