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
