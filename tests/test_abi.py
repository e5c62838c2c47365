"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: these tests run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "teraagent.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ta_[a-z_]+)\s*\(", text)))


def test_header_declares_the_exchange():
    names = declared()
    for n in ("ta_select_aura", "ta_serialize", "ta_view", "ta_delta_encode", "ta_delta_decode"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2509_24063_amd import native
    if not os.path.exists(native.LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(native.LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_bounds_without_gpu():
    from paper_2509_24063_amd import native
    if not os.path.exists(native.LIB):
        pytest.skip("library not built")
    L = native.lib()
    assert L.ta_serialize_bound(2, 3, 11) >= 2 * 32 + 16 + 3 * 88
    assert L.ta_delta_bound(1, 1000, 1000) >= 1000 + 64


def test_bench_refuses_more_than_one_gpu():
    """The bench measures one GPU; asked for more, it says so and exits
    before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
