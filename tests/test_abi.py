"""The C-ABI library loads and exports every entry point include/cc.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(cc_[a-z_]+)\s*\(", src, flags=re.M))
    return names


def test_header_declares_the_paper_entry_points():
    names = declared_functions()
    for f in ("cc_pair_timesteps", "cc_split_labels", "cc_kick", "cc_drift", "cc_evolve", "cc_evolve_batch"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_1407_7105_amd import cc
    path = cc.lib_path()
    if not os.path.exists(path):
        pytest.skip("library not built")
    lib = ctypes.CDLL(path)
    names = declared_functions()
    assert names == set(cc.SYMBOLS)
    for f in names:
        assert hasattr(lib, f), f


def test_binding_rejects_missing_library(tmp_path, monkeypatch):
    from paper_1407_7105_amd import cc
    monkeypatch.setattr(cc, "_LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(cc, "_lib", None)
    with pytest.raises(ImportError):
        cc.load_library()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with status 2 and says
    so before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
