"""CPU-side checks of the C ABI: the library loads and exports every symbol
the header declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

import paper_2110_10762_amd as pr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "parareal.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_solver_calls():
    syms = declared_symbols()
    for s in ("pr_create", "pr_solve_sync", "pr_solve_async", "pr_grad", "pr_destroy"):
        assert s in syms


@pytest.mark.skipif(not os.path.exists(pr.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pr.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert set(pr.EXPORTS) <= set(declared_symbols())


@pytest.mark.skipif(not os.path.exists(pr.LIB_PATH), reason="library not built")
def test_struct_layouts_match_header():
    # field order/count of the ctypes mirrors against the header text
    text = open(os.path.join(ROOT, "include", "parareal.h")).read()
    for cname, pyc in (("pr_config", pr.pr_config), ("pr_info", pr.pr_info),
                       ("pr_stats", pr.pr_stats), ("pr_async_opts", pr.pr_async_opts)):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), text, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = re.findall(r"\**\s*([a-z_A-Z0-9]+)\s*(?:,|;)", body)
        assert [f for f, _ in pyc._fields_] == names, cname


def test_create_without_gpu_fails_cleanly():
    if not os.path.exists(pr.LIB_PATH):
        pytest.skip("library not built")
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    lib = pr.load_library()
    cfg = pr.make_config(1, 10, 1.0, 1.0, 2, 1e-3)
    h = ctypes.c_void_p()
    rc = lib.pr_create(ctypes.byref(cfg), 1, 0, None, ctypes.byref(h))
    assert rc != 0 and not h.value
    assert lib.pr_last_error()


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for script in ("bench.py", "bench_delays.py"):
        res = subprocess.run([sys.executable, os.path.join(root, script), "--gpus", "2"],
                             capture_output=True, text=True, timeout=120)
        assert res.returncode == 2, (script, res.stderr)
        assert "one GPU" in res.stderr, (script, res.stderr)


def test_bench_source_digest_ignores_comments(tmp_path, monkeypatch):
    import importlib
    import shutil
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    bench = importlib.import_module("bench")
    src = os.path.join(root, "paper_2110_10762_amd", "csrc")
    fake = tmp_path / "paper_2110_10762_amd" / "csrc"
    shutil.copytree(src, fake)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.sources_digest()
    p = fake / "common.hpp"
    p.write_text(p.read_text() + "\n// a comment\n/* another\n one */\n")
    assert bench.sources_digest() == d0
    p.write_text(p.read_text() + "\nstatic int pr_digest_probe_ = 1;\n")
    assert bench.sources_digest() != d0
