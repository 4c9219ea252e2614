"""Host logic of the benchmark (CPU): the algorithmic byte counts behind the
roofline figures, the reading of the committed HBM-traffic summary, and the
refusal of a multi-GPU run."""
import os
import subprocess
import sys
from types import SimpleNamespace

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _info(n=10000, m=13000, nn=9999, nnz_l=20472, nnz_y=36000):
    return SimpleNamespace(n=n, m=m, nn=nn, nnz_l=nnz_l, nnz_y=nnz_y)


def test_byte_counts_follow_their_definitions():
    info = _info()
    F = info.nn + 2 * info.nnz_l
    # per NR iteration: admittances read, Jacobian stored and read, factors
    # written and read, L D U read by the substitutions, the bus vectors
    assert bench.newton_bytes_per_iter(info) == 16 * 36000 + (32 + 64 + 32) * F + 96 * 10000
    # the factorisation kept at the solution: no substitutions, no vectors
    assert bench.kept_factor_bytes(info) == 16 * 36000 + 96 * F
    assert bench.adjoint_bytes(info) == 32 * F + 32 * info.n + 16 * info.nn
    assert bench.branch_grad_bytes(info) == 16 * info.n + 16 * info.m
    # the figures of the 10,000-bus grid quoted with the results
    assert bench.newton_bytes_per_iter(info) == 8056704
    assert bench.kept_factor_bytes(info) == 5466528


def test_roofline_fields():
    rf = bench.roofline(8e9, 2.0, "k", 10, 8e8)
    assert rf["achieved"] == pytest.approx(4000.0)
    assert rf["frac"] == pytest.approx(0.5)
    assert rf["peak"] == 8000.0 and rf["unit"] == "GB/s" and rf["bound"] == "hbm"


def test_measured_traffic_only_while_sources_and_launch_match(tmp_path, monkeypatch):
    settings = {"threads": 512, "tail_budget": 161792, "interleave": 4}
    tag = bench.launch_tag(settings)
    assert tag == "T512-tail161792-C4"
    f = tmp_path / "traffic.md"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic(settings) is None  # no summary
    src = bench.kernel_source_hash()
    f.write_text(f"text\ntraffic: bytes_per_launch=1.25e+10 fetch=8e9 write=4.5e9 "
                 f"sources={src} launch={tag}\n")
    assert bench.measured_traffic(settings) == pytest.approx(1.25e10)
    assert bench.measured_traffic(None) is None
    assert bench.measured_traffic(dict(settings, interleave=2)) is None
    f.write_text(f"traffic: bytes_per_launch=1.25e+10 sources={'0' * 16} launch={tag}\n")
    assert bench.measured_traffic(settings) is None  # kernels changed since


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_sync_counts_of_a_one_case_launch():
    """Barriers per NR iteration: one workgroup takes a workgroup barrier per
    level step; a spread launch a grid barrier per shared step."""
    import gridgen
    from paper_1811_02512_amd import api

    g = gridgen.make_grid(2000, 1)
    sym = api.Symbolic(g.n, g.f, g.t)
    sym.set_launch(512, 0, 1)  # no tail: every level shared
    info = sym.info
    assert info.tail_levels == 0
    one = bench.sync_counts(sym, 0)
    assert one == {"workgroup_barriers": 1 + 2 * info.nlevels, "grid_barriers": 0}
    spread = bench.sync_counts(sym, 16)
    narrow = sum(1 for w in np.diff(sym.export()["level_ptr"]) if w <= 512)
    # mismatch, every factorisation level, the narrow backward levels' end
    # (workgroup 0), every wide backward level
    assert spread["grid_barriers"] == 1 + info.nlevels + 1 + (info.nlevels - narrow)
    assert spread["levels_on_workgroup_0"] == narrow
