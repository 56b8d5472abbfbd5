"""Host-side logic of bench.py: the byte models, the rocprofv3 summarizers
and the single-GPU contract (no GPU needed)."""
import csv
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_byte_models_terms():
    b = _bench()
    n, V, M, P, C, nt = 1000, 900, 1139, 4096, 16, 64
    bmin, bmeth, per = b.byte_models(n, V, M, P, C, nt)
    D = M / V
    # B_min: points read twice, gradients written once, list written once and
    # read twice, image / G / T_final
    assert bmin == pytest.approx(2 * n * (16 + 4 * C) + n * (16 + 4 * C) + 12 * D * V
                                 + 8 * P * (C + 1))
    # the recomputing step sorts twice
    assert bmeth - bmin == pytest.approx(2 * (64 * V + 24 * D * V))
    _, bkeep, _ = b.byte_models(n, V, M, P, C, nt, keep_lists=True)
    assert bkeep - bmin == pytest.approx(64 * V + 24 * D * V)
    # BF16 features halve the feature bytes of the point reads
    bmin16, _, per16 = b.byte_models(n, V, M, P, C, nt, bf=2)
    assert bmin - bmin16 == pytest.approx(2 * n * C * 2)
    assert per["blend_bwd"] - per16["blend_bwd"] == V * C * 2
    assert set(per) == {"project", "bin", "sort", "blend_fwd", "blend_bwd", "project_bwd"}


def test_entry_mapping_covers_every_kernel():
    b = _bench()
    names = ["k_project_count", "k_colscan", "k_group_scan", "k_place", "k_scatter",
             "k_split", "k_sort_wm", "k_sort_lx", "k_blend_fwd_bilinear8<16, float, true>",
             "k_zero", "k_blend_bwd_bilinear8<16, float, true>", "k_unpack_scalars",
             "k_bg_reduce", "k_project_bwd"]
    got = {k: b._entry_of(k) for k in names}
    assert all(got.values()), got
    assert got["k_unpack_scalars"] == "blend_bwd" and got["k_sort_lx"] == "sort"


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_trace_per_step(tmp_path, capsys):
    b = _bench()
    _write_csv(tmp_path / "run_kernel_stats.csv",
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
                "StdDev"],
               [["inpc::(anonymous namespace)::k_scatter(inpc::Cam, int)", 6, 1200000, 200000,
                 60, 1, 1, 0],
                ["void inpc::(anonymous namespace)::k_blend_fwd_bilinear8<16, float, true>"
                 "(inpc::BlendArgs)", 3, 900000, 300000, 40, 1, 1, 0]])
    b.summarize_trace(str(tmp_path), 3, "cmd")
    out = capsys.readouterr().out
    assert "`k_scatter` | bin | 6 | 2 | 200.0 | 400.0 |" in out
    # calls per step from the launch counts: bin twice, the forward blend once
    assert "| inpc_blend_fwd | 1 | 300.0 |" in out
    assert "| inpc_bin | 2 | 200.0 |" in out
    assert "sum of kernel time per step: 700.0 us" in out


def test_summarize_counters_means(tmp_path, capsys):
    b = _bench()
    _write_csv(tmp_path / "run_counter_collection.csv", ["Kernel_Name", "Counter_Name",
                                                          "Counter_Value"],
               [["k_sort_wm(int)", "SQ_INSTS_VALU", 10], ["k_sort_wm(int)", "SQ_INSTS_VALU", 30],
                ["k_zero(float*)", "SQ_INSTS_VALU", 5], ["not_ours(int)", "SQ_INSTS_VALU", 1]])
    b.summarize_counters(str(tmp_path), "cmd")
    out = capsys.readouterr().out
    assert "| `k_sort_wm` | sort | 20 |" in out
    assert "| `k_zero` | backward_zero | 5 |" in out
    assert "not_ours" not in out


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
