"""Host logic of bench.py (no GPU): the byte models behind the roofline figure,
workload naming, the rocprofv3 summary and its traffic file, and the refusal
of more than one GPU."""
import csv
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_byte_models_scale_with_the_work():
    C, N, P = 1 << 18, 200_000, 40
    for k in ("collide", "drag", "scan", "scatter", "contacts", "resolve"):
        b32 = bench.algorithmic_bytes(k, "fp32", C, N, P)
        assert b32 > 0
        # twice the cells and particles: at most twice the bytes, more than the fixed parts
        assert bench.algorithmic_bytes(k, "fp32", 2 * C, 2 * N, 2 * P) == pytest.approx(2 * b32)
    # storage precision changes only the population and working-type terms
    c32, c16 = bench.algorithmic_bytes("collide", "fp32", C, N, P), bench.algorithmic_bytes("collide", "fp16", C, N, P)
    assert c32 - c16 == 18 * 2 * C
    assert bench.algorithmic_bytes("scan", "fp16", C, N, P) == bench.algorithmic_bytes("scan", "fp64", C, N, P) == 12 * C
    assert bench.model_bytes_per_step("fp32", C, N, P) > bench.algorithmic_bytes("collide", "fp32", C, N, P)
    with pytest.raises(KeyError):
        bench.algorithmic_bytes("nope", "fp32", C, N, P)


def test_phase_split_sums_to_the_step_model():
    """The per-phase bytes of the roofline figure add up to the whole-step
    model: 18 s_f + 16 s_c + 20 per cell, 14 s_p + 16 per particle, 16 + 8 s_p
    per pair."""
    C, N, P = 2_097_152, 2_000_000, 747_730
    for prec in ("fp64", "fp32", "fp16", "bf16"):
        parts = sum(bench.model_kernel_bytes(k, prec, C, N, P)
                    for k in ("collide", "drag", "scan", "scatter", "contacts", "resolve"))
        assert parts == bench.model_bytes_per_step(prec, C, N, P)
    assert bench.model_bytes_per_step("fp32", 1, 0, 0) == 156
    assert bench.model_bytes_per_step("fp16", 1, 0, 0) == 120
    assert bench.model_bytes_per_step("fp64", 1, 0, 0) == 292
    assert bench.model_bytes_per_step("fp32", 0, 1, 0) == 72 and bench.model_bytes_per_step("fp32", 0, 0, 1) == 48
    # the contact phase: cell starts, positions, pairs written
    assert bench.model_kernel_bytes("contacts", "fp32", C, N, P) == 4 * C + 8 * N + 8 * P
    with pytest.raises(KeyError):
        bench.model_kernel_bytes("nope", "fp32", C, N, P)


def test_workload_names_carry_the_precision_run():
    assert bench.workload_name("bubble-256x1024-200k-fp32", "fp16") == "bubble-256x1024-200k-fp16"
    assert bench.workload_name("riser-2048x8192-16000000-fp32", "fp32") == "riser-2048x8192-16000000-fp32"
    assert bench.workload_name("beds", "bf16") == "beds"


def _csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_summary_matches_either_form_of_a_phase(tmp_path, monkeypatch):
    """Counter rows of k_drag_flat and k_contacts_small count for the drag and
    contact phases; FETCH and WRITE are scaled so a copy of known size reads
    and writes exactly its size."""
    d = tmp_path
    stats = [dict(Name="void lbdps::k_contacts_small<1>(...)", Calls="10", AverageNs="15000", MinNs="14000",
                  MaxNs="16000", TotalDurationNs="150000", Percentage="60"),
             dict(Name="void lbdps::k_drag_flat<1>(...)", Calls="10", AverageNs="10000", MinNs="9000",
                  MaxNs="11000", TotalDurationNs="100000", Percentage="40")]
    _csv(str(d / "stats" / "x_kernel_stats.csv"), stats)
    for ctr, vals in (("fetch", (100.0, 300.0)), ("write", (50.0, 70.0))):
        _csv(str(d / ctr / "x_counter_collection.csv"),
             [dict(Kernel_Name="void lbdps::k_contacts_small<1>(...)", Counter_Value=str(vals[0])),
              dict(Kernel_Name="void lbdps::k_drag_flat<1>(...)", Counter_Value=str(vals[1]))])
    # the copy probe: 1 MiB copied, FETCH reads half of it, WRITE all of it (KiB)
    _csv(str(d / "cf" / "c_counter_collection.csv"), [dict(Kernel_Name="__amd_rocclr_copyBuffer", Counter_Value="512")])
    _csv(str(d / "cw" / "c_counter_collection.csv"), [dict(Kernel_Name="__amd_rocclr_copyBuffer", Counter_Value="1024")])
    monkeypatch.setattr(bench, "ROOT", str(d))
    args = types.SimpleNamespace(stats=str(d / "stats"), fetch=str(d / "fetch"), write=str(d / "write"),
                                 copy_fetch=str(d / "cf"), copy_write=str(d / "cw"), copy_bytes=1 << 20,
                                 label="unit", command="cmd", workload="wl")
    bench.summarize(args)
    t = json.load(open(d / "profiles" / "traffic_wl.json"))
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["bytes_per_launch"]["contacts"] == int(100 * 1024 * 2 + 50 * 1024)
    assert t["bytes_per_launch"]["drag"] == int(300 * 1024 * 2 + 70 * 1024)
    md = open(d / "profiles" / "unit.md").read()
    assert "k_contacts_small" in md and "cmd" in md


def test_traffic_is_dropped_when_the_kernels_changed(tmp_path, monkeypatch):
    os.makedirs(tmp_path / "profiles")
    with open(tmp_path / "profiles" / "traffic_wl.json", "w") as fh:
        json.dump({"kernel_source_hash": "abc", "bytes_per_launch": {"contacts": 123}}, fh)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda *a: "abc")
    assert bench.measured_traffic("wl", "contacts") == 123
    monkeypatch.setattr(bench, "kernel_source_hash", lambda *a: "def")
    assert bench.measured_traffic("wl", "contacts") is None


def test_traffic_is_checked_against_the_sources_it_lists(tmp_path, monkeypatch):
    """A counter summary that names its kernel sources (the 3-D step's adds
    coupled3d.hpp) is valid only while the hash over exactly those files
    matches; one that names none is checked against the default list."""
    os.makedirs(tmp_path / "profiles")
    with open(tmp_path / "profiles" / "traffic_wl.json", "w") as fh:
        json.dump({"kernel_sources": ["a.hpp", "b.hpp"], "kernel_source_hash": "ab",
                   "bytes_per_launch": {"step3d": 7}}, fh)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda s=bench.KERNEL_SOURCES: "ab" if tuple(s) == ("a.hpp", "b.hpp") else "x")
    assert bench.measured_traffic("wl", "step3d") == 7
    monkeypatch.setattr(bench, "kernel_source_hash", lambda s=bench.KERNEL_SOURCES: "x")
    assert bench.measured_traffic("wl", "step3d") is None
    assert set(bench.KERNEL_SOURCES) < set(bench.KERNEL_SOURCES_3D) and "coupled3d.hpp" in bench.KERNEL_SOURCES_3D


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2 and "one GPU" in out.stderr
