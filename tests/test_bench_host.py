"""Host logic of bench.py (no GPU): the algorithmic bytes each kernel's
roofline is priced with, the refusal of several GPUs, and the HBM traffic and
trace summaries written from rocprofv3 output."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2212_10680_amd import workloads as wl  # noqa: E402

# every kernel name fl_step_timed_every reports
TIMED_KERNELS = ["k_moments_eos", "k_collide_stream", "k_collide_zmarch", "k_collide_zmarch_iso",
                 "k_collide_zmarch_iso_cs", "k_fused_step"]


def test_algorithmic_bytes_ternary_fp32_isotropic():
    """256^3 ternary FP32: populations 19 x 3 x 4 = 228 B each way, the
    rest-population reference 3 x 4 B, the FP64 fields rho~_i, ln f_i, phi
    7 x 8 B, the force history 3 x 4 B each way."""
    w = wl.WORKLOADS["ternary_droplets_3d"]
    ab = bench.algorithmic_bytes(w, "fp32", "isotropic", lap_pass=False)
    assert ab["k_moments_eos"] == 228 + 12 + 56
    assert ab["k_collide_zmarch_iso_cs"] == ab["k_collide_zmarch_iso"] == 2 * 228 + 12 + 56 + 2 * 12 == 548
    assert ab["step"] == 2 * 228 + 2 * 56 + 2 * 12 + 12 == 604
    assert "k_interface_lap" not in ab
    lap = bench.algorithmic_bytes(w, "fp32", "isotropic", lap_pass=True)
    assert lap["k_interface_lap"] == 16 and lap["step"] == 620


def test_algorithmic_bytes_binary_and_fp64():
    w = wl.WORKLOADS["binary_slab_3d"]
    ab = bench.algorithmic_bytes(w, "fp32", "axis")
    assert (ab["k_moments_eos"], ab["k_collide_zmarch"], ab["step"]) == (200, 376, 416)
    w3 = wl.WORKLOADS["ternary_droplets_3d"]
    ab = bench.algorithmic_bytes(w3, "fp64", "isotropic", lap_pass=True)
    # FP64 populations, no reference: 19 x 3 x 8 = 456 B each way, force history 3 x 8 B
    assert (ab["k_moments_eos"], ab["k_collide_stream"], ab["step"]) == (512, 1016, 1088)


@pytest.mark.parametrize("wname,precision,stencil", [("ternary_droplets_3d", "fp32", "isotropic"),
                                                     ("binary_slab_3d", "fp32", "axis"),
                                                     ("ternary_droplet_2d", "fp64", "axis")])
def test_every_timed_kernel_has_a_byte_count(wname, precision, stencil):
    ab = bench.algorithmic_bytes(wl.WORKLOADS[wname], precision, stencil)
    for k in TIMED_KERNELS:
        assert ab[k] > 0, k


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _pmc_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        wr.writeheader()
        for i, (name, kib) in enumerate(rows):
            wr.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})
            # a dispatch's row repeated (one per agent or per instance) counts once
            wr.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_traffic_scaled_by_the_copy(tmp_path, monkeypatch):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what they read
    for the 1 GiB device copy of the same run: here FETCH_SIZE counts half of
    the copy's bytes (scale 2), WRITE_SIZE all of them (scale 1)."""
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    k = "void fl::k_collide_zmarch_iso_cs<3, float, true>(fl::KParams, float const*)"
    copy = "__amd_rocclr_copyBuffer"
    fetch, write = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _pmc_csv(fetch, "FETCH_SIZE", [(copy, 524288.0), (k, 1000.0), (k, 1200.0)])
    _pmc_csv(write, "WRITE_SIZE", [(copy, 1048576.0), (k, 800.0), (k, 800.0)])
    w = wl.WORKLOADS["ternary_droplets_3d"]
    bench.write_traffic(str(fetch), str(write), w, "isotropic")
    out = json.load(open(tmp_path / "traffic.json"))
    assert out["scale"] == {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
    assert out["kernel_source_hash"] == bench.kernel_source_hash()
    (row,) = [r for r in out["kernels"] if r["kernel"] == "k_collide_zmarch_iso_cs"]
    assert row["launches"] == 2
    assert row["read_bytes"] == round(1100.0 * 1024 * 2)
    assert row["write_bytes"] == round(800.0 * 1024)
    assert row["bytes_per_launch"] == row["read_bytes"] + row["write_bytes"]
    assert row["nodes"] == w.nodes and row["stencil"] == "isotropic"


def test_trace_summary_table(tmp_path, capsys):
    p = tmp_path / "kernel_stats.csv"
    with open(p, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"])
        wr.writeheader()
        wr.writerow({"Name": "void fl::k_moments_eos<1, 3, float>(fl::KParams)", "Calls": 25,
                     "AverageNs": 936800.0, "MinNs": 922400.0, "MaxNs": 948000.0, "Percentage": 27.52})
    bench.trace_summary(str(p))
    lines = capsys.readouterr().out.strip().splitlines()
    assert lines[-1] == "| `fl::k_moments_eos<1, 3, float>` | 25 | 936.8 | 922.4 | 948.0 | 27.52 |"


def test_traffic_rows_per_precision_are_merged(tmp_path, monkeypatch):
    """A counter run of the FP64 form adds its rows beside the FP32 form's
    (same kernel name, lattice and stencil); stored_traffic tells them apart by
    precision, and a later run of one form replaces only that form's rows."""
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    copy = "__amd_rocclr_copyBuffer"
    k32 = "void fl::k_moments_eos<1, 3, float>(fl::KParams, float const*)"
    k64 = "void fl::k_moments_eos<1, 3, double>(fl::KParams, double const*)"
    w = wl.WORKLOADS["ternary_droplets_3d"]

    def run(kname, fetch_kib, tag):
        fetch, write = tmp_path / f"f{tag}.csv", tmp_path / f"w{tag}.csv"
        _pmc_csv(fetch, "FETCH_SIZE", [(copy, 1048576.0), (kname, fetch_kib)])
        _pmc_csv(write, "WRITE_SIZE", [(copy, 1048576.0), (kname, 100.0)])
        bench.write_traffic(str(fetch), str(write), w, "isotropic")

    run(k32, 1000.0, "a")
    run(k64, 3000.0, "b")
    out = json.load(open(tmp_path / "traffic.json"))
    assert sorted(r["precision"] for r in out["kernels"]) == ["fp32", "fp64"]
    assert bench.stored_traffic("k_moments_eos", w.nodes, "isotropic", "fp32") == 1100 * 1024
    assert bench.stored_traffic("k_moments_eos", w.nodes, "isotropic", "fp64") == 3100 * 1024
    run(k32, 2000.0, "c")
    assert bench.stored_traffic("k_moments_eos", w.nodes, "isotropic", "fp32") == 2100 * 1024
    assert bench.stored_traffic("k_moments_eos", w.nodes, "isotropic", "fp64") == 3100 * 1024
    assert len(json.load(open(tmp_path / "traffic.json"))["kernels"]) == 2
    # rows taken on other kernel sources are not reported
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.stored_traffic("k_moments_eos", w.nodes, "isotropic", "fp64") is None
