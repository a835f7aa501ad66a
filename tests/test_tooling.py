"""Host-side tooling: the rocprofv3 summaries, the profiled-traffic lookup of
bench.py and the kernel-source hash that ties the two together."""
import csv
import os

import pytest

from paper_2201_04269_amd import build, prof_summary

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write_counters(dirname, rows):
    os.makedirs(dirname, exist_ok=True)
    keys = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(os.path.join(dirname, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=keys)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(keys, r)))


def test_source_hash_is_stable_and_tracks_sources():
    h = build.source_hash()
    assert len(h) == 16 and h == build.source_hash()
    int(h, 16)


def test_build_compiles_every_source_and_hashes_its_flags(monkeypatch):
    """Every C++/HIP source is a unit of the library; the per-source flags
    (the dS scheduling strategy) name units that exist and enter the hash
    that ties the committed profiles to the kernels."""
    on_disk = sorted(n for n in os.listdir(build.CSRC) if n.endswith((".cpp", ".hip")))
    assert sorted(build.SOURCES) == on_disk
    assert set(build.SOURCE_FLAGS) <= set(build.SOURCES)
    h = build.source_hash()
    monkeypatch.setitem(build.SOURCE_FLAGS, "kernels_ds_5_4.hip", [])
    assert build.source_hash() != h


def test_kernel_names_are_shortened():
    n = "void mbc::(anonymous namespace)::ds_kernel<float, 3, 3, 1, 6, 256>(mbc::(anonymous namespace)::BwdArgs)"
    assert prof_summary._short(n) == "ds_kernel<float, 3, 3, 1, 6, 256>"
    assert prof_summary._short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_traffic_calibration_and_per_dispatch_bytes(tmp_path, capsys):
    k = "void mbc::(anonymous namespace)::ds_kernel<float, 3, 3, 1, 6, 256>(mbc::(anonymous namespace)::BwdArgs)"
    add = "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add<float>, x>(int)"
    # the kernel's counters summed over two instances (dimensions), two dispatches
    _write_counters(tmp_path / "fetch", [(1, k, "FETCH_SIZE", 100.0, 0, 10), (1, k, "FETCH_SIZE", 100.0, 0, 10),
                                         (2, k, "FETCH_SIZE", 300.0, 0, 10)])
    _write_counters(tmp_path / "write", [(1, k, "WRITE_SIZE", 50.0, 0, 10), (2, k, "WRITE_SIZE", 150.0, 0, 10)])
    # calibration: a 2048-byte copy that FETCH_SIZE counts as 1 KiB and WRITE_SIZE as 2 KiB
    _write_counters(tmp_path / "calf", [(1, add, "FETCH_SIZE", 1.0, 0, 10)])
    _write_counters(tmp_path / "calw", [(1, add, "WRITE_SIZE", 2.0, 0, 10)])
    prof_summary.traffic(str(tmp_path / "fetch"), str(tmp_path / "write"), str(tmp_path / "calf"),
                         str(tmp_path / "calw"), "2048")
    out = capsys.readouterr().out.splitlines()
    assert f"source_hash {build.source_hash()}" in out
    line = [ln for ln in out if ln.startswith("traffic ds_kernel<float,3,3,1,6,256>")][0].split()
    # fetch: factor 2, mean of 200 and 300 KiB; write: factor 1, mean of 50 and 150 KiB
    assert float(line[3]) == pytest.approx(2 * 1024 * 250)
    assert float(line[4]) == pytest.approx(1024 * 100)
    assert float(line[5]) == pytest.approx(2 * 1024 * 250 + 1024 * 100)


def test_bench_reports_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    text = (f"source_hash {build.source_hash()}\n"
            "traffic ds_kernel<float,3,3,1,6,256> 1 6.0e8 6.0e8 1.2e9\n"
            "traffic ds_kernel<double,3,3,1,6,256> 1 9.0e9 6.0e8 9.6e9\n")
    (prof / "traffic_wl.txt").write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("wl", "dS", "f32c") == pytest.approx(1.2e9)
    assert bench.profiled_traffic("wl", "dS", "f64") == pytest.approx(9.6e9)
    assert bench.profiled_traffic("wl", "dW", "f32c") is None
    assert bench.profiled_traffic("other", "dS", "f32c") is None
    (prof / "traffic_wl.txt").write_text(text.replace(build.source_hash(), "0" * 16))
    assert bench.profiled_traffic("wl", "dS", "f32c") is None


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
