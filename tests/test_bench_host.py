"""Host logic of bench.py, no GPU: the one-GPU contract, the source hash
that keys the HBM-traffic record (blind to comments and layout), the gate
that drops a stale record, and the counter summary that writes it."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_device_call():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _hash_of(tmp_path, monkeypatch, text):
    (tmp_path / "k.hip").write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.hip"])
    return bench.kernel_hash()


def test_kernel_hash_ignores_comments_and_layout(tmp_path, monkeypatch):
    base = "int f(int x) {\n    return x + 1;  // next\n}\n"
    h = _hash_of(tmp_path, monkeypatch, base)
    assert _hash_of(tmp_path, monkeypatch, "/* the successor */\nint f(int x)\n{ return x + 1; }\n") == h
    assert _hash_of(tmp_path, monkeypatch, "int f(int x) {\n    return x + 2;  // next\n}\n") != h


def test_traffic_record_is_used_only_for_the_recorded_sources(tmp_path, monkeypatch):
    rec = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    assert bench.load_traffic() is None                      # no record
    rec.write_text(json.dumps({"kernel_hash": bench.kernel_hash(), "bytes_per_launch": 1234}))
    assert bench.load_traffic() == 1234
    rec.write_text(json.dumps({"kernel_hash": "0" * 16, "bytes_per_launch": 1234}))
    assert bench.load_traffic() is None                      # sources changed since
    rec.write_text("{not json")
    assert bench.load_traffic() is None


def _csv(path, counter, rows):
    lines = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    for i, (kernel, value) in enumerate(rows):
        lines.append(f'{i},"{kernel}",{counter},{value}')
    lines.append(f'{len(rows)},"{bench.DOMINANT}",OTHER_COUNTER,999999')
    path.write_text("\n".join(lines) + "\n")


def test_counter_summary_scales_by_the_calibration_kernel(tmp_path, monkeypatch):
    """The calibration kernel moves COPY_BYTES each way: a counter reading
    half of that (in KiB) gives the scale 2.  The dominant kernel's bytes are
    its mean reading per dispatch times that scale."""
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    cal = "void at::native::vectorized_elementwise_kernel<4, at::native::MulFunctor<float>>"
    half_kib = bench.COPY_BYTES // 2 // 1024
    full_kib = bench.COPY_BYTES // 1024
    f = tmp_path / "fetch.csv"
    w = tmp_path / "write.csv"
    _csv(f, "FETCH_SIZE", [(bench.DOMINANT, 100), (bench.DOMINANT, 300), ("other_kernel", 5)]
         + [(cal, half_kib)] * 3)
    _csv(w, "WRITE_SIZE", [(bench.DOMINANT, 50), (bench.DOMINANT, 50)] + [(cal, full_kib)] * 3)
    bench.summarize_pmc(str(f), str(w))
    rec = json.loads(out.read_text())
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["fetch_bytes"] == 2 * 200 * 1024
    assert rec["write_bytes"] == 50 * 1024
    assert rec["bytes_per_launch"] == 2 * 200 * 1024 + 50 * 1024
    assert rec["dispatches"] == [2, 2]
    assert rec["kernel_hash"] == bench.kernel_hash()


def test_counter_table_without_record(tmp_path, monkeypatch, capsys):
    """--no-record prints every kernel's scaled bytes and leaves the record alone."""
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    cal = "void at::native::vectorized_elementwise_kernel<4, at::native::MulFunctor<float>>"
    f = tmp_path / "fetch.csv"
    w = tmp_path / "write.csv"
    _csv(f, "FETCH_SIZE", [("void lbm::k_fused2d<float, 0, 1, 0>(lbm::StepArgs)", 1000)]
         + [(cal, bench.COPY_BYTES // 2 // 1024)] * 3)
    _csv(w, "WRITE_SIZE", [("void lbm::k_fused2d<float, 0, 1, 0>(lbm::StepArgs)", 500)]
         + [(cal, bench.COPY_BYTES // 1024)] * 3)
    bench.summarize_pmc(str(f), str(w), record=False)
    text = capsys.readouterr().out
    assert "| lbm::k_fused2d<float, 0, 1, 0> | 1 | 1,000 | 500 | 2.0 | 0.5 |" in text
    assert "MulFunctor" not in text
    assert not out.exists()


def test_counter_summary_needs_the_calibration_kernel(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    f = tmp_path / "fetch.csv"
    w = tmp_path / "write.csv"
    _csv(f, "FETCH_SIZE", [(bench.DOMINANT, 100)])
    _csv(w, "WRITE_SIZE", [(bench.DOMINANT, 50)])
    with pytest.raises(SystemExit):
        bench.summarize_pmc(str(f), str(w))
    assert not (tmp_path / "traffic.json").exists()


def test_workload_text():
    # the headline description, as the benchmark has always reported it
    assert bench.workload_text(4096) == (
        "D2Q9 periodic Taylor-Green + random-phase perturbation 4096x4096, FP32 shifted SoA, nu=1e-4, "
        "trimming + 3x3 median limiter (delta=1e-4), polynomial f*, quadratic dS, per-workgroup partials "
        "every step, FP64 global stats of the last step")
    assert "median limiter (delta=0)" in bench.workload_text(4096, delta_median=0.0)
    assert "ELBM collisions, no limiter, entropic f*" in bench.workload_text(4096, "elbm")
    assert "smooth ensemble factor (k=0.5, delta=0.01), polynomial f*" in bench.workload_text(4096, "smooth")
