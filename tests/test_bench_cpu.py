"""Host-side checks of the benchmark driver (no GPU needed)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_record_matches_kernel_sources_or_is_withheld(tmp_path, monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    v = bench.measured_traffic("k_build_batch<6,false,0>")
    assert v is None or v == int(round(rec["kernels"]["k_build_batch<6,false,0>"]["bytes_per_launch"]))
    # a record taken on other kernel sources is not reported
    fake = dict(rec, source_sha256="0" * 64)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(fake))
    for f in bench.KERNEL_SOURCES:
        os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
        (tmp_path / f).write_bytes(open(os.path.join(ROOT, f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_build_batch<6,false,0>") is None


def test_flop_constants_are_consistent():
    assert bench.FLOP_PER_CAND_LAYER == (bench.FLOP_SCATTER + bench.FLOP_PROPAGATE + bench.FLOP_TRANSPORT +
                                         bench.FLOP_WINDOW)
    assert bench.FLOP_PER_FIT_STEP == bench.FLOP_SCATTER + bench.FLOP_PROPAGATE + bench.FLOP_TRANSPORT
