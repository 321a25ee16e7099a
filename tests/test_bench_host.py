"""Host logic of the benchmark: the refusal of several GPUs, the per-run
JSONL record, the stored-traffic guard and the roofline's byte and flop
counts."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2501_16122_amd import synth  # noqa: E402


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single-GPU only" in r.stderr and r.stdout == ""


def test_record_appends_one_line_per_run(tmp_path):
    p = tmp_path / "runs.jsonl"
    bench.append_record(str(p), {"metric": "m", "value": 1.5})
    bench.append_record(str(p), {"metric": "m", "value": 2.5})
    lines = p.read_text().splitlines()
    assert len(lines) == 2
    recs = [json.loads(x) for x in lines]
    assert [r["result"]["value"] for r in recs] == [1.5, 2.5]
    for r in recs:
        assert r["kernel_source_hash"] == bench.kernel_source_hash()
        assert r["commit"] == "unknown" or len(r["commit"].split("+")[0]) == 40
        assert r["time_utc"].endswith("Z")
        assert r["machine"]["host"]["cores"] == os.cpu_count() and r["machine"]["host"]["cpu_model"]


def test_stored_traffic_only_for_its_kernel_and_sources():
    with open(bench.COUNTERS_FILE) as f:
        c = json.load(f)
    got = bench.stored_traffic(c["kernel"])
    if c.get("kernel_source_hash") == bench.kernel_source_hash():
        assert got == c["hbm_bytes_per_launch"]
    else:
        assert got is None
    assert bench.stored_traffic(c["kernel"] + " (another)") is None


def test_roofline_counts():
    w = synth.C2_GLS
    # 12 B per sample (int32 index + FP64 angle) over 2^28 samples
    assert bench.ALG_BYTES_PER_SAMPLE_F64 * w.n_samples == 12 * 2 ** 28
    # flops of one launch: 2 complex FFTs of N points at 5 N log2 N, 8 N for
    # the spectral step, 4 per window sample, per tile, and 6 per sample
    for n_fft, tiles_per_chunk in ((8192, 128), (16384, 43)):
        L = 2 * n_fft
        per_tile = 2 * 5 * n_fft * (n_fft.bit_length() - 1) + 8 * n_fft + 4 * L
        want = 256 * tiles_per_chunk * per_tile + 6 * w.n_samples
        assert bench.fft_flops_per_launch(w, n_fft) == pytest.approx(want)
