"""Host-side pieces of bench.py (CPU only): the algorithmic flop count, the traffic
summary reader and the one-GPU guard."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_flops_per_pair_count():
    """110 (P + 1) + 70 flops per (pixel, Gaussian) pair: 290, 510 and 840 for P = 1, 3, 6."""
    assert [bench.alg_flops_per_pair(P) for P in (1, 3, 6)] == [290, 510, 840]
    for P in range(7):
        assert bench.alg_flops_per_pair(P) == 110 * (P + 1) + 70


def test_traffic_reader_needs_the_current_kernel_sources(tmp_path):
    good = tmp_path / "good.txt"
    good.write_text(f"comment line\nbytes_per_launch: 12345\nkernel_fingerprint: {bench.kernel_fingerprint()}\n")
    assert bench.read_traffic(str(good)) == 12345.0
    stale = tmp_path / "stale.txt"
    stale.write_text("bytes_per_launch: 12345\nkernel_fingerprint: 0000000000000000\n")
    assert bench.read_traffic(str(stale)) is None
    assert bench.read_traffic(str(tmp_path / "missing.txt")) is None
    # the rotation loop's summary: its own key and sources
    rot = tmp_path / "rot.txt"
    rot.write_text(f"pixel_loop_bytes_per_query: 777\n"
                   f"kernel_fingerprint: {bench.kernel_fingerprint(bench.ROTATION_LOOP_SOURCES)}\n")
    assert bench.read_traffic(str(rot), "pixel_loop_bytes_per_query", bench.ROTATION_LOOP_SOURCES) == 777.0
    assert bench.read_traffic(str(rot), "pixel_loop_bytes_per_query") is None   # other sources
    assert bench.kernel_fingerprint(bench.ROTATION_LOOP_SOURCES) != bench.kernel_fingerprint()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "error" in line


def test_cpu_baseline_runs_on_several_workers():
    from paper_2503_00308_amd import synth
    scene, intr, box, _ = synth.config(1)
    r = bench.cpu_baseline(scene, intr, box, budget_s=0.5, workers=2)
    assert r["cores"] == 2 and r["kind"] == "oracle" and r["value"] > 0 and "worker" in r["sample"]
