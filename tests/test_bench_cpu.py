"""Host logic of the benchmark (CPU, no GPU): the algorithmic operation
tables, the weighing of the generate kernels' re-computation, the reading of
the committed profile summaries, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np

import bench
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_operation_mix_adds_up_to_the_counts():
    assert set(bench.ALU_MIX) == set(bench.ALU_OPS) == set(bench.ALU_UNIT)
    for k, ops in bench.ALU_OPS.items():
        mix = bench.ALU_MIX[k]
        assert set(mix) == {"mul", "shr64", "add64", "trans", "other"}, k
        assert abs(sum(mix.values()) - ops) < 1e-9, k


def test_paired_share_follows_the_parity_of_the_first_counter():
    g = 0x9E3779B97F4A7C15
    cfg = {"n": np.array([10, 30, 60], dtype=np.uint64),
           # first z = seed + offset + gamma: odd, even, even
           "seed": np.array([(1 - g) % (1 << 64), (2 - g) % (1 << 64), (4 - g) % (1 << 64)], dtype=np.uint64),
           "offset": np.array([0, 0, 0], dtype=np.uint64)}
    assert bench.paired_share(cfg) == 0.9
    # the offset moves the first counter too
    cfg["offset"] = np.array([1, 0, 1], dtype=np.uint64)
    assert bench.paired_share(cfg) == 0.4
    # the headline workload: about half of its outputs in each kind of stream
    f = bench.paired_share(synth.batched_streams())
    assert 0.4 < f < 0.6
    assert bench.recomputed_ops("polar_generate", 1.0) == 27
    assert bench.recomputed_ops("polar_generate", 0.0) == 32
    assert bench.recomputed_ops("ratio_generate", 0.5) == 31.5


def test_profile_summaries_are_read_only_for_the_current_kernels(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    h = bench.kernel_source_hash()
    (tmp_path / "avg_k.txt").write_text("# c\nsource_hash=%s\navg_ms=0.5\n" % h)
    (tmp_path / "traffic_k.txt").write_text("# c\nsource_hash=%s\nhbm_bytes_per_launch=123\n" % h)
    assert bench.read_profile_avg("k") == 0.5
    assert bench.read_traffic("k") == 123.0
    (tmp_path / "avg_k.txt").write_text("source_hash=0000000000000000\navg_ms=0.5\n")
    (tmp_path / "traffic_k.txt").write_text("source_hash=0000000000000000\nhbm_bytes_per_launch=123\n")
    assert bench.read_profile_avg("k") is None
    assert bench.read_traffic("k") is None
    assert bench.read_profile_avg("missing") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--no-extras", "--no-cpu"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stderr + r.stdout) or "1 GPU" in (r.stderr + r.stdout)
