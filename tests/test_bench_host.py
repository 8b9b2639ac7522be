"""Host-side pieces of bench.py: the committed counter summaries it reads for
the roofline's `traffic` field, the algorithmic byte and flop models, and the
one-GPU rule (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2404_03399_amd import workloads as W  # noqa: E402


def test_traffic_is_read_for_each_profiled_launch_shape():
    """Every committed FETCH/WRITE summary carries the current kernel-source
    hash and one traffic line per launch shape the tuner can pick; the value
    is within a few percent of the algorithmic bytes (no re-reads)."""
    w = W.c2_advection_large("adg_at")
    alg20 = bench.BYTES_PER_DOF_STEP_FUSED * w.n_elem * 4 + 2 * bench.ring_bytes_per_step(w)
    for R in (2, 4):
        t = bench.read_traffic(R, 2)
        assert t is not None and 1.0 <= t / alg20 < 1.1, (R, t, alg20)
        assert bench.read_traffic(R, 2, 1 << 24) is not None
        assert bench.read_traffic(R, 2, profile="pmc_fused_step_ensemble_c4.md") is not None
    assert bench.read_traffic(1, 2) is None          # not profiled: no traffic figure
    assert bench.read_traffic(2, 1) is None
    assert bench.read_traffic(2, 2, 1 << 22) is None  # no summary for this size


def test_traffic_refused_for_other_kernel_sources(tmp_path, monkeypatch):
    """A summary taken on other kernel sources gives no traffic figure."""
    src = os.path.join(ROOT, "profiles", "pmc_fused_step_advection_2p20.md")
    text = open(src).read().replace(bench.kernel_source_hash(), "0" * 16)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "pmc_fused_step_advection_2p20.md").write_text(text)
    h = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.read_traffic(2, 2) is None
    (tmp_path / "profiles" / "pmc_fused_step_advection_2p20.md").write_text(open(src).read())
    assert bench.read_traffic(2, 2) is not None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
