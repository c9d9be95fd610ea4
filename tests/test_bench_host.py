"""Host logic of bench.py that needs no GPU: the one-GPU refusal and the counter-traffic record,
which bench.py reports only while it was taken on the same kernel and the current source."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 1" in r.stderr
    assert r.stdout == ""  # no JSON line for a run that did not happen


@pytest.mark.parametrize("kernel", ["forward", "backward"])
def test_committed_traffic_records_match_the_kernel_sources(kernel):
    path = os.path.join(ROOT, "profiles", "hbm_traffic_%s_fp32_mfma3_32x32_Ltau160.md" % kernel)
    rec = [json.loads(l[len("traffic_json:"):]) for l in open(path) if l.startswith("traffic_json:")]
    assert len(rec) == 1
    rec = rec[0]
    assert rec["source"] == "paper_2510_13866_amd/csrc/" + bench.KERNEL_SOURCES[kernel]["fp32_mfma3"]
    name = rec["kernel"].split("<")[0]
    got = bench.measured_traffic(kernel, "fp32_mfma3", name)
    if rec["source_sha256"] == bench.source_sha(bench.KERNEL_SOURCES[kernel]["fp32_mfma3"]):
        assert got == rec["fetch_bytes"] + rec["write_bytes"]
        assert got > 0
    else:
        assert got is None
    # a record of another kernel is never reported
    assert bench.measured_traffic(kernel, "fp32_mfma3", "k_not_this_kernel") is None


def test_traffic_record_is_dropped_after_a_source_change(monkeypatch):
    monkeypatch.setattr(bench, "source_sha", lambda name: "0000000000000000")
    assert bench.measured_traffic("forward", "fp32_mfma3", "k_forward_mfma2") is None
    assert bench.measured_traffic("backward", "fp32_mfma3", "k_backward_win") is None


def test_no_traffic_without_a_record():
    # the FFT path has no committed counter record
    assert bench.measured_traffic("forward", "fp32", "k_forward_fft") is None
