"""Host-side checks of bench.py (no GPU needed): the measured-traffic lookup in the
committed counter summaries, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _summary(blocks):
    """A counter summary in the committed format: one fenced block per kernel."""
    out = ["# HBM traffic of a test kernel", ""]
    for name, nbytes, sha in blocks:
        out += ["```", f"kernel: {name}  dispatches: fetch 3, write 3",
                f"hbm_bytes_per_launch: {nbytes:e}", f"kernel_source_sha256_16: {sha}", "```",
                ""]
    return "\n".join(out)


def test_measured_traffic_matches_kernel_and_source_hash(tmp_path, monkeypatch):
    h = bench.kernel_hash()
    path = tmp_path / "t.md"
    path.write_text(_summary([
        ("k_sweep_vec<float, float, 4, 0, false, false, false>", 1.0e9, h),
        ("k_sweep_tb3<float, float, 0, false, 28>", 1.5e9, h),
        ("_ZN12_GLOBAL__N_111k_batch_tb3IDF16_fLi0ELb0ELi24EE", 2.5e9, h),
        ("k_sweep_tb2<float, float, 0, false>", 3.5e9, "0000000000000000"),
    ]))
    monkeypatch.setitem(bench.PROFILE_TRAFFIC, "t", str(path))
    assert bench.measured_traffic("t", "k_sweep_tb3") == 1.5e9
    assert bench.measured_traffic("t", "k_sweep_vec") == 1.0e9
    assert bench.measured_traffic("t", "k_batch_tb3") == 2.5e9    # mangled FP16 name
    assert bench.measured_traffic("t", "k_sweep_tb2") is None     # taken on other source
    assert bench.measured_traffic("t", "k_sweep") is None         # a prefix is not a name
    assert bench.measured_traffic("missing", "k_sweep_tb3") is None


# the kernel bench.py reports for each workload: the FP32 box takes four steps per
# launch, the FP16 box three, the ensemble the batched three-step pass (its tuner may
# also pick the four-step one)
REPORTED = {"box4096_f32": "k_sweep_tb4", "box8192_f16": "k_sweep_tb3",
            "ensemble64_f32": "k_batch_tb3"}


def _has_block(txt, kernel):
    n = len(kernel)
    return f"kernel: {kernel}" in txt or f"kernel: _ZN12_GLOBAL__N_1{n}{kernel}" in txt


def test_committed_summaries_hold_a_block_for_their_kernel():
    """Each committed summary parses and has a block for the kernel bench.py reports
    (its source hash may be older than the working tree's while a kernel is changed)."""
    for workload, path in bench.PROFILE_TRAFFIC.items():
        txt = open(path).read()
        assert _has_block(txt, REPORTED[workload]), path
        assert "kernel_source_sha256_16:" in txt and "hbm_bytes_per_launch:" in txt, path
    for workload, path in bench.PROFILE_VALU.items():
        txt = open(path).read()
        assert _has_block(txt, REPORTED[workload]), path
        assert "valu_active_quad_cycles_per_launch:" in txt, path


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr
