"""bench.py's command-line contract and roofline arithmetic, on the CPU."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")]
                          + list(args), capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_workloads():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("field1024", "volume1920", "grad1024", "batch64", "plain256"):
        assert w in r.stdout


def test_issue_ceiling_and_flop_count():
    # 32 sines/cosines and 32 FMAs per lane plus G matrix-core products per
    # 32 x 32 block, on 1024 SIMDs at 2.4 GHz
    cyc = 32 * 9.03 + 32 * 2.68 + 3 * 36.0
    assert bench.issue_ceiling(3) == pytest.approx(1024 * 2.4e9 * 1024 / cyc)
    assert bench.issue_ceiling(3) == pytest.approx(5.21e12, rel=2e-3)
    assert bench.flops_per_eval(10) == 31
    r = bench.alu_roofline("k", 1e9, 0.5, 4, 10, 3)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(1e9 * 31 / 0.5e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])


def test_profiled_traffic_follows_the_kernel_source(tmp_path):
    # a summary taken on the current kernel source gives its bytes; one
    # taken on other source, an unknown workload or kernel give none
    k = "k_adjoint<3, false>"
    for name, sha in (("now", bench.kernel_source_sha256()), ("old", "0" * 64)):
        (tmp_path / ("wgs_kernels_%s.txt" % name)).write_text(
            "kernels_hip_sha256: %s\ntraffic_bytes_per_launch[%s]: 1.5e8 bytes\n"
            % (sha, k))
    val, src = bench.profiled_traffic("now", k, profiles=str(tmp_path))
    assert val == 1.5e8 and src.endswith("wgs_kernels_now.txt")
    assert bench.profiled_traffic("old", k, profiles=str(tmp_path))[0] is None
    assert bench.profiled_traffic("now", "k_nosuch", profiles=str(tmp_path))[0] is None
    assert bench.profiled_traffic("nosuch", k, profiles=str(tmp_path)) == (None, None)
