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
    # 32 x 32 block, on 1024 SIMDs at 2.4 GHz, with given issue costs
    cost = {"fma": 2.68, "trans": 9.03, "mfma": 36.0}
    cyc = 32 * 9.03 + 32 * 2.68 + 3 * 36.0
    assert bench.issue_ceiling(3, cost) == pytest.approx(1024 * 2.4e9 * 1024 / cyc)
    assert bench.flops_per_eval(10) == 31
    # the roofline's peak: a measured mix ceiling in evaluations/s, in the
    # same algorithmic flops per evaluation as the achieved rate
    r = bench.alu_roofline("k", 1e9, 0.5, 4, 10, 3, ceiling=(4e12, 5))
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(1e9 * 31 / 0.5e-3 / 1e12)
    assert r["peak"] == pytest.approx(4e12 * 31 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"]) == pytest.approx(0.5)
    assert r["frac_of_fp32_vector_peak"] == pytest.approx(r["achieved"] / 157.3)
    # the slot model of the baseline: (D+4)/2 + 1 + 2 r slots per evaluation
    sm = bench.slot_model(1e12, 10, cost)
    assert sm["slots_per_eval"] == pytest.approx(8 + 2 * 9.03 / 2.68)
    assert sm["pct"] == pytest.approx(100 * 1e12 * sm["slots_per_eval"]
                                      / (256 * 64 * 2.4e9))


def test_issue_utilisation_from_counters(tmp_path):
    # a kernel at exactly the irreducible instruction mix for 1024 x 3
    # evaluations per SIMD, timed at that many cycles, is fully utilised
    cost = {"fma": 2.0, "trans": 8.0, "mfma": 32.0}
    k = "k_forward<3, false>"
    evals = 1024 * 1024 * 3.0
    blocks = evals / 1024
    counters = {"SQ_INSTS_VALU": 64 * blocks, "SQ_INSTS_VALU_TRANS_F32": 32 * blocks,
                "SQ_INSTS_MFMA": 3 * blocks}
    cycles_per_simd = 3 * (32 * 8.0 + 32 * 2.0 + 3 * 32.0)
    ms = cycles_per_simd / 2.4e9 * 1e3
    u = bench.issue_utilisation(counters, evals, ms, cost)
    assert u["issue_utilisation"] == pytest.approx(1.0)
    assert u["valu_per_eval"] == pytest.approx(64 / 1024)
    # counters are read from a summary only while its source hash matches
    (tmp_path / "wgs_kernels_w.txt").write_text(
        "kernels_hip_sha256: %s\n| counter | ash::%s | ash::k_reduce |\n"
        "|---|---|---|\n| SQ_INSTS_MFMA | 1.5e+07 | 0 |\n"
        % (bench.kernel_source_sha256(), k))
    got = bench.profiled_counters("w", k, profiles=str(tmp_path))
    assert got == {"SQ_INSTS_MFMA": 1.5e7}
    assert bench.profiled_counters("w", "k_reduce", profiles=str(tmp_path)) == {
        "SQ_INSTS_MFMA": 0.0}
    assert bench.profiled_counters("nosuch", k, profiles=str(tmp_path)) is None


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
