"""Host-only code under the address and undefined-behaviour sanitizers.

The principal-mode rotation (csrc/principal.cpp) and the set-up argument
checks (csrc/validate.cpp) are plain C++ with no device code; each is built
here with g++ alone and both sanitizers, together with a driver
(tests/host/*_driver.cpp) that exercises several shapes and the error
paths.  Any sanitizer report fails the test.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_principal_modes_under_asan_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "principal_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "principal_driver.cpp"),
           os.path.join(ROOT, "paper_2505_08777_amd", "csrc", "principal.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stdout[-400:])
    env = dict(os.environ)
    # the sanitizer runtime need not come first among preloaded libraries
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:verify_asan_link_order=0"
    run = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                         text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout[-2000:]
    assert "principal driver ok" in run.stdout
    assert "runtime error" not in run.stdout and "ERROR:" not in run.stdout


def test_argument_checks_under_asan_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "validate_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "validate_driver.cpp"),
           os.path.join(ROOT, "paper_2505_08777_amd", "csrc", "validate.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stdout[-400:])
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:verify_asan_link_order=0"
    run = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                         text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout[-2000:]
    assert "validate driver ok" in run.stdout
    assert "runtime error" not in run.stdout and "ERROR:" not in run.stdout
