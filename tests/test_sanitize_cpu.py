"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host C/C++
code, run on the CPU: the FP64 oracle (FP, BP, SART with one and several
projections per update, the CSR build; hollow, one-sector, ragged and posed
scans), the host half of pose estimation (point tracking, pose from the axis,
azimuthal phase) and the host set-up of the library (argument checks of
cyl_geom_create and a well-formed call up to the device query).  Built with
gcc/g++ only: the device code is not part of these programs."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
HIP_INC = "/opt/rocm/include"


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_san")
    subprocess.check_call(["gcc"] + SAN + [os.path.join(ROOT, "tests/sanitize/oracle_driver.c"), "-o", exe,
                                           "-lm", "-lpthread"])
    assert "ok" in _run(exe)


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(HIP_INC), reason="needs g++ and the HIP headers")
def test_pose_host_under_sanitizers(tmp_path):
    exe = str(tmp_path / "pose_san")
    subprocess.check_call(["g++", "-std=c++17"] + SAN + [
        "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INC, "-I" + os.path.join(ROOT, "include"),
        "-I" + os.path.join(ROOT, "paper_2005_11976_amd/csrc"),
        os.path.join(ROOT, "tests/sanitize/pose_driver.cpp"),
        os.path.join(ROOT, "paper_2005_11976_amd/csrc/cyl_pose.cpp"), "-o", exe])
    assert "ok" in _run(exe)


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists("/opt/rocm/lib/libamdhip64.so"),
                    reason="needs g++ and the HIP runtime")
def test_host_setup_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_san")
    subprocess.check_call(["g++", "-std=c++17"] + SAN + [
        "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INC, "-I" + os.path.join(ROOT, "include"),
        "-I" + os.path.join(ROOT, "paper_2005_11976_amd/csrc"),
        os.path.join(ROOT, "tests/sanitize/host_driver.cpp"),
        os.path.join(ROOT, "paper_2005_11976_amd/csrc/cyl_host.cpp"), "-o", exe,
        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    assert "ok" in _run(exe)
