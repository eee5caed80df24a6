"""The host C++ of the library (argument checks, handles, tables) built with
AddressSanitizer and UndefinedBehaviorSanitizer on the host side only, linked
with the device objects of the regular build, and driven through its
argument-validation paths on the CPU (tests/sanitize_driver.cpp): any
out-of-bounds access, use after free or undefined behaviour aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2202_00832_amd")
OBJ = os.path.join(PKG, "_build")
DEVICE_OBJS = ["green_theta", "energy_full", "energy_full_lp", "energy_lo", "energy_lo_lp", "energy_hr", "energy_md",
               "residual", "setup"]


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    objs = [os.path.join(OBJ, o + ".o") for o in DEVICE_OBJS]
    if not os.path.exists(hipcc) or not all(os.path.exists(o) for o in objs):
        pytest.skip("needs hipcc and the regular build's objects (python -m paper_2202_00832_amd.build)")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops"]
    host_obj = str(tmp_path / "lofqmc_san.o")
    drv_obj = str(tmp_path / "driver.o")
    exe = str(tmp_path / "driver")
    steps = [
        [hipcc, "-x", "hip", *common, *san, *inc, "-c", os.path.join(PKG, "csrc", "lofqmc.cpp"), "-o", host_obj],
        [hipcc, "-x", "hip", *common, *san, *inc, "-c", os.path.join(ROOT, "tests", "sanitize_driver.cpp"),
         "-o", drv_obj],
        [hipcc, "--offload-arch=gfx950", *san, drv_obj, host_obj, *objs, "-o", exe, "-L", "/opt/rocm/lib",
         "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr
    if shutil.which("nm"):
        syms = subprocess.run(["nm", exe], capture_output=True, text=True).stdout
        assert "__asan_init" in syms and "__ubsan_handle" in syms   # the runtimes are really linked
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK (0 failures)" in r.stdout
