"""The library's host-only code -- cut-map validation, the contraction
planner, the cut search and the batch set-up of the C ABI (abi.cpp, plan.cpp,
cutmap.cpp, cutfind.cpp) -- built with AddressSanitizer and
UndefinedBehaviorSanitizer and driven on generated valid and malformed
inputs (tests/host_sanitize/driver.cpp).  Device launchers are replaced by
stubs that report no device (tests/host_sanitize/stubs.cpp), so every call
runs its host logic and then its error path.  A sanitizer report aborts the
driver and fails the test.  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_05836_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "host_sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no host C++ compiler or HIP headers")
    flags = ["-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, "-I", "/opt/rocm/include"] + SAN
    srcs = [os.path.join(CSRC, f) for f in ("abi.cpp", "plan.cpp", "cutmap.cpp", "cutfind.cpp")]
    srcs += [os.path.join(HERE, f) for f in ("stubs.cpp", "driver.cpp")]
    procs, objs = [], []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([cxx] + flags + ["-c", src, "-o", obj], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
    for p, src in zip(procs, srcs):
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, f"compile {src}:\n{out[-3000:]}"
    exe = str(tmp_path / "driver")
    r = subprocess.run([cxx] + SAN + ["-o", exe] + objs + ["-L/opt/rocm/lib", "-lamdhip64",
                                                            "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
    lines = r.stdout.splitlines()
    assert lines[-1] == "done", r.stdout
    valid = int(lines[0].split()[2])
    solved = int(lines[1].split()[2])
    assert valid > 500 and solved > 50, r.stdout  # the generators reach the valid paths
