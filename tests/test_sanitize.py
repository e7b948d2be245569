"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/sanitize/host_check.cpp drives the planner, the lane-split lowering,
the Hamiltonian tables with their window cover and the cutoff rules on
random and structured inputs.  The sanitizers instrument host code only
(each -fsanitize= goes to the host pass); the device code is compiled as in
the library and never runs: none of the calls exercised touches a device."""
import os
import subprocess

import pytest

from paper_2402_11878_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def test_host_code_under_sanitizers(tmp_path):
    try:
        cc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    flags = [f for f in B.common_flags() if f != "-O3"] + ["-O1"] + SAN
    srcs = [os.path.join(B.CSRC, s) for s in B.SOURCES] + [os.path.join(ROOT, "tests", "sanitize", "host_check.cpp")]
    procs, objs = [], []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src).replace(".", "_") + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([cc, *flags, "-x", "hip", "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for src, p in zip(srcs, procs):
        out, _ = p.communicate(timeout=900)
        assert p.returncode == 0, (src, out.decode(errors="replace")[-3000:])
    exe = str(tmp_path / "host_check")
    r = subprocess.run([cc, f"--offload-arch={B.ARCH}", *SAN, *objs, "-lhiprtc", "-o", exe],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    syms = subprocess.run(["nm", exe], capture_output=True, text=True).stdout
    assert "__asan_init" in syms and "__ubsan_handle" in syms      # both runtimes are in
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "host checks passed" in r.stdout
