"""The library's host layer under the thread and the address/undefined-
behaviour sanitizers, driven from four threads at once (one plan per
thread, as the serving loop uses it).

The host layer (argument checks, workspace layout, pair and slot schedules,
internal streams and events, graph caching, the first-launch guard) is
compiled as plain C++ with a host-only stand-in for the HIP runtime and for
the kernel launchers (tests/host_harness/); the stand-in launchers write the
whole extent of every output buffer, so the address sanitizer checks the
layout's offsets and sizes against the allocations.  CPU only.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "host_harness")
CSRC = os.path.join(ROOT, "paper_1801_09263_amd", "csrc")

SANITIZERS = {
    "thread": ["-fsanitize=thread"],
    "address": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                "-fno-omit-frame-pointer"],
}


@pytest.mark.parametrize("kind", list(SANITIZERS))
def test_host_layer_threads_under_sanitizer(tmp_path, kind):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    # the host layer is plain C++; compile a copy under a C++ name
    host_src = tmp_path / "lace_api_host.cpp"
    shutil.copyfile(os.path.join(CSRC, "lace_api.hip"), host_src)
    exe = tmp_path / f"drive_{kind}"
    cmd = [gxx, "-std=c++17", "-O1", "-g", *SANITIZERS[kind],
           "-I", HARNESS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           str(host_src), os.path.join(HARNESS, "stub_runtime.cpp"),
           os.path.join(HARNESS, "stub_launch.cpp"),
           os.path.join(HARNESS, "drive.cpp"), "-o", str(exe), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66",
               ASAN_OPTIONS="detect_leaks=1 exitcode=67")
    r = subprocess.run([str(exe), "4", "2"], capture_output=True, text=True,
                       timeout=300, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "host layer: 4 threads x 2 reps ok" in out
    for bad in ("ThreadSanitizer", "AddressSanitizer", "runtime error",
                "LeakSanitizer"):
        assert bad not in out, out[-4000:]
