"""The native server's scheduling core under ThreadSanitizer, on the CPU.

rt_serve.cpp is compiled unchanged against a simulated device
(tests/serve_stub: a stand-in HIP header, streams run by worker threads,
events as stream positions, a "kernel" that writes each job's image from its
request) with g++ -fsanitize=thread, and driven by several client threads
through admission against a small image pool, first-come-first-served
launches, submits that launch from the caller's thread, waits, releases,
rejections and both shutdown paths.  The run must report no data race and no
failed check."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STUB = os.path.join(ROOT, "tests", "serve_stub")


def test_server_core_under_thread_sanitizer(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "serve_tsan")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
           "-I", os.path.join(STUB, "include"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1211_5595_amd", "csrc"),
           os.path.join(ROOT, "paper_1211_5595_amd", "csrc", "rt_serve.cpp"),
           os.path.join(STUB, "stub_device.cpp"), os.path.join(STUB, "driver.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert "ok: 0 failed checks" in r.stdout
