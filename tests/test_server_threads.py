"""The solve server's threads on the CPU: the server (its scheduler, worker
threads and set-up cache), the device-memory cache and the C-ABI glue are
compiled with g++ against a host-only stand-in of the HIP runtime, with the
set-up and solve replaced by stubs that sleep and touch their buffers, and
driven by thousands of requests under ThreadSanitizer and under
AddressSanitizer/UBSan.  A data race, a use after free or an overflow in
the server's hand-over of requests and cached set-ups fails the test.
The same host build checks the opt-in crash report (IBM_CRASH_TRACE): a
store through a null pointer in a thread of the host program must print the
signal and a native stack and still end the process by SIGSEGV.
No GPU is used."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2605_04335_amd", "csrc")
STUB = os.path.join(HERE, "server_host")


def _build(tmp_path, san):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path / ("drive_" + (san or "plain").replace(",", "_")))
    srcs = [os.path.join(CSRC, "server.hip"), os.path.join(CSRC, "memory.hip"), os.path.join(CSRC, "capi.hip"),
            os.path.join(STUB, "stubs.cpp"), os.path.join(STUB, "drive.cpp")]
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer"] + (["-fsanitize=" + san] if san else []) + [
        "-I", STUB, "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    for s in srcs:
        cmd += ["-x", "c++", s]
    cmd += ["-o", out, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _run(exe, args, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True, timeout=300, env=env)
    return r


# (requests, arrivals per second, budget MB, cached set-ups): admission bound,
# cache hits and evictions; no cache; a large cache
CASES = [(2000, 3000, 24, 8), (1500, 8000, 16, 2), (1500, 2000, 200, 0)]


def test_server_threads_tsan(tmp_path):
    exe = _build(tmp_path, "thread")
    for c in CASES:
        r = _run(exe, c, {"TSAN_OPTIONS": "halt_on_error=1 second_deadlock_stack=1"})
        assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-6000:]
        assert r.returncode == 0, (c, r.stdout[-2000:], r.stderr[-4000:])
        assert "failed 0" in r.stdout, r.stdout


def test_server_threads_asan_ubsan(tmp_path):
    exe = _build(tmp_path, "address,undefined")
    for c in CASES:
        r = _run(exe, c, {"ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "halt_on_error=1"})
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
        assert r.returncode == 0, (c, r.stdout[-2000:], r.stderr[-4000:])
        assert "failed 0" in r.stdout, r.stdout


def test_crash_trace_reports_and_passes_the_signal_on(tmp_path):
    import signal
    exe = _build(tmp_path, None)
    r = _run(exe, ["crash", 0], {"IBM_CRASH_TRACE": "1"})
    assert r.returncode == -signal.SIGSEGV, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "[ibm] fatal signal %d at address 0x0 in thread " % signal.SIGSEGV in r.stderr, r.stderr[-4000:]
    # backtrace_symbols_fd names the executable in each frame of the stack
    assert sum(1 for line in r.stderr.splitlines() if os.path.basename(exe) in line) >= 2, r.stderr[-4000:]
    assert "no crash" not in r.stdout
    # without the variable the handler is not installed: the plain default action
    r = _run(exe, ["crash", 0], {})
    assert r.returncode == -signal.SIGSEGV and "[ibm] fatal signal" not in r.stderr, r.stderr[-2000:]
