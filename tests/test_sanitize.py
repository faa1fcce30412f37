"""The server's host code under AddressSanitizer + UndefinedBehaviorSanitizer and
under ThreadSanitizer, on the CPU (mock executor: no device calls).

Every library source is compiled with the sanitizer on its host code only
(hipcc -Xarch_host -fsanitize=...), linked with tests/sanitize/server_stress.cpp
-- concurrent clients submitting, waiting, cancelling and releasing, several
threads waiting on one ticket and racing to release it, quantum-bounded
launches, destroy with work in flight -- and run; any sanitizer report or
failed check fails the test.  (The race between a release and a concurrent
wait on the same ticket, before releases were refused while a waiter is
inside, showed here as a heap-use-after-free.)
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = {
    "asan": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined"],
    "tsan": ["-Xarch_host", "-fsanitize=thread"],
}


def _build(kind):
    out = os.path.join(ROOT, "_build", f"san_{kind}")
    os.makedirs(out, exist_ok=True)
    csrc = os.path.join(ROOT, "paper_2607_16946_amd", "csrc")
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", csrc] + FLAGS[kind]
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".hip"))
    srcs.append(os.path.join(ROOT, "tests", "sanitize", "server_stress.cpp"))
    procs, objs = [], []
    for s in srcs:
        o = os.path.join(out, os.path.basename(s) + ".o")
        lang = ["-x", "hip"] if s.endswith(".cpp") else []
        procs.append(subprocess.Popen([HIPCC, *common, *lang, "-c", s, "-o", o], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
        objs.append(o)
    for p, s in zip(procs, srcs):
        log = p.communicate()[0]
        assert p.returncode == 0, f"{s}:\n{log}"
    exe = os.path.join(out, "server_stress")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", *FLAGS[kind], "-o", exe, *objs], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["asan", "tsan"])
def test_server_scheduler_under_sanitizers(kind):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = _build(kind)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:second_deadlock_stack=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-6000:]
    assert "server_stress: ok" in r.stdout
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer"):
        assert marker not in report, report[-6000:]
