"""The request loop's policy core on the CPU.

The core (csrc/asep_server.cpp, which calls no HIP function) is linked with a
test executor that runs every request on the oracle (tests/helpers/
serve_fake.cpp): a memory budget, slow completions, refused shared launches,
few records per quantum.  Through the public calls it checks that every
request of a mixed stream (shifted and sub-lattice schedules, rings and two
lanes, disorder) equals the oracle's run alone, that admission follows
arrival order under back-pressure, that cancelling a queued or a resident
request leaves the others intact, that quanta are cut to the executor's
limit, that requests of one shape share launches, the BUSY / NOMEM / INVAL
paths, and several client threads at once.  The same program is also built
with ThreadSanitizer (host code only, clang's runtime) and must report no
race: the worker calls the executor without holding the server's lock.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


CHECKS = ("mix.equals_alone", "mix.shared_counted", "mix.admission_in_arrival_order",
          "backpressure.admission_order", "cancel.status", "cancel.others", "limits.busy",
          "limits.nomem", "limits.invalid", "packing.shared_launches", "quantum.clamped",
          "quantum.schedule_echoed", "concurrent.all_requests")


def _sources():
    return [os.path.join(ROOT, "tests", "helpers", "serve_fake.cpp"),
            os.path.join(ROOT, "paper_1012_0385_amd", "csrc", "asep_server.cpp")]


def _includes():
    return ["-I", os.path.join(ROOT, "paper_1012_0385_amd", "csrc"), "-I", os.path.join(ROOT, "oracle")]


def _check_output(r):
    lines = r.stdout.splitlines()
    failed = [l for l in lines if l.startswith("FAIL")]
    assert r.returncode == 0 and not failed, (failed, r.stderr[-3000:])
    assert lines[-1].startswith("PASSED")
    names = {l.split()[1] for l in lines if l.startswith("OK")}
    for want in CHECKS:
        assert want in names, want


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not shutil.which("gcc") or not shutil.which("g++"):
        pytest.skip("gcc/g++ not available")
    d = tmp_path_factory.mktemp("serve")
    orc = str(d / "orc.o")
    exe = str(d / "serve_fake")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-c", os.path.join(ROOT, "oracle", "asep_oracle.c"),
                           "-o", orc])
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-pthread"] + _includes() +
                          _sources() + [orc, "-o", exe, "-lm"])
    return exe


def test_request_loop_policy_on_the_oracle(harness):
    _check_output(subprocess.run([harness], capture_output=True, text=True, timeout=240))


# GCC 11's ThreadSanitizer runtime does not intercept pthread_cond_clockwait
# (libstdc++'s steady-clock waits), which makes every timed wait look like a
# lock held across it; the ROCm toolchain's clang runtime does.
CLANG = "/opt/rocm/llvm/bin/clang"


def test_request_loop_under_thread_sanitizer(tmp_path):
    if not (os.path.exists(CLANG) and os.path.exists(CLANG + "++")):
        pytest.skip("clang with a ThreadSanitizer runtime not available")
    orc = str(tmp_path / "orc_tsan.o")
    exe = str(tmp_path / "serve_fake_tsan")
    tsan = "-fsanitize=thread"
    subprocess.check_call([CLANG, "-O1", "-g", "-std=c11", tsan, "-c",
                           os.path.join(ROOT, "oracle", "asep_oracle.c"), "-o", orc])
    subprocess.check_call([CLANG + "++", "-O1", "-g", "-std=c++17", "-pthread", tsan] +
                          _includes() + _sources() + [orc, "-o", exe, "-lm"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    _check_output(r)
