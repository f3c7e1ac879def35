"""The request loop's policy core on the CPU.

The core (csrc/asep_server.cpp, which calls no HIP function) is linked with a
test executor that runs every request on the oracle (tests/helpers/
serve_fake.cpp): a memory budget, slow completions, refused shared launches,
few records per quantum.  Through the public calls it checks that every
request of a mixed stream (shifted and sub-lattice schedules, rings and two
lanes, disorder) equals the oracle's run alone, that admission follows
arrival order under back-pressure, that cancelling a queued or a resident
request leaves the others intact, and the BUSY / NOMEM / INVAL paths.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not shutil.which("gcc") or not shutil.which("g++"):
        pytest.skip("gcc/g++ not available")
    d = tmp_path_factory.mktemp("serve")
    orc = str(d / "orc.o")
    exe = str(d / "serve_fake")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-c", os.path.join(ROOT, "oracle", "asep_oracle.c"),
                           "-o", orc])
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-pthread",
                           "-I", os.path.join(ROOT, "paper_1012_0385_amd", "csrc"),
                           "-I", os.path.join(ROOT, "oracle"),
                           os.path.join(ROOT, "tests", "helpers", "serve_fake.cpp"),
                           os.path.join(ROOT, "paper_1012_0385_amd", "csrc", "asep_server.cpp"),
                           orc, "-o", exe, "-lm"])
    return exe


def test_request_loop_policy_on_the_oracle(harness):
    r = subprocess.run([harness], capture_output=True, text=True, timeout=240)
    lines = r.stdout.splitlines()
    failed = [l for l in lines if l.startswith("FAIL")]
    assert r.returncode == 0 and not failed, (failed, r.stderr[-2000:])
    assert lines[-1].startswith("PASSED")
    names = {l.split()[1] for l in lines if l.startswith("OK")}
    for want in ("mix.equals_alone", "mix.shared_launches", "mix.admission_in_arrival_order",
                 "backpressure.admission_order", "cancel.status", "cancel.others", "limits.busy",
                 "limits.nomem", "limits.invalid"):
        assert want in names, want
