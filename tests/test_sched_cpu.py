"""The solve server's scheduling policy on the CPU (no GPU): the host-only
policy header driven by a fake engine, built with g++ plainly and under
ThreadSanitizer.  Scenarios: an idle engine holder and a submit to another
matrix under a one-engine budget (the interleaving is forced through the
policy's wait hooks), turns under a one-engine budget, a request alone and in
a mix, random load from two client threads, shutdown with work in flight.
The serving model is Section 2.2's: independent realizations sharing one
operator, arriving as separate solves."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "sched_fake_engine.cpp")
INC = [os.path.join(ROOT, "paper_1711_10622_amd", "csrc"), os.path.join(ROOT, "include")]


def _build(tmp_path, extra):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "sched_fake_engine")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-pthread", "-Wall", *extra,
           *[f"-I{d}" for d in INC], SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


@pytest.mark.parametrize("variant", ["plain", "tsan"])
def test_server_policy_on_fake_engine(tmp_path, variant):
    extra = ["-fsanitize=thread"] if variant == "tsan" else []
    exe = _build(tmp_path, extra)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert out.count("PASS") == 5 and "ThreadSanitizer" not in out, out[-6000:]
