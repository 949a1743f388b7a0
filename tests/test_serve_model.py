"""The served form's scheduler (serve_sched.h) on a host-only model of the
device (tests/serve_model.cpp), built with ThreadSanitizer: every request of
the replayed sequences must end, with its expected count, within a bounded
wait, and no data race may be reported.

The sequences are the ones the served form runs on the GPU: saturated
replays of 512 requests followed by Poisson arrivals; 40 requests mixing host
and device texts; many small requests over 16 slots with launch failures
injected; a small budget with rescans, a list that never fits and shutdown
while requests wait for memory."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "serve_model.cpp")


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("serve_model") / "serve_model")
    # clang's ThreadSanitizer runtime intercepts the timed condition-variable
    # waits of libstdc++; fall back to the host compiler without it
    clang = "/opt/rocm/llvm/bin/clang++"
    if os.path.exists(clang):
        cmd = [clang, "-fsanitize=thread"]
    else:
        cmd = [shutil.which("g++") or "g++"]
    cmd += ["-std=c++17", "-O1", "-g", "-pthread", f"-I{ROOT}/include",
            f"-I{ROOT}/paper_1403_1305_amd/csrc", SRC, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


@pytest.mark.parametrize("scenario", ["saturated", "mix", "slots16", "memory"])
@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_every_request_ends(model, scenario, seed):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([model, scenario, str(seed)], capture_output=True, text=True, timeout=240, env=env)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert r.stdout.startswith(f"ok {scenario}"), r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
