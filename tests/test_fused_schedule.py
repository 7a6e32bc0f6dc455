"""The fused X-Y pass's work order and wait protocol, checked on the host.

tests/fused_schedule_sim.cpp includes the kernel's own ordering function
(fused_schedule.h) and runs host threads as workgroups with the kernel's
protocol (tickets per queue, consumers wait for all producer items of their
plane, producers publish).  Configurations include the 1024^3 forward and
backward item counts, planes fewer than queues, lags of 0 .. more than the
planes of a queue, and one thread per queue (the tightest case: the only
workgroup of a queue must never wait for work it has not done yet).
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1905_02803_amd", "csrc")


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sim") / "fused_schedule_sim")
    subprocess.run(["/opt/rocm/bin/hipcc", "-x", "hip", "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-I", CSRC, os.path.join(ROOT, "tests", "fused_schedule_sim.cpp"), "-o", exe, "-pthread"],
                   check=True, capture_output=True)
    return exe


@pytest.mark.parametrize("cfg", [
    (1024, 8, 2, 32, 33, 4),   # 1024^3 forward: 32 X items, 33 Y items per plane
    (1024, 8, 2, 33, 32, 4),   # 1024^3 backward: Y first
    (64, 8, 2, 16, 17, 1),     # one workgroup per queue
    (3, 8, 2, 32, 33, 2),      # fewer planes than queues
    (1, 8, 1, 5, 7, 3),
    (20, 8, 0, 4, 3, 2),       # no look-ahead
    (20, 8, 5, 4, 3, 2),       # look-ahead beyond a queue's planes
    (37, 3, 2, 7, 9, 5),
], ids=lambda c: "-".join(map(str, c)))
def test_schedule_and_protocol(sim, cfg):
    r = subprocess.run([sim] + [str(v) for v in cfg] + ["3"], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 timeouts, 0 bad" in r.stdout
