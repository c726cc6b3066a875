"""The order of work of the persistent batched iteration, checked on the host
(no GPU): `tests/host/persistent_check.cpp` runs every workgroup of a launch
as a CPU thread through the same host/device walk the kernel takes (a real
barrier between phases, atomic tile queues) and checks that all of them pass
the same barriers with the right targets, that every tile and block of every
phase is done exactly once per iteration between the right barriers (tiles by
a workgroup of their queue), and that the buffer parities are those of one
launch per step."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_persistent_walk(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "persistent_check")
    subprocess.run([gxx, "-O1", "-std=c++17", "-Wall", "-pthread", "-o", exe,
                    os.path.join(ROOT, "tests", "host", "persistent_check.cpp")], check=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("ok")
    assert out.stdout.count("barriers each") == 9
