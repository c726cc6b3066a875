"""The tiled matrix format of the products, checked on the host (no GPU).

`tests/host/tile_check.cpp` includes the library source, builds the format
from synthetic CSR matrices with the library's own builder and decodes it
independently of the kernels: every matrix entry stored exactly once with its
value bits, padding that adds zero, lane-owned 24-bit lists, distinct rows per
group in 32-bit lists, and a permutation per tile when rows are dealt to the
waves; and the packed arrays built on one host thread and on eight are byte
for byte the same.  Cases: dealt rows, 16 waves over 3 slabs, the 32-bit format, long row
runs with duplicate entries, the contiguous order kept past 2^24 counts, and
2048 rows per wave (11-bit rows, 13-bit columns), and 24 seeded random
schedules across both formats."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tiled_format_round_trips(tmp_path):
    from paper_1601_08201_amd.build import LIB_PATH, compile_flags, hipcc
    if not os.path.exists(LIB_PATH):
        pytest.skip("library not built")
    exe = str(tmp_path / "tile_check")
    cmd = [hipcc()] + [f for f in compile_flags() if f not in ("-fPIC",)] + [
        "-x", "hip", os.path.join(ROOT, "tests", "host", "tile_check.cpp"),
        "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1601_08201_amd", "csrc"),
        "-L" + os.path.dirname(LIB_PATH), "-lsgtv", "-Wl,-rpath," + os.path.dirname(LIB_PATH), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("ok")
    assert out.stdout.count("dealt rows") >= 3 and "contiguous rows" in out.stdout
    assert out.stdout.count("identical with 1 and 8 host threads") == 5
    assert "2048 rows per wave, dealt rows" in out.stdout
    assert out.stdout.count("random ") == 24
