"""The committed HBM counter summary is keyed on the product kernels' code,
the host builder of the tiled format and the schedule: an edit of comments or
white space keeps it valid, an edit of code or another schedule does not
(CPU only)."""
import importlib.util
import os
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = ("sgtv_tiled.hip", "sgtv_device.h", "sgtv_kernels.h", "sgtv_api.hip")


@pytest.fixture()
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def copy_tree(tmp_path):
    dst = tmp_path / "paper_1601_08201_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in FILES:
        shutil.copy(os.path.join(ROOT, "paper_1601_08201_amd", "csrc", f), dst / f)
    return dst


def test_committed_summary_is_readable(bench):
    """The summary holds a 64-hex key and per-product bytes; bench reads them
    back while the key matches the kernels (else it reports no traffic)."""
    import json
    import re
    text = open(os.path.join(ROOT, "profiles", "tiled_product_fp32_paper_scan.md")).read()
    rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
    assert re.fullmatch(r"[0-9a-f]{64}", rec["kernel_source_sha256"])
    for k in ("forward", "back"):
        assert 0.8e9 < rec["traffic_bytes_per_launch"][k] < 1.2e9
        got = bench.measured_traffic(k, "f32", "tiled", "paper", rec.get("schedule"))
        if rec["kernel_source_sha256"] == bench.kernel_fingerprint(rec.get("schedule")):
            assert got == rec["traffic_bytes_per_launch"][k]
        else:
            assert got is None


def test_comments_do_not_change_the_fingerprint(bench, tmp_path, monkeypatch):
    ref = bench.kernel_fingerprint()
    dst = copy_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_fingerprint() == ref
    p = dst / "sgtv_kernels.h"
    p.write_text("// a new comment line\n/* and a block\n   comment */\n" + p.read_text().replace("\n", "\n\n"))
    assert bench.kernel_fingerprint() == ref
    p = dst / "sgtv_tiled.hip"
    p.write_text(p.read_text().replace("kXPrefetch = 4", "kXPrefetch = 2"))
    assert bench.kernel_fingerprint() != ref


def test_builder_and_schedule_change_the_fingerprint(bench, tmp_path, monkeypatch):
    dst = copy_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    ref = bench.kernel_fingerprint({"waves": 16})
    assert bench.kernel_fingerprint({"waves": 8}) != ref
    p = dst / "sgtv_api.hip"
    text = p.read_text()
    assert "16380" in text[text.find("TileParams choose_tiles("):text.find("struct System {")]
    p.write_text(text.replace("std::min<int64_t>(16380,", "std::min<int64_t>(16376,", 1))
    assert bench.kernel_fingerprint({"waves": 16}) != ref
