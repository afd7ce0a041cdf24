"""bench.py's counter-record check on the CPU: a record's HBM traffic is used only while
the sha256 of the kernel's sources equals the one stored with it; otherwise (or with no
record) the traffic is reported as null."""
import json
import os

import bench


def test_traffic_follows_the_sources(tmp_path, monkeypatch):
    csrc = tmp_path / "csrc"
    prof = tmp_path / "profiles"
    csrc.mkdir()
    prof.mkdir()
    (csrc / "a.hip").write_text("kernel a\n")
    (csrc / "b.h").write_text("header b\n")
    monkeypatch.setattr(bench, "CSRC", str(csrc))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setitem(bench.KERNEL_SOURCES, "probe", ["a.hip", "b.h"])
    assert bench._traffic("probe_rec", "probe") is None              # no record
    rec = {"sources_sha256": bench.sources_sha("probe"), "hbm_bytes_per_launch": 1.25e8}
    (prof / "probe_rec_counters.json").write_text(json.dumps(rec))
    assert bench._traffic("probe_rec", "probe") == 1.25e8
    (csrc / "b.h").write_text("header b, changed\n")                 # a source changed
    assert bench._traffic("probe_rec", "probe") is None


def test_committed_records_name_existing_sources():
    for kernel, names in bench.KERNEL_SOURCES.items():
        for n in names:
            assert os.path.exists(os.path.join(bench.CSRC, n)), (kernel, n)
