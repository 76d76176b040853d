"""The HBM traffic that bench.py reports is tied to the kernel sources'
code: a change of comments or whitespace keeps it, a change of code turns it
into null (host only)."""
import os
import shutil

import bench


def _copy_sources(tmp_path):
    for f in bench.TRAFFIC_SOURCES:
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, f), dst)
    return str(tmp_path)


def test_comment_edits_keep_the_hash(tmp_path):
    root = _copy_sources(tmp_path)
    h0 = bench.sources_sha1(root)
    f = os.path.join(root, bench.TRAFFIC_SOURCES[0])
    text = open(f).read()
    text = text.replace("\n", "\n// an added comment line\n", 1) + "\n/* a trailing\n   block comment */\n"
    open(f, "w").write(text.replace("  ", "    ", 3))
    assert bench.sources_sha1(root) == h0


def test_code_edits_change_the_hash(tmp_path):
    root = _copy_sources(tmp_path)
    h0 = bench.sources_sha1(root)
    f = os.path.join(root, bench.TRAFFIC_SOURCES[1])
    open(f, "a").write("\nstatic int an_added_function() { return 1; }\n")
    assert bench.sources_sha1(root) != h0


def test_traffic_is_tied_to_its_schedule(monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC", {"sources_sha1": bench.sources_sha1(), "river": {"4:1": 7, "3:1": 8},
                                           "batch": {"4:1": 5, "4:2": 6}})
    assert bench.measured_traffic("batch", (4, 1)) == 5
    assert bench.measured_traffic("batch", (4, 2)) == 6
    assert bench.measured_traffic("batch", (3, 8)) is None
    assert bench.measured_traffic("river", (4, 1)) == 7
    assert bench.measured_traffic("river", (3, 1)) == 8
    assert bench.measured_traffic("river", (2, 1)) is None
    monkeypatch.setattr(bench, "TRAFFIC", {"sources_sha1": "0" * 40, "river": {"4:1": 7}, "batch": {"4:2": 6}})
    assert bench.measured_traffic("batch", (4, 2)) is None
    assert bench.measured_traffic("river", (4, 1)) is None
