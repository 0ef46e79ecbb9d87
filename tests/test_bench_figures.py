"""CPU: bench.py reports HBM traffic and issue fractions from the committed
rocprofv3 summaries only while the kernel sources hash to the value the
summary records."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_committed_figures_follow_the_source_hash(tmp_path):
    h = bench.kernel_source_hash()
    good = tmp_path / "good.md"
    good.write_text(f"# x\n\n- traffic-bytes-per-launch: 1.5e+09\n- kernel-source-sha256: `{h}`\n")
    assert bench.committed_figures(str(good))["traffic-bytes-per-launch"] == "1.5e+09"
    stale = tmp_path / "stale.md"
    stale.write_text("- traffic-bytes-per-launch: 1.5e+09\n- kernel-source-sha256: `" + "0" * 64 + "`\n")
    assert bench.committed_figures(str(stale)) == {}
    assert bench.committed_figures(str(tmp_path / "missing.md")) == {}


def test_committed_summaries_parse():
    """The committed summaries carry the machine-readable lines bench.py reads."""
    for path, key in ((bench.COUNTERS_FILE, "traffic-bytes-per-launch"), (bench.SQ_FILE, "valu-frac")):
        text = open(path).read()
        assert f"- {key}:" in text and "- kernel-source-sha256:" in text, path
