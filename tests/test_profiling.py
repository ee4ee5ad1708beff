"""Host-side checks of the rocprofv3 summary helpers (no GPU)."""
from paper_1903_10977_amd import profiling as P


def _summary(tmp_path, sha, traffic=123456):
    p = tmp_path / "t.txt"
    p.write_text(f"# header\nkernel: k\nkernel_source_sha256: {sha}\ntraffic_bytes_per_launch: {traffic}\n")
    return str(p)


def test_traffic_read_only_for_current_sources(tmp_path):
    assert P.read_traffic(_summary(tmp_path, P.kernel_source_hash())) == 123456
    assert P.read_traffic(_summary(tmp_path, "0" * 16)) is None
    assert P.read_traffic(str(tmp_path / "missing.txt")) is None


def test_committed_traffic_summaries_parse():
    import os
    d = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles")
    for f in os.listdir(d):
        if f.startswith("traffic_"):
            vals = dict(l.split(":", 1) for l in open(os.path.join(d, f)) if ":" in l and not l.startswith("#"))
            assert int(vals["traffic_bytes_per_launch"]) > 0
            assert len(vals["kernel_source_sha256"].strip()) == 16
