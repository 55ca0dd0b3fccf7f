"""Host logic of the benchmark: the counter-pass summary it reads the
measured traffic from (no GPU)."""
import bench

TUNING = {"alpha": 4, "level_blocks": 2048, "scatter_blocks": 4096}


def _summary(tmp_path, digest, tuning="alpha=4,level_blocks=2048,scatter_blocks=4096", value="236840125",
             builder=None):
    builder = bench.source_digest("ccgpu.hip") if builder is None else builder
    p = tmp_path / "pmc.md"
    p.write_text("# counter passes\n\nSummary:\n\n"
                 f"- bfs_batched.hip sha256[:16]: `{digest}`\n"
                 f"- ccgpu.hip sha256[:16]: `{builder}`\n"
                 f"- tuning: `{tuning}`\n"
                 "- FETCH_SIZE scale: 1.9997\n"
                 f"- scaled HBM bytes per launch: {value}\n")
    return str(p)


def test_traffic_read_when_digest_and_knobs_match(tmp_path):
    path = _summary(tmp_path, bench.source_digest())
    assert bench.measured_traffic("rmat20", TUNING, path) == 236840125.0


def test_traffic_dropped_when_source_or_knobs_differ(tmp_path):
    assert bench.measured_traffic("rmat20", TUNING, _summary(tmp_path, "0" * 16)) is None
    # the graph builder decides the hub prefix the kernel gathers over
    assert bench.measured_traffic("rmat20", TUNING, _summary(tmp_path, bench.source_digest(), builder="0" * 16)) is None
    path = _summary(tmp_path, bench.source_digest())
    assert bench.measured_traffic("rmat20", {**TUNING, "alpha": 8}, path) is None
    assert bench.measured_traffic("rmat20", TUNING, _summary(tmp_path, bench.source_digest(), value="n/a")) is None
