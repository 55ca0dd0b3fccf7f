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


def test_merge_roofline_counts_own_pulls_and_live_nodes():
    """The merge kernel's figure: its own pulls (arcs scanned minus the
    scatter's) at 4 + 8W B and the live groups' node slots at 4 + 24W B, over
    the level batches' time minus the scatter launches'."""
    t = dict(scatter_launches=8, kernel_ms=1.0, scatter_ms=0.6, arcs_scanned=5_000_000, scatter_arcs=3_000_000,
             nodes_visited=1_000_000)
    r = bench.merge_roofline([t, t], 2)
    per_launch = (2 * 2_000_000 * 20 + 2 * 1_000_000 * 52) / 16
    assert r["algorithmic_bytes_per_launch"] == int(per_launch)
    assert r["avg_launch_us"] == 50.0
    assert abs(r["achieved"] - per_launch / 50e-6 / 1e9) < 0.1
    assert r["frac"] == round(r["achieved"] / bench.HBM_PEAK_GBS, 4)
    assert bench.merge_roofline([dict(t, kernel_ms=0.6)], 2)["frac"] is None
