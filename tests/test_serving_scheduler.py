"""Scheduler of the serving loop, on the CPU with a fake byte-counting executor."""

import pytest

from paper_1907_01005_amd.serving import FakeExecutor, Request, Server, request_stream, summarize


def _req(i, t, M, iters=10):
    return Request(i, t, (16, 16, 16), 2, M, 4.0, 0, iters, i)


def test_budget_and_slots_are_respected():
    reqs = [_req(i, 0.001 * i, M) for i, M in enumerate([300, 300, 300, 100, 500, 50, 50])]
    ex = FakeExecutor(bytes_of=lambda r: r.M * 1000, seconds_of=lambda r: 0.05)
    rep = Server(ex, byte_budget=700_000, max_slots=3).run(reqs, realtime=False)
    assert ex.max_live <= 700_000
    assert rep.max_concurrent <= 3
    assert len(rep.results) == len(reqs)
    # FIFO admission: requests start in arrival order
    starts = [rid for kind, rid, _ in ex.events if kind == "start"]
    assert starts == sorted(starts)
    # requests that arrive while others run are admitted before those finish
    # (continuous batching), as soon as bytes allow
    t_start = {rid: t for kind, rid, t in ex.events if kind == "start"}
    t_fin = {rid: t for kind, rid, t in ex.events if kind == "finish"}
    assert t_start[1] < t_fin[0]


def test_oversized_request_is_rejected_not_blocking():
    reqs = [_req(0, 0.0, 100), _req(1, 0.0, 5000), _req(2, 0.0, 100)]
    ex = FakeExecutor()
    rep = Server(ex, byte_budget=1_000_000, max_slots=4).run(reqs, realtime=False)
    assert rep.results[1].get("rejected")
    assert not rep.results[0].get("rejected") and not rep.results[2].get("rejected")


def test_memory_is_released_and_queue_drains():
    reqs = [_req(i, 0.0, 400) for i in range(6)]
    ex = FakeExecutor(seconds_of=lambda r: 0.02)
    rep = Server(ex, byte_budget=800_000, max_slots=8).run(reqs, realtime=False)
    assert ex.live_bytes == 0
    assert rep.max_concurrent == 2
    s = summarize(rep)
    assert s["requests_done"] == 6 and s["apply_ms_p50"] == 1.0


def test_request_stream_recipe():
    rs = request_stream(n=96, rate=40.0, seed=5)
    assert len(rs) == 96
    arr = [r.arrival for r in rs]
    assert arr == sorted(arr)
    assert 1.0 < arr[-1] < 5.0                  # 96 arrivals at 40/s
    assert all(32 <= r.M <= 640 for r in rs)
    assert all(3.0 <= r.radius <= 5.0 for r in rs)
    assert {r.degree for r in rs} == {2, 4}


def test_apply_overlap_intervals():
    """Overlap of apply intervals: union, sum and the time two requests run
    together, on hand-made intervals."""
    from paper_1907_01005_amd.serving import apply_overlap
    r = apply_overlap([(0.0, 2.0, 1), (1.0, 3.0, 2), (5.0, 6.0, 1), (5.5, 5.75, 1)])
    assert r["apply_union_s"] == pytest.approx(4.0)
    assert r["apply_sum_s"] == pytest.approx(5.25)
    # request 1's two intervals overlapping each other are not concurrency
    assert r["apply_concurrent_s"] == pytest.approx(1.0)
    assert r["apply_concurrent_frac"] == pytest.approx(0.25)


def test_trace_overlap_csv(tmp_path):
    """The kernel-trace summary of the bench: library kernels only, overlap
    counted across streams."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "bench_mod", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    rows = [("mfb::gpu::a", 0, 100, 1), ("mfb::gpu::b", 50, 150, 2), ("other", 0, 1000, 3),
            ("mfb::gpu::c", 120, 130, 2), ("mfb::gpu::d", 200, 300, 1)]
    p = tmp_path / "kernel_trace.csv"
    with open(p, "w") as f:
        f.write("Kernel_Name,Stream_Id,Start_Timestamp,End_Timestamp\n")
        for n, a, b, sid in rows:
            f.write(f"{n},{sid},{a},{b}\n")
    r = bench.trace_overlap(str(p))
    assert r["kernels"] == 4 and r["streams"] == 2
    assert r["busy_union_ms"] == pytest.approx(250e-6)
    assert r["kernel_sum_ms"] == pytest.approx(310e-6)
    assert r["concurrent_ms"] == pytest.approx(50e-6)
    assert r["most_streams_at_once"] == 2
