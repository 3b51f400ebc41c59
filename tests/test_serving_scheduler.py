"""Scheduler of the serving loop, on the CPU with a fake byte-counting executor."""

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
