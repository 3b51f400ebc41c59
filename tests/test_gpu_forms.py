"""GPU tests of the execution forms: autotuned kernels, the hipGraph loop, the
serving loop (each result the same alone and in the mix), the update kernel
and the 640-orbital uneven-block workload."""

import numpy as np
import pytest

import synth
from helpers import attach_inputs, device_problem, gate, gpu_available, oracle_full, rel_fro, say
from oracle.workload import OracleProblem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.fail("GPU tests need a visible GPU (run with -m 'not gpu' on CPU)")


def _small(seed=11, degree=2, M=29, sizes=(8, 5, 12, 4)):
    ms = synth.MeshSpec(8, 6, 4, (8.0, 6.0, 4.0), degree)
    wl = synth.custom_workload(ms, M, 2.2, seed, potential="wells")
    wl.colblock_sizes = np.asarray(sizes, dtype=np.int32)
    return wl


def test_autotune_and_graph_loop_match_eager():
    import torch
    from paper_1907_01005_amd import FP32_MFMA, FP64
    from paper_1907_01005_amd.autotune import GraphLoop, tune
    wl = synth.make_workload(1)
    say("autotune + graph")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    dp.apply(FP64)
    dp.overlap()
    torch.cuda.synchronize()
    Y0 = dp.Y.clone()
    S0 = dp.S.clone()
    for prec, tol in ((FP64, 1e-14), (FP32_MFMA, 1e-5)):
        choice = tune(dp, prec, iters=5, warmup=1)
        say(f"tuned {choice.describe()}")
        loop = GraphLoop(dp, choice, n=3)
        for rep in range(3):
            dp.Y.zero_()
            dp.S.zero_()
            torch.cuda.synchronize()
            loop.replay()
            torch.cuda.synchronize()
            eY = (dp.Y - Y0).abs().max().item() / Y0.abs().max().item()
            eS = (dp.S - S0).abs().max().item() / S0.abs().max().item()
            say(f"graph replay {rep} prec={prec}: maxrel Y {eY:.2e} S {eS:.2e}")
            assert eY <= tol and eS <= tol
            # eager work between replays
            dp.apply(FP64)
            dp.overlap()
            torch.cuda.synchronize()
            assert (dp.S - S0).abs().max().item() <= 1e-14 * S0.abs().max().item()


def test_update_kernel_definition():
    import torch
    from paper_1907_01005_amd import FP64
    wl = _small()
    say("update kernel")
    op = OracleProblem(wl, values="generic", value_seed=4)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    dp.apply(FP64)
    S = torch.zeros_like(dp.S)
    S2 = torch.zeros_like(dp.S)
    tr = torch.zeros(2, dtype=torch.float64, device=dp.S.device)
    dp.overlap_into(S, tr[0:1])
    dp.overlap_into(S2, tr[1:2], Y=dp.X)
    torch.cuda.synchronize()
    X0 = dp.X.cpu().numpy()[:dp.nvalues].copy()
    Yh = dp.Y.cpu().numpy()[:dp.nvalues]
    d = np.diag(S.cpu().numpy()) / np.diag(S2.cpu().numpy())
    pat = dp.layout.pattern()
    col = np.empty(dp.nvalues, dtype=np.int64)
    sizes = np.diff(pat["col_block_start"])
    for k, C in enumerate(pat["colidx"]):
        o0, o1 = pat["block_offset"][k], pat["block_offset"][k + 1]
        col[o0:o1] = pat["col_block_start"][C] + np.arange(o1 - o0) % sizes[C]
    tau = 0.07
    expect = X0 - tau * (Yh - X0 * d[col])
    dp.update(S, S2, tau)
    torch.cuda.synchronize()
    got = dp.X.cpu().numpy()[:dp.nvalues]
    assert np.abs(got - expect).max() <= 1e-14 * np.abs(expect).max()
    # X^T X through tmmult equals the plain column dots
    Xd = X0
    for c in range(dp.M):
        assert abs(S2.cpu().numpy()[c, c] - np.sum(Xd[col == c] ** 2)) <= 1e-12 * max(1.0, S2.cpu().numpy()[c, c])


def test_serving_results_same_alone_and_in_mix():
    from paper_1907_01005_amd import FP32_MFMA, FP64
    from paper_1907_01005_amd.serving import GpuExecutor, Request, Server, summarize
    say("serving alone vs mix")
    reqs = []
    shapes = [((8, 8, 8), 2), ((10, 8, 6), 4), ((12, 8, 8), 2), ((8, 6, 6), 4), ((16, 8, 8), 2),
              ((8, 8, 8), 4)]
    for i, (cells, deg) in enumerate(shapes):
        prec = FP64 if i % 2 == 0 else FP32_MFMA
        reqs.append(Request(i, 0.002 * i, cells, deg, 20 + 7 * i, 3.0, prec, 4, 100 + i))
    attach_inputs(reqs)
    ex = GpuExecutor(planner_threads=2, keep_X=True)
    budget = 3 * max(ex.footprint(ex._plan(r)) for r in reqs)   # forces queueing
    mix = Server(ex, byte_budget=budget, max_slots=3).run(reqs)
    s = summarize(mix)
    say(f"mix: {s}")
    assert s["requests_done"] == len(reqs) and mix.max_concurrent >= 2
    for r in reqs:
        alone = Server(GpuExecutor(planner_threads=1, keep_X=True), byte_budget=budget,
                       max_slots=1).run([Request(r.rid, 0.0, r.cells, r.degree, r.M, r.radius,
                                                 r.prec, r.iters, r.seed, inputs=r.inputs)])
        a, b = alone.results[r.rid]["X"], mix.results[r.rid]["X"]
        tol = 1e-12 if r.prec == FP64 else 1e-5
        err = rel_fro(b, a)
        say(f"request {r.rid} prec={r.prec}: alone-vs-mix rel {err:.2e}")
        assert err <= tol


@pytest.mark.parametrize("mesh_index", [0, 1])
def test_uneven_blocks_640_orbitals_full(mesh_index):
    """128x40x40 Q2 / 64x20x20 Q4 (1686177 DoFs), 640 orbitals in uneven column
    blocks: every stored entry of Y, all of S and the trace against one oracle
    pass, after an fp64 and an fp32-MFMA apply; S bitwise on repeat; then the
    autotuned 20-iteration hipGraph loop of apply_H + tmmult in both forms,
    its replay's Y, S and trace against the same oracle result."""
    import torch
    from paper_1907_01005_amd import FP32_MFMA, FP64
    from paper_1907_01005_amd.autotune import GraphLoop, tune
    wl = synth.make_workload(4)
    say(f"640 orbitals mesh {mesh_index}")
    op = OracleProblem(wl, mesh_index)
    dp = device_problem(wl, mesh_index)
    dp.set_X_coo(op.node, op.orb, op.val)
    node, orb = dp.layout.entry_coords()
    Yo, So, tro = oracle_full(op, node, orb)
    say(f"640 orbitals mesh {mesh_index}: oracle done, {len(node)} stored entries")

    def check(tag, tol):
        Yg = dp.Y.cpu().numpy()[:dp.nvalues]
        gate(Yg, Yo, tol, f"{tag} Y")
        gate(dp.S_original_order(), So, tol, f"{tag} S")
        et = abs(float(dp.trace.cpu()[0]) - tro) / abs(tro)
        say(f"{tag} trace rel {et:.2e}")
        assert et <= tol

    for prec, tol in ((FP64, 1e-12), (FP32_MFMA, 1e-5)):
        dp.apply(prec)
        dp.overlap()
        torch.cuda.synchronize()
        check(f"640 orbitals mesh {mesh_index} prec={prec}", tol)
        Sa = dp.S.clone()
        dp.overlap()
        torch.cuda.synchronize()
        assert torch.equal(Sa, dp.S)
    for prec, tol in ((FP64, 1e-12), (FP32_MFMA, 1e-5)):
        choice = tune(dp, prec, iters=5, warmup=1)
        say(f"mesh {mesh_index}: tuned {choice.describe()}")
        loop = GraphLoop(dp, choice, n=20)
        dp.Y.zero_()
        dp.S.zero_()
        dp.trace.zero_()
        torch.cuda.synchronize()
        loop.replay()
        torch.cuda.synchronize()
        check(f"640 orbitals mesh {mesh_index} graph of 20 prec={prec}", tol)


def test_serving_orbital_minimisation_alone_and_in_mix():
    """method "om": steepest descent on the energy inside the serving loop;
    each request's X equal alone and in the mix, its energy decreasing."""
    from paper_1907_01005_amd import FP32_MFMA, FP64
    from paper_1907_01005_amd.serving import GpuExecutor, Request, Server, summarize
    say("serving om")
    shapes = [((8, 8, 8), 2), ((8, 6, 6), 4), ((10, 8, 6), 2), ((8, 8, 4), 4)]
    reqs = attach_inputs([Request(i, 0.002 * i, cells, deg, 16 + 5 * i, 3.0,
                                  FP64 if i % 2 == 0 else FP32_MFMA, 4, 300 + i, "om")
                          for i, (cells, deg) in enumerate(shapes)])
    ex = GpuExecutor(planner_threads=2, keep_X=True)
    budget = 2 * max(ex.footprint(ex._plan(r)) for r in reqs)
    mix = Server(ex, byte_budget=budget, max_slots=3).run(reqs)
    s = summarize(mix)
    say(f"om mix: {s}")
    assert s["requests_done"] == len(reqs) and mix.max_concurrent >= 2
    for r in reqs:
        res = mix.results[r.rid]
        en = res["energies"]
        say(f"om request {r.rid}: tau {res['tau']:.3e} energies {en}")
        assert res["tau"] > 0 and all(b < a for a, b in zip(en, en[1:]))
        # bounded: shifted by 2, the energy of M normalised columns stays O(M)
        assert en[-1] > -20.0 * r.M
        alone = Server(GpuExecutor(planner_threads=1, keep_X=True), byte_budget=budget,
                       max_slots=1).run([Request(r.rid, 0.0, r.cells, r.degree, r.M, r.radius,
                                                 r.prec, r.iters, r.seed, "om",
                                                 inputs=r.inputs)])
        err = rel_fro(res["X"], alone.results[r.rid]["X"])
        say(f"om request {r.rid}: alone-vs-mix rel {err:.2e}")
        assert err <= (1e-12 if r.prec == FP64 else 1e-5)


def test_graph_replays_with_overlap_tasks():
    """apply_H + tmmult captured in a hipGraph on a layout whose dense row
    blocks run as overlap tasks (runs of row blocks, Q1, 16x12x8 cells, 96
    orbitals, radius 6): every replay, with eager work between replays,
    gives the eager Y and S (Y is summed with atomics, so to rounding), and
    an eager overlap of the replay's Y gives the replay's S bitwise (the
    overlap sums in a fixed order)."""
    import numpy as np
    import torch
    from paper_1907_01005_amd import FP64
    sizes = [8, 5, 12, 4, 16, 7, 9, 3, 11, 6, 10, 5]
    ms = synth.MeshSpec(16, 12, 8, (16.0, 12.0, 8.0), 1, 0x3F)
    wl = synth.custom_workload(ms, sum(sizes), 6.0, 5, potential="wells", name="16x12x8-Q1-dense")
    wl.colblock_sizes = np.asarray(sizes, dtype=np.int32)
    say("graph with overlap tasks")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    assert dp.layout.info["tm_tasks"] > 0
    dp.set_X_coo(op.node, op.orb, op.val)
    dp.apply(FP64)
    dp.overlap()
    torch.cuda.synchronize()
    Y0, S0, t0 = dp.Y.clone(), dp.S.clone(), dp.trace.clone()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            dp.apply(FP64)
            dp.overlap()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        dp.Y.zero_()
        dp.S.zero_()
        dp.trace.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        eY = (dp.Y - Y0).abs().max().item() / Y0.abs().max().item()
        eS = (dp.S - S0).abs().max().item() / S0.abs().max().item()
        et = abs(dp.trace.item() - t0.item()) / abs(t0.item())
        Sg, tg = dp.S.clone(), dp.trace.clone()
        dp.overlap()
        torch.cuda.synchronize()
        say(f"replay {rep}: maxrel Y {eY:.2e} S {eS:.2e} trace {et:.2e}")
        assert eY <= 1e-14 and eS <= 1e-13 and et <= 1e-13
        assert torch.equal(dp.S, Sg) and torch.equal(dp.trace, tg)
        dp.apply(FP64)
        dp.overlap()
        torch.cuda.synchronize()


@pytest.mark.parametrize("degree", [2, 4])
def test_overlapped_loop_matches_oracle(degree):
    """The double-buffered step loop (zero fill of the next destination on a
    second stream, mfb_apply_H_acc on the current one) gives the oracle's Y,
    S and trace on every replay, with eager work in between; and
    mfb_apply_H_acc on a zeroed Y equals mfb_apply_H."""
    import torch
    from paper_1907_01005_amd import FP64, apply_H_acc, mv_zero
    from paper_1907_01005_amd.autotune import OverlappedLoop
    wl = _small(degree=degree)
    say(f"overlapped loop Q{degree}")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    node, orb = dp.layout.entry_coords()
    Yo, So, tro = oracle_full(op, node, orb)
    dp.apply(FP64)
    torch.cuda.synchronize()
    Y_plain = dp.Y.clone()
    Yacc = torch.full_like(dp.Y, 7.0)
    mv_zero(dp.layout, Yacc)
    apply_H_acc(dp.mesh, dp.layout, dp.X, Yacc, FP64)
    torch.cuda.synchronize()
    assert (Yacc - Y_plain).abs().max().item() <= 1e-14 * Y_plain.abs().max().item()
    loop = OverlappedLoop(dp, FP64, n=5)
    for rep in range(3):
        loop.replay()
        torch.cuda.synchronize()
        Yg = loop.last_Y.cpu().numpy()[:dp.nvalues]
        gate(Yg, Yo, 1e-12, f"overlapped replay {rep} Y")
        gate(dp.S_original_order(), So, 1e-12, f"overlapped replay {rep} S")
        assert abs(float(dp.trace.cpu()[0]) - tro) <= 1e-12 * abs(tro)
        # eager work between replays (the buffers are shared with it)
        dp.apply(FP64)
        dp.overlap()
        torch.cuda.synchronize()
