#!/usr/bin/env python3
"""Benchmark of the hot path: Y = mask(H X) (apply_H) then S = X^T Y, tr S.

One step = one pass of the whole path over the resident multivector of the
paper-scale quadratic workload (64x40x40 Q2 cells, 846369 DoFs, 320 orbitals
in 40 column blocks of 8, support radius 4 cells).  The K timed steps run as
one hipGraph of K steps (the kernels of every step, no host launch per
kernel); an eager loop with events around each launch gives the per-launch
latencies and the roofline figures.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp64|fp64-mfma|fp32|fp32-mfma]
                    [--config 2|3] [--kernel 0|1|2|7|8] [--no-cpu-baseline] [--no-forms]
                    [--no-q4] [--no-config4] [--serve N]

Without --no-forms the line also carries the other precision forms, the energy
and descent step, hipGraph loops, curved cells, the Q4 workload with its own
roofline, the 640-orbital workloads' hipGraph loops and a short serving stream.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector (= FP64 matrix)
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X FP32 matrix
PRECS = {"fp64": 0, "fp64-mfma": 1, "fp32-mfma": 2, "fp32": 3}


def flops_per_cell_column(p: int) -> int:
    """Sum-factorised cell operator: 12 one-dimensional sweeps of n^4 multiply-adds
    (S and D forward/backward along three axes) plus 7 n^3 scaling/adds."""
    n = p + 1
    return 24 * n ** 4 + 7 * n ** 3


def algorithmic(dp, degree: int):
    """Bytes and flops one apply_H must move / perform on this layout."""
    info = dp.layout.info
    E = dp.nvalues
    n3 = (degree + 1) ** 3
    # (batch, C) pairs whose own row block is stored are the ones whose
    # gathered values are non-zero for orbital-supported inputs
    own = info["apply_pairs_own"]
    sizes = np.diff(dp.layout.pattern()["col_block_start"])
    pat = dp.layout.pattern()
    widths = sizes[pat["colidx"]]                     # |C| of each stored block
    cell_cols = 8 * int(widths.sum())                 # 8 cells x |C| per own pair
    active_batches = int(np.count_nonzero(np.diff(pat["rowptr"])))
    bytes_ = 16 * E + 8 * n3 * 8 * active_batches
    flops = flops_per_cell_column(degree) * cell_cols
    return {"E": E, "bytes": bytes_, "flops": flops, "own_pairs": own,
            "cell_columns": cell_cols, "active_batches": active_batches}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, budget_s: float = 12.0, one_thread: bool = False):
    """The oracle's whole step (apply + overlap) timed on the host cores (or on
    one thread), repeated for about budget_s seconds."""
    from oracle.workload import OracleProblem
    if one_thread:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            rec = cpu_baseline(wl, budget_s)
        rec["cores"] = 1
        rec["sample"] = rec["sample"].replace(" s on ", " s on one thread of ")
        return rec
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    op = OracleProblem(wl)
    # whole steps (masked apply of every column block, then S = X^T Y and its
    # trace), repeated until the budget is spent
    t0 = time.perf_counter()
    steps = 0
    while True:
        S, tr = op.overlap()
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    entries = stored_entries(op) * steps
    return {"value": entries / dt / 1e9, "unit": "GDoF*cols/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{steps} whole steps of the oracle (masked apply of all {op.pattern.ncb} "
                      f"column blocks with element matrices built on the fly, then S = X^T Y and "
                      f"its trace; {entries // steps} stored entries each), {dt:.1f} s on "
                      f"{os.cpu_count()} visible host cores ({cpu_model()})"}


def stored_entries(op) -> int:
    """Stored entries of the oracle's pattern: rows of each stored block x its width."""
    rows = op.pattern.rb_start[1:] - op.pattern.rb_start[:-1]
    total = 0
    for C in range(op.pattern.ncb):
        k = np.nonzero(op.pattern.colidx == C)[0]
        rb = np.searchsorted(op.pattern.rowptr, k, side="right") - 1
        total += int(rows[rb].sum()) * len(op.block_orbitals(C))
    return total


def measured_traffic(workload: str, prec: str):
    """HBM bytes per apply_H launch from the committed counter summary, or None
    when the kernel source has changed since the counters were taken."""
    import hashlib
    src = os.path.join(ROOT, "paper_1907_01005_amd", "csrc", "kernels.hip")
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if not digest.startswith(rec.get("kernel_sha256_prefix", "-")) or rec.get("prec") != prec:
        return None
    return rec.get("apply_H_bytes_per_launch")


def copy_bandwidth(mib: int = 1024, reps: int = 5) -> float:
    """Device-to-device copy rate in GB/s (bytes read + bytes written), the
    practical HBM ceiling the apply's byte rate is also compared with."""
    import torch
    src = torch.ones(mib << 17, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    t = a.elapsed_time(b) * 1e-3 / reps
    gbs = 2 * src.numel() * 8 / t / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def fp64_fma_rate(reps: int = 5) -> float:
    """TFLOP/s of the library's fp64 FMA probe (16 independent chains per
    thread, 8 workgroups of 256 threads per CU): the fp64 vector-ALU rate this
    device reaches, beside the 78.6 TF/s it is rated at."""
    import torch
    from paper_1907_01005_amd import api
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    blocks, iters = 8 * cus, 20000
    api.probe_fp64_fma(out, blocks, iters)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        flops = api.probe_fp64_fma(out, blocks, iters)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b) * 1e-3)
    return flops / float(np.median(ts)) / 1e12


def build_problem(cfg: int, mesh_index: int = 0, radius: float = 0.0, bend: float = 0.0):
    """The seeded workload of configuration `cfg` on the GPU; radius > 0 replaces the
    support radius (same centres, potential and blocks; a different workload); bend > 0
    bends the cells (curved-cell form, amplitude in cell widths)."""
    import dataclasses
    import synth
    from paper_1907_01005_amd.problem import DeviceProblem
    wl = synth.make_workload(cfg)
    if radius > 0:
        wl = dataclasses.replace(wl, radius=float(radius), name=f"{wl.name}-r{radius:g}")
    if bend > 0:
        meshes = list(wl.meshes)
        meshes[mesh_index] = dataclasses.replace(meshes[mesh_index], bend=float(bend))
        wl = dataclasses.replace(wl, meshes=meshes, name=f"{wl.name}-bent{bend:g}")
    ms = wl.meshes[mesh_index]
    dp = DeviceProblem((ms.nx, ms.ny, ms.nz), ms.L, ms.degree, ms.dirichlet, wl.centres,
                       wl.radius, wl.colblock_sizes, lambda P: synth.potential_at(wl, P),
                       node_map=ms.bend_points if ms.bend else None)
    node, orb, val = synth.orbital_values(wl, mesh_index)
    dp.set_X_coo(node, orb, val)
    return wl, dp


def graph_form(dp, prec: int, n: int = 20, reps: int = 5):
    """Autotuned kernel, n iterations of apply_H + tmmult in one hipGraph."""
    import torch
    from paper_1907_01005_amd.autotune import GraphLoop, tune
    choice = tune(dp, prec, iters=10, warmup=2)
    loop = GraphLoop(dp, choice, n=n)
    loop.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        loop.replay()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b) * 1e-3 / n)
    it = float(np.median(times))
    return {"tuned": choice.describe(), "iter_ms": it * 1e3,
            "gdofcols_s": dp.nvalues / it / 1e9, "iterations_per_graph": n}


def energy_form(dp, reps: int = 20):
    """One evaluation of eq. energy: H X and M X onto the closure of X's
    pattern, Hbar = X^T H X and Mbar = X^T M X, E = tr((2 I - Mbar) Hbar)."""
    import torch
    out = {}
    for name, prec in (("fp64", PRECS["fp64"]), ("fp32-mfma", PRECS["fp32-mfma"])):
        for _ in range(3):
            dp.energy(prec)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for a, b in evs:
            a.record()
            dp.energy(prec)
            b.record()
        torch.cuda.synchronize()
        t = float(np.median([a.elapsed_time(b) for a, b in evs])) * 1e-3
        out[name] = {"ms": t * 1e3, "E": float(dp.E.cpu()[0])}
        # one orbital-minimisation step: E, the gradient (two Alg. 7 products),
        # tr(G^T G) and X <- X - tau G (tau = 0 keeps X for the next form)
        for a, b in evs:
            a.record()
            dp.descent_step(0.0, prec)
            b.record()
        torch.cuda.synchronize()
        out[name]["om_step_ms"] = float(np.median([a.elapsed_time(b) for a, b in evs]))
    out["closure_entries"] = dp.closure.nvalues
    out["x_entries"] = dp.nvalues
    out["rel_diff_E_fp32_vs_fp64"] = abs(out["fp32-mfma"]["E"] - out["fp64"]["E"]) / abs(out["fp64"]["E"])
    return out


def config4_forms():
    """640 orbitals in uneven column blocks on the 1686177-DoF Q2 and Q4 meshes:
    autotuned kernels, hipGraph of 20 iterations, fp32-MFMA operator with fp64
    overlap, error against the fp64 operator on the same GPU."""
    import torch
    out = {}
    for mi, tag in ((0, "Q2"), (1, "Q4")):
        print(f"[bench] config 4 mesh {tag}", file=sys.stderr, flush=True)
        wl, dp = build_problem(4, mi)
        rec = {"workload": f"{wl.meshes[mi].nx}x{wl.meshes[mi].ny}x{wl.meshes[mi].nz}-{tag}",
               "stored_entries": dp.nvalues, "colblock_sizes": [int(wl.colblock_sizes.min()),
                                                               int(wl.colblock_sizes.max())]}
        dp.apply(0)
        dp.overlap()
        torch.cuda.synchronize()
        Y64 = dp.Y.clone()
        S64 = dp.S.clone()
        t64 = dp.trace.clone()
        rec["fp64"] = graph_form(dp, 0)
        rec["fp32-mfma"] = graph_form(dp, 2)
        dp.apply(2)
        dp.overlap()
        torch.cuda.synchronize()
        rec["fp32-mfma"]["rel_err_Y"] = float((dp.Y - Y64).norm() / Y64.norm())
        rec["fp32-mfma"]["rel_err_S"] = float((dp.S - S64).norm() / S64.norm())
        rec["fp32-mfma"]["rel_err_trace"] = float(((dp.trace - t64).abs() / t64.abs()).item())
        rec["fp32-mfma"]["speedup_vs_fp64"] = rec["fp64"]["iter_ms"] / rec["fp32-mfma"]["iter_ms"]
        out[tag] = rec
        del dp
    return out


def attach_inputs(reqs, threads: int = 8):
    """The client side: every request's data (potential at the library's
    quadrature points, orbital centres and values) drawn before the stream
    starts, as the clients of a service would send them."""
    from concurrent.futures import ThreadPoolExecutor
    import synth
    from paper_1907_01005_amd import Mesh

    def one(r):
        m = Mesh(*r.cells, tuple(float(c) for c in r.cells), r.degree)
        r.inputs = synth.request_inputs(r.cells, r.degree, r.M, r.radius, r.seed, m.qp_points())
    with ThreadPoolExecutor(max_workers=threads) as pool:
        list(pool.map(one, reqs))
    return reqs


def serving_form(n: int, budget_mb: int, method: str = "rayleigh", rate: float = 40.0):
    from paper_1907_01005_amd.serving import GpuExecutor, Server, request_stream, summarize
    reqs = request_stream(n=n, rate=rate, method=method)
    t0 = time.perf_counter()
    attach_inputs(reqs)
    t_inputs = time.perf_counter() - t0
    ex = GpuExecutor(planner_threads=8)
    def progress(k, total):
        if k % 8 == 0 or k == total:
            print(f"[bench] serving: {k}/{total} requests done", file=sys.stderr, flush=True)
    rep = Server(ex, byte_budget=budget_mb << 20, max_slots=8).run(reqs, progress=progress)
    s = summarize(rep)
    s.update({"requests": n, "rate_per_s": rate, "byte_budget_mb": budget_mb, "method": method,
              "client_inputs_s": t_inputs})
    if method == "om":
        done = [r for r in rep.results.values() if "energies" in r]
        s["om_energy_decreased"] = sum(1 for r in done if r["energies"][-1] < r["energies"][0])
    return s


def trace_overlap(path: str, prefix: str = "mfb::") -> dict:
    """Device-side overlap of the library's kernels across streams, from a
    rocprofv3 kernel trace (csv): the busy time (union of the kernels'
    intervals), the sum of their durations, the time during which kernels on
    two or more streams run at once, and the most streams active together."""
    import csv
    spans = []
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        if prefix not in name:
            continue
        spans.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Stream_Id"]))
    if not spans:
        return {"kernels": 0}
    ev = sorted([(a, 1, s) for a, b, s in spans] + [(b, -1, s) for a, b, s in spans])
    active: dict = {}
    union = multi = 0
    most = 0
    last = None
    for t, d, sid in ev:
        if last is not None and active:
            union += t - last
            if len(active) >= 2:
                multi += t - last
        active[sid] = active.get(sid, 0) + d
        if active[sid] == 0:
            del active[sid]
        most = max(most, len(active))
        last = t
    total = sum(b - a for a, b, _ in spans)
    per_stream = {}
    for a, b, sid in spans:
        per_stream[sid] = per_stream.get(sid, 0) + (b - a)
    return {"kernels": len(spans), "streams": len(per_stream),
            "window_ms": (max(b for _, b, _ in spans) - min(a for a, _, _ in spans)) * 1e-6,
            "busy_union_ms": union * 1e-6, "kernel_sum_ms": total * 1e-6,
            "concurrent_ms": multi * 1e-6,
            "concurrent_frac_of_busy": multi / union if union else 0.0,
            "sum_over_union": total / union if union else 0.0,
            "most_streams_at_once": most,
            "per_stream_ms": {k: v * 1e-6 for k, v in sorted(per_stream.items())}}


def time_path(dp, prec: int, steps: int, warmup: int, kernel: int = 0):
    """Warm up, then time `steps` steps; per-apply and per-overlap event times."""
    import torch
    stream = torch.cuda.current_stream()

    def step():
        if kernel == 0:
            dp.apply(prec)
        else:
            dp.apply_tuned(prec, kernel=kernel)
        dp.overlap()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        a, b, c = ev[i]
        a.record(stream)
        if kernel == 0:
            dp.apply(prec)
        else:
            dp.apply_tuned(prec, kernel=kernel)
        b.record(stream)
        dp.overlap()
        c.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_apply = np.array([a.elapsed_time(b) for a, b, _ in ev]) * 1e-3
    t_tm = np.array([b.elapsed_time(c) for _, b, c in ev]) * 1e-3
    return wall, t_apply, t_tm


def curved_form(cfg: int, bend: float = 0.3, steps: int = 50):
    """The same workload on bent cells (isoparametric map, amplitude `bend` cell
    widths): apply_H with the per-cell metric, and the step, in fp64 and fp32-MFMA."""
    import torch
    print(f"[bench] curved form (bend {bend})", file=sys.stderr, flush=True)
    wl, dp = build_problem(cfg, bend=bend)
    alg = algorithmic(dp, wl.mesh.degree)
    n3 = (wl.mesh.degree + 1) ** 3
    # X read, Y written, and per active cell JxW V plus the six metric planes
    geo_bytes = 16 * alg["E"] + 7 * 8 * n3 * 8 * alg["active_batches"]
    out = {"workload": wl.name, "algorithmic_bytes": geo_bytes}
    for name in ("fp64", "fp32-mfma"):
        wall, ta, tt = time_path(dp, PRECS[name], steps, 5)
        t_ap = float(np.mean(ta))
        out[name] = {"apply_ms_p50": float(np.percentile(ta, 50) * 1e3),
                     "apply_gdofcols_s": alg["E"] / t_ap / 1e9,
                     "apply_hbm_frac": geo_bytes / t_ap / 1e9 / HBM_PEAK_GBS,
                     "tmmult_ms_mean": float(np.mean(tt) * 1e3),
                     "step_ms": wall / steps * 1e3}
    del dp
    torch.cuda.empty_cache()
    return out


def time_graph(dp, prec: int, steps: int, kernel: int = 0) -> float:
    """Wall seconds of `steps` steps captured once in a hipGraph and replayed
    once (after one warm replay): the same kernels as the eager loop, without
    a host launch per kernel, as a solver iteration would run."""
    import torch

    def step():
        if kernel == 0:
            dp.apply(prec)
        else:
            dp.apply_tuned(prec, kernel=kernel)
        dp.overlap()

    step()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for _ in range(steps):
                step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    graph.replay()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def time_overlapped(dp, prec: int, steps: int) -> float:
    """Wall seconds of `steps` steps as one hipGraph in the double-buffered
    form (autotune.OverlappedLoop: the zero fill of the next destination on a
    second stream while the current step's apply and overlap run), replayed
    once after one warm replay."""
    import torch
    from paper_1907_01005_amd.autotune import OverlappedLoop
    loop = OverlappedLoop(dp, prec, n=steps)
    loop.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loop.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    del loop
    return wall


def time_in_graph(one, n: int = 100, reps: int = 3) -> float:
    """Mean duration of one call of `one` (an apply_H launch: zero fill + apply
    kernel; or a tmmult: its stage kernels) when n calls run back to back in
    one hipGraph: HIP events on the replay's stream around the whole replay,
    divided by n (median of reps replays).  The eager loop's per-call events
    also hold the host's launch gaps between the call's kernels; this is the
    call as a solver iteration runs it."""
    import torch

    one()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for _ in range(n):
                one()
    torch.cuda.current_stream().wait_stream(side)
    graph.replay()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        graph.replay()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b) * 1e-3 / n)
    del graph
    return float(np.median(out))


def cold_times(dp, prec: int, reps: int = 10, scrub_mib: int = 1024):
    """apply_H and tmmult with L2 and MALL cleared first: a 1 GiB scrub write
    before each timed call evicts X, Y and the metadata (the warm loop keeps
    the ~70 MB of X and Y resident in the 256 MB MALL)."""
    import torch
    scrub = torch.empty(scrub_mib << 17, dtype=torch.float64, device="cuda")
    ta, tt = [], []
    for _ in range(reps):
        for fn, acc in ((lambda: dp.apply(prec), ta), (dp.overlap, tt)):
            scrub.fill_(1.0)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            acc.append(a.elapsed_time(b) * 1e-3)
    del scrub
    return float(np.median(ta)), float(np.median(tt))


KERNELS = {0: "default", 1: "queue", 2: "batch-grid", 7: "loader-pipelined", 8: "register-waves",
           9: "line-per-thread"}


def default_apply_kernel(dp, degree: int, prec_name: str) -> str:
    """The kernel mfb_apply_H launches after the zero fill on box cells (the
    library's rule: at p >= 3 the line kernel in fp64 and fp32 on the vector
    ALUs (the only kernel at p = 5, 6); fp32 at p = 2, the fused grid; fp64 at
    p = 2, the fused grid below 64 own items per CU, else the loader pipeline;
    the matrix-core forms, the loader pipeline at p = 2 and the shared-stage
    pipeline at p = 3, 4 while X's byte offsets fit 31 bits)."""
    import torch
    if degree >= 5 or (degree >= 3 and prec_name in ("fp64", "fp32")):
        return "apply_line_kernel"
    if prec_name == "fp32":
        return "apply_fused_kernel"
    if degree == 2:
        cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
        own = dp.layout.info["apply_items_own"]
        if prec_name == "fp64" and own < 64 * cus:
            return "apply_fused_kernel"
        return "apply_ws_kernel"
    if degree >= 3 and dp.nvalues * 8 < 2 ** 31:
        return "apply_pipe1_kernel"
    return "apply_fused_kernel"


def executed_flops_per_cell_column(p: int) -> int:
    """Flops the vector-ALU kernels execute per cell and column: the gradient
    terms go through the 1D stiffness K1 = D^T diag(w) D (one n x n product per
    line and direction instead of D, a scaling and D^T), so 18 n^4 + 7 n^3 + 3 n^3
    (the line scales) against the 24 n^4 + 7 n^3 of the sum-factorised form."""
    n = p + 1
    return 18 * n ** 4 + 10 * n ** 3


def measure(wl, dp, prec_name: str, steps: int, warmup: int, kernel: int, copy_gbs: float,
            cold: bool = True, fma_tfs: float = 0.0) -> dict:
    """One workload: the K steps as one hipGraph (value), the eager loop with
    events around every launch (latencies, the roofline of the apply_H launch)
    and, with cold, apply_H and tmmult after a scrub of L2 and MALL (the
    roofline's HBM fraction is then the cold one)."""
    degree = dp.mesh.degree
    prec = PRECS[prec_name]
    alg = algorithmic(dp, degree)
    wall, t_apply, t_tm = time_path(dp, prec, steps, warmup, kernel)
    wall_g = time_graph(dp, prec, steps, kernel)
    wall_o = time_overlapped(dp, prec, steps) if kernel == 0 else None
    t_eager = float(np.mean(t_apply))
    if kernel == 0:
        t_ap = time_in_graph(lambda: dp.apply(prec), min(steps, 100))
    else:
        t_ap = time_in_graph(lambda: dp.apply_tuned(prec, kernel=kernel), min(steps, 100))
    t_tg = time_in_graph(dp.overlap, min(steps, 100))
    gbs = alg["bytes"] / t_ap / 1e9
    tfl = alg["flops"] / t_ap / 1e12
    peak_f = FP32_MFMA_PEAK_TFLOPS if prec_name == "fp32-mfma" else FP64_PEAK_TFLOPS
    t_hbm = alg["bytes"] / (HBM_PEAK_GBS * 1e9)
    t_alu = alg["flops"] / (peak_f * 1e12)
    if t_alu >= t_hbm:
        roof = {"bound": "mfma" if prec_name in ("fp32-mfma", "fp64-mfma") else "alu",
                "achieved": tfl, "peak": peak_f, "unit": "TFLOP/s", "frac": tfl / peak_f}
    else:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS}
    vector_form = prec_name in ("fp64", "fp32")
    exe = executed_flops_per_cell_column(degree) * alg["cell_columns"] if vector_form else alg["flops"]
    default_kernel = default_apply_kernel(dp, degree, prec_name)
    roof.update({"traffic": measured_traffic(wl.name, prec_name),
                 "kernel": "apply_H launch (fill_zero_kernel + %s)" % (
                     default_kernel if kernel == 0 else {1: "apply_queue_kernel",
                                                         2: "apply_fused_kernel",
                                                         7: "apply_ws_kernel",
                                                         8: "apply_reg_kernel",
                                                         9: "apply_line_kernel"}[kernel]),
                 "algorithmic_bytes": alg["bytes"], "algorithmic_flops": alg["flops"],
                 "executed_flops": exe, "executed_frac": exe / t_ap / 1e12 / peak_f,
                 "avg_launch_s": t_ap, "timing": "apply_H launches back to back in one hipGraph, "
                 "HIP events around the replay on its stream", "eager_launch_s": t_eager,
                 "hbm_frac_warm": gbs / HBM_PEAK_GBS,
                 "alu_frac": tfl / peak_f,
                 # min(P, B I): the roof at this arithmetic intensity
                 "attainable_frac": tfl / min(peak_f, HBM_PEAK_GBS * alg["flops"] / alg["bytes"] / 1e3),
                 "copy_gbs": copy_gbs, "hbm_frac_vs_copy": gbs / copy_gbs,
                 "fp64_fma_probe_tflops": fma_tfs or None,
                 "alu_frac_vs_probe": tfl / fma_tfs if fma_tfs else None})
    tm_bytes = 16 * alg["E"] + 8 * dp.M * dp.M
    t_t = float(np.mean(t_tm))
    rec = {
        "value": alg["E"] * steps / wall_g / 1e9,
        "ms_per_step": wall_g / steps * 1e3,
        "eager": {"value": alg["E"] * steps / wall / 1e9, "ms_per_step": wall / steps * 1e3},
        "overlapped_fill": None if wall_o is None else {
            "value": alg["E"] * steps / wall_o / 1e9, "ms_per_step": wall_o / steps * 1e3,
            "form": "the same K steps as one hipGraph with two destinations: each step's zero fill "
                    "runs on a second stream one step ahead (mfb_mv_zero, then mfb_apply_H_acc)"},
        "apply_ms_p50": float(np.percentile(t_apply, 50) * 1e3),
        "apply_ms_p99": float(np.percentile(t_apply, 99) * 1e3),
        "apply_gdofcols_s": alg["E"] / t_ap / 1e9,
        "tmmult_ms_mean": t_t * 1e3,
        "tmmult_hbm_frac_eager": tm_bytes / t_t / 1e9 / HBM_PEAK_GBS,
        "tmmult_ms_graph": t_tg * 1e3,
        "tmmult_hbm_frac": tm_bytes / t_tg / 1e9 / HBM_PEAK_GBS,
        "roofline": roof,
    }
    if cold:
        ca, ct = cold_times(dp, prec)
        rec["cold"] = {"apply_ms_p50": ca * 1e3, "tmmult_ms_p50": ct * 1e3,
                       "apply_hbm_frac": alg["bytes"] / ca / 1e9 / HBM_PEAK_GBS,
                       "apply_alu_frac": alg["flops"] / ca / 1e12 / peak_f,
                       "tmmult_hbm_frac": tm_bytes / ct / 1e9 / HBM_PEAK_GBS,
                       "note": "each timed call follows a 1 GiB scrub write (L2 and MALL cold)"}
        # X, Y and the metadata (about 120 MB) stay in the 256 MB MALL between
        # warm launches: the HBM fraction is the cold one
        roof["hbm_frac"] = rec["cold"]["apply_hbm_frac"]
    else:
        roof["hbm_frac"] = None
    return rec


def precision_forms(dp, t_fp64_s: float, degree: int) -> dict:
    """apply_H in the other precision forms (and kernel variants), each with its
    speedup over the fp64 vector form on the same layout."""
    forms = {}
    for name in ("fp64-mfma", "fp32", "fp32-mfma"):
        _, ta, _ = time_path(dp, PRECS[name], 50, 5)
        forms[name] = {"apply_ms_mean": float(np.mean(ta) * 1e3),
                       "speedup_vs_fp64": t_fp64_s / float(np.mean(ta))}
    _, ta, _ = time_path(dp, PRECS["fp64"], 50, 5, kernel=1)
    forms["queue-kernel"] = {"apply_ms_mean": float(np.mean(ta) * 1e3)}
    if degree <= 2:
        _, ta, _ = time_path(dp, PRECS["fp64"], 50, 5, kernel=8)
        forms["register-waves"] = {"apply_ms_mean": float(np.mean(ta) * 1e3),
                                   "speedup_vs_fp64": t_fp64_s / float(np.mean(ta))}
    return forms


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prec", default="fp64", choices=sorted(PRECS))
    ap.add_argument("--config", type=int, default=2, choices=[2, 3])
    ap.add_argument("--kernel", type=int, default=0, choices=[0, 1, 2, 7, 8, 9],
                    help="0: the library's default apply; otherwise an explicit kernel of "
                         "mfb_apply_H_tuned (1: persistent queue, 2: batch grid, "
                         "7: loader-pipelined, 8: register-resident waves)")
    ap.add_argument("--radius", type=float, default=0.0,
                    help="replace the support radius (e.g. 16: the paper's density, ~575 MB "
                         "of X at config 2; not the baseline workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--config4", action="store_true",
                    help="also run the 640-orbital uneven-block workload (tuned + hipGraph)")
    ap.add_argument("--serve", type=int, default=16, metavar="N",
                    help="the serving stream with N requests (0: none; with --no-forms none)")
    ap.add_argument("--no-q4", action="store_true", help="leave the Q4 workload out of the forms")
    ap.add_argument("--no-config4", action="store_true",
                    help="leave the 640-orbital hipGraph loops out of the forms")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving stream (--serve N requests) and print its summary")
    ap.add_argument("--trace-overlap", metavar="CSV",
                    help="summarise the cross-stream overlap of the library's kernels in a "
                         "rocprofv3 kernel trace (no GPU needed) and exit")
    ap.add_argument("--serve-rate", type=float, default=40.0,
                    help="mean arrival rate of the serving stream (requests per second)")
    ap.add_argument("--serve-budget-mb", type=int, default=1024)
    ap.add_argument("--serve-method", default="rayleigh", choices=["rayleigh", "om"],
                    help="request iterations: Rayleigh-quotient steps or orbital minimisation")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one device copy of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args(argv)

    if args.trace_overlap:
        print(json.dumps(trace_overlap(args.trace_overlap)), flush=True)
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the path is not sharded across GPUs "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.serve_only:
        n = args.serve or 16
        print(f"[bench] serving {n} requests", file=sys.stderr, flush=True)
        print(json.dumps({"serving": serving_form(n, args.serve_budget_mb, args.serve_method,
                                                  args.serve_rate)}), flush=True)
        return 0
    print(f"[bench] building config {args.config}", file=sys.stderr, flush=True)
    wl, dp = build_problem(args.config, radius=args.radius)
    degree = wl.mesh.degree
    prec = PRECS[args.prec]
    print(f"[bench] E={dp.nvalues} items={dp.layout.info['apply_items']}; timing {args.steps} steps",
          file=sys.stderr, flush=True)
    copy_gbs = copy_bandwidth()
    fma_tfs = fp64_fma_rate()
    rec = measure(wl, dp, args.prec, args.steps, args.warmup, args.kernel, copy_gbs, fma_tfs=fma_tfs,
                  cold=not args.no_forms)
    out = {
        "metric": "apply_H GDoF*cols/s (stored BCSR entries per second, apply_H + tmmult step)",
        "value": rec.pop("value"),
        "unit": "GDoF*cols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec.startswith("fp64") else "f32 contractions, f64 storage/scaling/S",
        "data": "synthetic (seeded centres, Gaussian-well potential, N(0,1) orbital values)",
        "config": {"workload": wl.name, "dofs": dp.mesh.ndofs, "orbitals": dp.M,
                   "colblocks": int(len(wl.colblock_sizes)), "radius": wl.radius,
                   "degree": degree, "stored_entries": dp.nvalues, "prec": args.prec,
                   "kernel": KERNELS[args.kernel]},
        "launch": "the K timed steps as one hipGraph (apply_H: zero fill + apply; tmmult: the "
                  "stage-1 classes present in the layout and stage 2, which also sums the "
                  "trace); eager loop below",
    }
    out.update(rec)
    if not args.no_forms:
        t_fp64 = out["roofline"]["eager_launch_s"]
        forms = precision_forms(dp, t_fp64, degree)
        forms["energy"] = energy_form(dp)
        forms["graph20-" + args.prec] = graph_form(dp, prec)
        forms["graph20-fp32-mfma"] = graph_form(dp, PRECS["fp32-mfma"])
        forms["curved"] = curved_form(args.config)
        if args.config == 2 and not args.no_q4:
            # the same box as Q4 (32x20x20 cells, 846369 DoFs, 320 orbitals)
            print("[bench] Q4 workload", file=sys.stderr, flush=True)
            del dp
            import torch
            torch.cuda.empty_cache()
            wl3, dp3 = build_problem(3)
            q4 = measure(wl3, dp3, args.prec, min(args.steps, 100), args.warmup, 0, copy_gbs,
                         fma_tfs=fma_tfs)
            q4["workload"] = wl3.name
            q4["stored_entries"] = dp3.nvalues
            q4["forms"] = precision_forms(dp3, q4["roofline"]["eager_launch_s"], 4)
            forms["q4"] = q4
            del dp3
            torch.cuda.empty_cache()
        out["forms"] = forms
    if args.config4 or not (args.no_forms or args.no_config4):
        out["config4"] = config4_forms()
    if args.serve and not args.no_forms:
        print(f"[bench] serving {args.serve} requests", file=sys.stderr, flush=True)
        out["serving"] = serving_form(args.serve, args.serve_budget_mb, args.serve_method,
                                      args.serve_rate)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = int(src.numel() * 8)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        # the oracle's apply is numpy work on small element matrices: it runs on
        # one thread whatever the BLAS pool holds, so the baseline is taken on
        # one thread (cores = 1 exactly) and the pool's run is reported beside it
        out["cpu_baseline"] = cpu_baseline(wl, one_thread=True)
        out["cpu_baseline_all_threads"] = cpu_baseline(wl, budget_s=5.0)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
