"""Continuous-batching request loop over device-resident BCSR multivectors.

A request is a small minimisation run on its own mesh, ``iters`` iterations
of one of two methods on the pattern of X:

* "rayleigh":  Y = H X;  S = X^T Y;  S2 = X^T X;
               X <- X - tau (Y - X diag(S)/diag(S2))
  (a column-wise Rayleigh-quotient step over the required operations);
* "om": steepest descent on the energy of eq. energy: H X and M X onto the
  closure of X's pattern, Hbar, Mbar and E, the gradient of eq. gradient by
  Alg. 7 truncated to X's pattern, X <- X - tau G.  The functional is
  bounded below only where H is negative on the growing directions, so H is
  shifted by -shift M (the potential V - shift; H - shift M is exactly that
  operator) and the columns are first scaled to diag(X^T M X) = 1/4, inside
  the basin where components along positive directions decay.  Every step
  takes a backtracking (Armijo) line search: tau is doubled from the last
  accepted value and halved until E(X - tau G) <= E(X) - tau tr(G^T G) / 2
  (eq. G_ops4 gives the directional derivative).  The searches read E back,
  so an "om" request runs its loop in a host thread of its own; the
  scheduler keeps polling the other requests meanwhile.

Requests
arrive over time; the server admits a waiting request as soon as a slot is
free and its device footprint (BCSR values, metadata, workspace, S) fits in
the byte budget, so requests that arrive while others run are started at
once and their kernels overlap on the device (one HIP stream per slot).
Completion is detected with events, memory is released, and the next
waiting request is admitted: the batch changes continuously.

The scheduler is independent of the GPU: it drives an ``Executor``.  A
request carries its data (potential at the quadrature points, orbital
centres and values), prepared by the client before it is sent.  The GPU
executor plans each request in the library (mesh, BCSR layout, packing) in
a worker pool when it arrives, and on admission allocates, uploads and
enqueues all iterations on the slot's stream.
"""

from __future__ import annotations

import math
import statistics
import threading
import time
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional, Sequence, Tuple

import numpy as np

from .api import FP32_MFMA, FP64

# mesh choices of the request stream (cells, unit cell width)
MESHES = [(16, 16, 16), (24, 16, 16), (32, 20, 20), (32, 32, 32), (48, 32, 32), (64, 40, 40)]


@dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the stream starts
    cells: Tuple[int, int, int]
    degree: int
    M: int
    radius: float
    prec: int
    iters: int
    seed: int
    method: str = "rayleigh"       # "rayleigh" or "om" (see the module docstring)
    shift: float = 2.0             # "om": the spectral shift (potential V - shift)
    # the request's data, prepared by the client before it is sent: box
    # lengths and Dirichlet faces, orbital centres, support radius, column-
    # block sizes, the potential at the quadrature points of the mesh
    # ([ncells][nq], library cell order) and the orbital values as (node,
    # orbital, value) triplets
    inputs: Optional[dict] = None


def request_stream(n: int = 96, rate: float = 40.0, seed: int = 5, meshes=MESHES,
                   m_range=(32, 640), r_range=(3.0, 5.0), precs=(FP32_MFMA, FP64),
                   degrees=(2, 4), iters: int = 10, method: str = "rayleigh") -> List[Request]:
    """Poisson arrivals; mesh uniform over `meshes`; degree and precision 50/50;
    M log-uniform in m_range; support radius uniform in r_range."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        cells = tuple(int(c) for c in meshes[int(rng.integers(len(meshes)))])
        degree = int(degrees[int(rng.integers(len(degrees)))])
        M = int(round(math.exp(rng.uniform(math.log(m_range[0]), math.log(m_range[1])))))
        r = float(rng.uniform(*r_range))
        prec = int(precs[int(rng.integers(len(precs)))])
        out.append(Request(i, t, cells, degree, M, r, prec, iters, seed * 1000 + i, method))
    return out


# ----------------------------------------------------------------- scheduler
@dataclass
class Slot:
    req: Request
    handle: Any
    token: Any
    admitted: float


@dataclass
class ServeReport:
    results: Dict[int, dict] = field(default_factory=dict)
    admit_order: List[int] = field(default_factory=list)
    max_bytes_in_use: int = 0
    max_concurrent: int = 0
    wall_s: float = 0.0


class Server:
    """FIFO admission by slot count and device-byte budget."""

    def __init__(self, executor, byte_budget: int, max_slots: int = 8):
        self.ex = executor
        self.budget = int(byte_budget)
        self.max_slots = int(max_slots)

    def run(self, requests: Sequence[Request], realtime: bool = True,
            poll_s: float = 0.0005, progress=None) -> ServeReport:
        """progress: optional callable, given (finished, total) after each request."""
        rep = ServeReport()
        queue = sorted(requests, key=lambda r: r.arrival)
        arrived: List[Tuple[Request, Future]] = []
        active: List[Slot] = []
        in_use = 0
        t0 = time.perf_counter()
        nxt = 0
        clock = (lambda: time.perf_counter() - t0) if realtime else None
        sim_now = 0.0
        while nxt < len(queue) or arrived or active:
            now = clock() if realtime else sim_now
            while nxt < len(queue) and queue[nxt].arrival <= now:
                arrived.append((queue[nxt], self.ex.prepare_async(queue[nxt])))
                nxt += 1
            # admit in arrival order while slots and bytes allow
            while arrived and len(active) < self.max_slots:
                req, fut = arrived[0]
                if not fut.done():
                    break
                handle = fut.result()
                need = self.ex.footprint(handle)
                if need > self.budget:
                    arrived.pop(0)
                    rep.results[req.rid] = {"rejected": True, "bytes": need}
                    continue
                if in_use + need > self.budget:
                    break
                arrived.pop(0)
                in_use += need
                tok = self.ex.start(handle)
                active.append(Slot(req, handle, tok, clock() if realtime else sim_now))
                rep.admit_order.append(req.rid)
                rep.max_bytes_in_use = max(rep.max_bytes_in_use, in_use)
                rep.max_concurrent = max(rep.max_concurrent, len(active))
            # retire finished requests
            still = []
            for s in active:
                if self.ex.done(s.token):
                    res = self.ex.finish(s.token)
                    end = clock() if realtime else sim_now
                    res.update({"arrival": s.req.arrival, "admitted": s.admitted, "finished": end,
                                "latency_s": end - s.req.arrival})
                    rep.results[s.req.rid] = res
                    in_use -= self.ex.footprint(s.handle)
                    self.ex.release(s.handle)
                    if progress is not None:
                        progress(len(rep.results), len(queue))
                else:
                    still.append(s)
            active = still
            if realtime:
                time.sleep(poll_s)
            else:
                sim_now = self.ex.advance(sim_now)
        rep.wall_s = (time.perf_counter() - t0) if realtime else sim_now
        return rep


def apply_overlap(spans) -> dict:
    """Device time the applies of different requests run together: spans are
    (start, end, request) on one device timeline.  Returns the union of the
    apply intervals, the sum of their lengths, the time during which applies
    of two or more requests run at once, and its fraction of the union."""
    ev = sorted([(t0, 1, rid) for t0, t1, rid in spans] + [(t1, -1, rid) for t0, t1, rid in spans])
    active: Dict[int, int] = {}
    union = multi = 0.0
    last = None
    for t, d, rid in ev:
        if last is not None and active:
            union += t - last
            if len(active) >= 2:
                multi += t - last
        active[rid] = active.get(rid, 0) + d
        if active[rid] == 0:
            del active[rid]
        last = t
    total = sum(t1 - t0 for t0, t1, _ in spans)
    return {"apply_union_s": union, "apply_sum_s": total, "apply_concurrent_s": multi,
            "apply_concurrent_frac": multi / union if union > 0 else 0.0}


def summarize(rep: ServeReport) -> dict:
    done = [r for r in rep.results.values() if not r.get("rejected")]
    applies = [t for r in done for t in r.get("apply_s", [])]
    entries = sum(r.get("entries", 0) * len(r.get("apply_s", [])) for r in done)
    gpu_apply_s = sum(applies)
    out = {
        "requests_done": len(done),
        "requests_rejected": len(rep.results) - len(done),
        "wall_s": rep.wall_s,
        "requests_per_s": len(done) / rep.wall_s if rep.wall_s > 0 else 0.0,
        "max_concurrent": rep.max_concurrent,
        "max_bytes_in_use": rep.max_bytes_in_use,
    }
    spans = [(t0, t1, rid) for rid, r in rep.results.items() if not r.get("rejected")
             for t0, t1 in r.get("apply_spans", [])]
    if spans:
        out.update(apply_overlap(spans))
    if applies:
        out.update({
            "apply_ms_p50": 1e3 * statistics.median(applies),
            "apply_ms_p99": 1e3 * float(np.percentile(applies, 99)),
            "aggregate_gdofcols_s": entries / rep.wall_s / 1e9 if rep.wall_s > 0 else 0.0,
            "apply_gdofcols_s_busy": entries / gpu_apply_s / 1e9 if gpu_apply_s > 0 else 0.0,
            "latency_s_p50": statistics.median(r["latency_s"] for r in done),
            "latency_s_p99": float(np.percentile([r["latency_s"] for r in done], 99)),
        })
    return out


# ----------------------------------------------------------------- GPU executor
@dataclass
class _Plan:
    req: Request
    mesh: Any
    layout: Any
    values: np.ndarray
    nbytes: int
    h: float
    closure: Any = None


class GpuExecutor:
    """Plans on the host (worker pool), runs each request on its own stream."""

    def __init__(self, device: str = "cuda", planner_threads: int = 4, tau_scale: float = 0.05,
                 keep_X: bool = False):
        self.device = device
        self.pool = ThreadPoolExecutor(max_workers=planner_threads)
        self.tau_scale = tau_scale
        self.keep_X = keep_X
        self._lock = threading.Lock()
        self._t0 = None  # a device event every apply interval is measured from

    # -- planning (host only)
    def _plan(self, req: Request) -> _Plan:
        """Library planning of one request from the data it carries (host)."""
        from .api import Layout, Mesh
        d = req.inputs
        if d is None:
            raise ValueError(f"request {req.rid} carries no inputs (the client prepares them)")
        cells = req.cells
        mesh = Mesh(*cells, d["L"], req.degree, d["dirichlet"])
        V = np.asarray(d["v_qp"], dtype=np.float64)
        mesh.set_potential(V - req.shift if req.method == "om" else V)
        layout = Layout(mesh, d["centres"], d["radius"], d["colblock_sizes"])
        values = layout.pack(d["node"], d["orb"], d["val"])
        M = layout.M
        nbytes = (2 * 8 * max(layout.nvalues, 1) + mesh.meta_bytes + layout.meta_bytes
                  + layout.work_bytes + 2 * 8 * M * M + 16)
        closure = None
        if req.method == "om":
            from .api import energy_work_bytes
            closure = layout.closure()
            # X, G, trial X; H X and M X on the closure; its metadata and
            # workspace; Hbar, Mbar; energy and dot scratch
            nbytes = (3 * 8 * max(layout.nvalues, 1) + 2 * 8 * max(closure.nvalues, 1)
                      + mesh.meta_bytes + layout.meta_bytes + closure.meta_bytes
                      + closure.work_bytes + 2 * 8 * M * M + energy_work_bytes(M) + 8 * 1024
                      + 8 * (req.iters + 8))
        return _Plan(req, mesh, layout, values, nbytes, 1.0, closure)

    def prepare_async(self, req: Request) -> Future:
        return self.pool.submit(self._plan, req)

    def footprint(self, plan: _Plan) -> int:
        return plan.nbytes

    # -- execution
    def start(self, plan: _Plan):
        import torch
        if self._t0 is None:
            self._t0 = torch.cuda.Event(enable_timing=True)
            self._t0.record()
        if plan.req.method == "om":
            return self._start_om(plan)
        from .api import mv_update, apply_H, tmmult
        stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(stream):
            plan.mesh.bind(self.device, stream)
            plan.layout.bind(self.device, stream)
            lay = plan.layout
            X = torch.from_numpy(plan.values).to(self.device, non_blocking=False) \
                if lay.nvalues else torch.zeros(1, dtype=torch.float64, device=self.device)
            Y = lay.new_values(self.device)
            work = lay.new_work(self.device)
            S = torch.zeros((lay.M, lay.M), dtype=torch.float64, device=self.device)
            S2 = torch.zeros_like(S)
            tr = torch.zeros(2, dtype=torch.float64, device=self.device)
            tau = self.tau_scale * plan.h * plan.h
            evs = []
            for _ in range(plan.req.iters):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                apply_H(plan.mesh, lay, X, Y, plan.req.prec, stream)
                b.record(stream)
                tmmult(lay, X, Y, S, tr[0:1], work, stream)
                tmmult(lay, X, X, S2, tr[1:2], work, stream)
                mv_update(lay, X, Y, S, S2, tau, stream)
                evs.append((a, b))
            end = torch.cuda.Event()
            end.record(stream)
        return {"plan": plan, "stream": stream, "evs": evs, "end": end,
                "bufs": (X, Y, work, S, S2, tr)}

    def _start_om(self, plan: _Plan):
        """Orbital-minimisation steps on the slot's stream, driven by a host
        thread (see the module docstring)."""
        import torch
        tok = {"plan": plan, "evs": [], "tau": 0.0, "energies": [], "error": None}
        tok["thread"] = threading.Thread(target=self._run_om, args=(tok,), daemon=True)
        tok["thread"].start()
        return tok

    def _run_om(self, tok) -> None:
        import torch
        from .api import (DOT_WORK_DOUBLES, OP_H, OP_M, apply_op, energy, energy_work_bytes,
                          mmult, mv_axpy, mv_dot, mv_scale_columns, tmmult)
        try:
            plan = tok["plan"]
            dev, lay, clo, mesh, prec = (self.device, plan.layout, plan.closure, plan.mesh,
                                         plan.req.prec)
            stream = torch.cuda.Stream(device=dev)
            tok["stream"] = stream
            M = lay.M
            with torch.cuda.stream(stream):
                mesh.bind(dev, stream)
                lay.bind(dev, stream)
                clo.bind(dev, stream)
                X = torch.from_numpy(plan.values).to(dev) if lay.nvalues else \
                    torch.zeros(1, dtype=torch.float64, device=dev)
                Xt, G = lay.new_values(dev), lay.new_values(dev)
                YH, YM = clo.new_values(dev), clo.new_values(dev)
                work = clo.new_work(dev)
                Hb = torch.zeros((M, M), dtype=torch.float64, device=dev)
                Mb = torch.zeros_like(Hb)
                tr = torch.zeros(2, dtype=torch.float64, device=dev)
                wE = torch.zeros(energy_work_bytes(M) // 8, dtype=torch.float64, device=dev)
                wD = torch.zeros(DOT_WORK_DOUBLES, dtype=torch.float64, device=dev)
                E = torch.zeros(1, dtype=torch.float64, device=dev)
                gg = torch.zeros(1, dtype=torch.float64, device=dev)

                def energy_at(Xv, timed=False) -> float:
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    apply_op(mesh, lay, clo, OP_H, Xv, YH, prec, stream)
                    b.record(stream)
                    apply_op(mesh, lay, clo, OP_M, Xv, YM, prec, stream)
                    tmmult(clo, Xv, YH, Hb, tr[0:1], work, stream)
                    tmmult(clo, Xv, YM, Mb, tr[1:2], work, stream)
                    energy(M, Mb, Hb, E, wE, stream)
                    if timed:
                        tok["evs"].append((a, b))
                    stream.synchronize()
                    return float(E.cpu()[0])

                # columns to diag(X^T M X) = 1/4
                energy_at(X)
                d = torch.diagonal(Mb).cpu().numpy()
                sc = np.where(d > 0, 0.5 / np.sqrt(np.where(d > 0, d, 1.0)), 1.0)
                scale = torch.from_numpy(sc).to(dev)
                mv_scale_columns(lay, scale, X, stream)
                tau = 0.0
                for k in range(plan.req.iters):
                    e0 = energy_at(X, timed=True)
                    tok["energies"].append(e0)
                    mmult(clo, lay, YM, Hb, -2.0, 0.0, G, False, stream)
                    mmult(clo, lay, YH, Mb, -2.0, 4.0, G, True, stream)
                    mv_dot(lay, G, G, gg, wD, stream)
                    stream.synchronize()
                    g0 = float(gg.cpu()[0])
                    if not g0 > 0.0:
                        break
                    tau = 2.0 * tau if tau > 0 else 0.5 * max(abs(e0), 1.0) / g0
                    for _ in range(60):
                        Xt.copy_(X)
                        mv_axpy(lay, -tau, G, Xt, stream)
                        if energy_at(Xt) <= e0 - 0.5 * tau * g0:
                            break
                        tau *= 0.5
                    X.copy_(Xt)
                tok["energies"].append(energy_at(X))
                tok["tau"] = tau
                tok["bufs"] = (X,)
                tok["keep"] = (Xt, G, YH, YM, work, Hb, Mb, tr, wE, wD, E, gg, scale)
                stream.synchronize()
        except Exception as e:  # reported by finish()
            tok["error"] = e

    def done(self, tok) -> bool:
        if "thread" in tok:
            return not tok["thread"].is_alive()
        return tok["end"].query()

    def finish(self, tok) -> dict:
        plan = tok["plan"]
        if "thread" in tok:
            tok["thread"].join()
            if tok["error"] is not None:
                raise tok["error"]
        else:
            tok["end"].synchronize()
        apply_s = [a.elapsed_time(b) * 1e-3 for a, b in tok["evs"]]
        # each apply's interval on the device timeline (seconds from the
        # executor's reference event): overlap across slot streams
        spans = [(self._t0.elapsed_time(a) * 1e-3, self._t0.elapsed_time(b) * 1e-3)
                 for a, b in tok["evs"]] if self._t0 is not None else []
        if plan.req.method == "om":
            X = tok["bufs"][0]
            out = {"apply_s": apply_s, "apply_spans": spans, "entries": plan.layout.nvalues,
                   "tau": tok["tau"],
                   "energies": tok["energies"], "prec": plan.req.prec,
                   "bytes": plan.nbytes, "method": "om"}
        else:
            X, Y, work, S, S2, tr = tok["bufs"]
            trs = tr.cpu().numpy()
            out = {"apply_s": apply_s, "apply_spans": spans, "entries": plan.layout.nvalues,
                   "trace": float(trs[0]),
                   "trace_xx": float(trs[1]),
                   "x_norm2": float((X[:plan.layout.nvalues] ** 2).sum()),
                   "prec": plan.req.prec, "bytes": plan.nbytes}
        if self.keep_X:
            out["X"] = X[:plan.layout.nvalues].cpu().numpy()
        return out

    def release(self, plan: _Plan) -> None:
        # device buffers die with the token; drop the device copies of the metadata
        plan.mesh._meta = None
        plan.layout._meta = None
        if plan.closure is not None:
            plan.closure._meta = None

    def advance(self, now: float) -> float:
        return now


# ----------------------------------------------------------------- fake executor (tests)
class FakeExecutor:
    """Counts bytes and simulates run time in a virtual clock (scheduler tests)."""

    def __init__(self, bytes_of=None, seconds_of=None, dt: float = 0.001):
        self.bytes_of = bytes_of or (lambda r: r.M * 1000)
        self.seconds_of = seconds_of or (lambda r: 0.01 * r.iters)
        self.dt = dt
        self.now = 0.0
        self.live_bytes = 0
        self.max_live = 0
        self.events: List[Tuple[str, int, float]] = []

    def prepare_async(self, req):
        f: Future = Future()
        f.set_result(req)
        return f

    def footprint(self, req):
        return self.bytes_of(req)

    def start(self, req):
        self.live_bytes += self.bytes_of(req)
        self.max_live = max(self.max_live, self.live_bytes)
        self.events.append(("start", req.rid, self.now))
        return {"req": req, "t_end": self.now + self.seconds_of(req)}

    def done(self, tok):
        return tok["t_end"] <= self.now

    def finish(self, tok):
        self.events.append(("finish", tok["req"].rid, self.now))
        return {"apply_s": [1e-3] * tok["req"].iters, "entries": tok["req"].M}

    def release(self, req):
        self.live_bytes -= self.bytes_of(req)

    def advance(self, now: float) -> float:
        self.now = now + self.dt
        return self.now
