"""Shared helpers of the test-suite: build the same seeded workload on the GPU
library and in the CPU oracle, and compare results in global coordinates."""

from __future__ import annotations

import sys

import numpy as np

import synth


def say(msg: str) -> None:
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def device_problem(wl, mesh_index: int = 0):
    from paper_1907_01005_amd.problem import DeviceProblem
    ms = wl.meshes[mesh_index]
    return DeviceProblem((ms.nx, ms.ny, ms.nz), ms.L, ms.degree, ms.dirichlet, wl.centres,
                         wl.radius, wl.colblock_sizes, lambda P: synth.potential_at(wl, P),
                         node_map=ms.bend_points if getattr(ms, "bend", 0.0) else None)


def rel_fro(a: np.ndarray, b: np.ndarray) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def max_rel(a: np.ndarray, b: np.ndarray) -> float:
    """max |a - b| / max |b|: a few badly wrong entries fail this even where
    the Frobenius norm of the difference stays small."""
    mb = float(np.max(np.abs(b))) if np.size(b) else 0.0
    if np.size(a) == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0))


def gate(got: np.ndarray, ref: np.ndarray, tol: float, what: str) -> None:
    """Both bars of the parity tests: relative Frobenius error and max|diff| /
    max|ref|, each within tol."""
    ef, em = rel_fro(got, ref), max_rel(got, ref)
    say(f"{what}: rel_F {ef:.2e} max_rel {em:.2e} (tol {tol:.0e})")
    assert ef <= tol and em <= tol, (what, ef, em)


def oracle_full(op, node: np.ndarray, orb: np.ndarray):
    """Oracle Y at every given (node, orbital) coordinate, and S = X^T Y with
    its trace (original orbital order), from one pass over the column blocks."""
    import scipy.sparse as sp
    from oracle.apply import overlap, trace
    out = np.full(len(node), np.nan)
    rows, cols, vals = [], [], []
    for C in range(op.pattern.ncb):
        orbs = op.block_orbitals(C)
        Y = op.Y_columns(orbs)
        col = {int(a): j for j, a in enumerate(orbs)}
        sel = np.isin(orb, orbs)
        j = np.array([col[int(a)] for a in orb[sel]], dtype=np.int64)
        out[sel] = Y[node[sel], j]
        r, c = np.nonzero(Y)
        rows.append(r)
        cols.append(orbs[c])
        vals.append(Y[r, c])
    Ys = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(op.mesh.ndofs, op.M))
    S = overlap(op.X_sparse(), Ys)
    assert not np.isnan(out).any(), "a stored entry outside every column block"
    return out, S, trace(S)


def attach_inputs(reqs):
    """Client side of the serving tests: each request's data (potential at the
    library's quadrature points, orbital centres and values), drawn before
    the requests are sent."""
    from paper_1907_01005_amd import Mesh
    for r in reqs:
        m = Mesh(*r.cells, tuple(float(c) for c in r.cells), r.degree)
        r.inputs = synth.request_inputs(r.cells, r.degree, r.M, r.radius, r.seed, m.qp_points())
    return reqs
