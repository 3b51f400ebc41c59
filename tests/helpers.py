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


def oracle_Y_at(op, node: np.ndarray, orb: np.ndarray, blocks=None) -> np.ndarray:
    """Oracle Y at the given (node, orbital) coordinates, block by block."""
    out = np.full(len(node), np.nan)
    blocks = range(op.pattern.ncb) if blocks is None else blocks
    for C in blocks:
        orbs = op.block_orbitals(C)
        Y = op.Y_columns(orbs)
        col = {int(a): j for j, a in enumerate(orbs)}
        sel = np.isin(orb, orbs)
        j = np.array([col[int(a)] for a in orb[sel]], dtype=np.int64)
        out[sel] = Y[node[sel], j]
    return out
