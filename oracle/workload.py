"""Oracle results for a seeded synthetic workload (test infrastructure).

Builds the oracle's own mesh, pattern and potential from a ``synth``
workload and evaluates Y = mask(H X), S = X^T Y and tr S in global
coordinates (node id, original orbital id), column block by column block.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

import synth

from .apply import block_mask, dense_columns, energy, gradient, masked_apply, overlap, trace
from .mesh import BoxMesh
from .pattern import build_pattern, closure_pattern, entry_coords


class OracleProblem:
    def __init__(self, wl, mesh_index: int = 0, values: str = "orbitals", hilbert: bool = True,
                 value_seed: int = 0):
        ms = wl.meshes[mesh_index]
        self.wl = wl
        self.mesh = BoxMesh(ms.nx, ms.ny, ms.nz, tuple(ms.L), ms.degree, ms.dirichlet)
        if getattr(ms, "bend", 0.0):
            # curved cells: the seeded map applied to this oracle's own box nodes
            self.mesh = BoxMesh(ms.nx, ms.ny, ms.nz, tuple(ms.L), ms.degree, ms.dirichlet,
                                nodes=ms.bend_points(self.mesh.node_points()))
        qp = self.mesh.qp_points()
        self.v_qp = synth.potential_at(wl, qp.reshape(-1, 3)).reshape(qp.shape[:2])
        self.pattern = build_pattern(self.mesh, wl.centres, wl.radius, wl.colblock_sizes,
                                     hilbert, hilbert)
        if values == "orbitals":
            self.node, self.orb, self.val = synth.orbital_values(wl, mesh_index)
        elif values == "generic":
            # a value at every stored entry, off the Dirichlet rows
            node, orb = entry_coords(self.pattern)
            val = synth.orbital_values_generic(len(node), value_seed)
            keep = ~self.mesh.dirichlet_mask()[node]
            self.node, self.orb, self.val = node[keep], orb[keep].astype(np.int32), val[keep]
        else:
            raise ValueError(values)

    @property
    def M(self):
        return self.wl.M

    def block_orbitals(self, C: int) -> np.ndarray:
        p = self.pattern
        return p.col_perm[p.cb_start[C]:p.cb_start[C + 1]]

    def X_columns(self, orbs) -> np.ndarray:
        return dense_columns(self.mesh.ndofs, self.node, self.orb, self.val, orbs)

    def closure(self):
        """Destination pattern that holds H X and M X entirely."""
        if not hasattr(self, "_closure"):
            self._closure = closure_pattern(self.pattern)
        return self._closure

    def Y_columns(self, orbs, op: str = "H", dest: str = "x") -> np.ndarray:
        """H X (op "H") or M X (op "M") for the columns ``orbs``, kept on the
        pattern of X (dest "x") or on its closure (dest "closure")."""
        pat = self.pattern if dest == "x" else self.closure()
        return masked_apply(pat, self.v_qp, self.X_columns(orbs), orbs, op=op)

    def Y_blocks(self, blocks):
        """{C: (orbs, dense Y (N, |C|))} for the listed column blocks."""
        return {C: (self.block_orbitals(C), self.Y_columns(self.block_orbitals(C))) for C in blocks}

    def Y_all_sparse(self, op: str = "H", dest: str = "x") -> sp.csc_matrix:
        """Y for every column as a sparse N x M matrix (original orbital order)."""
        rows, cols, vals = [], [], []
        for C in range(self.pattern.ncb):
            orbs = self.block_orbitals(C)
            Y = self.Y_columns(orbs, op, dest)
            r, c = np.nonzero(Y)
            rows.append(r)
            cols.append(orbs[c])
            vals.append(Y[r, c])
        return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.mesh.ndofs, self.M))

    def X_sparse(self) -> sp.csc_matrix:
        return sp.csc_matrix((self.val, (self.node, self.orb)), shape=(self.mesh.ndofs, self.M))

    def overlap(self, Y: sp.csc_matrix | None = None):
        Y = self.Y_all_sparse() if Y is None else Y
        S = overlap(self.X_sparse(), Y)
        return S, trace(S)

    def projected(self):
        """(Mbar, Hbar, E): X^T M X and X^T H X through the closure destination,
        and the energy of eq. energy (original orbital order)."""
        Hbar = overlap(self.X_sparse(), self.Y_all_sparse("H", "closure"))
        Mbar = overlap(self.X_sparse(), self.Y_all_sparse("M", "closure"))
        return Mbar, Hbar, energy(Mbar, Hbar)

    def gradient_dense(self):
        """(G, E): eq. gradient on the pattern of X as a dense N x M array
        (original orbital order), and the energy; for small problems."""
        orbs = np.arange(self.M)
        X = self.X_columns(orbs)
        HX = self.Y_columns(orbs, "H", "closure")
        MX = self.Y_columns(orbs, "M", "closure")
        Hbar, Mbar = X.T @ HX, X.T @ MX
        G = gradient(MX, HX, Mbar, Hbar, block_mask(self.pattern, orbs))
        return G, energy(Mbar, Hbar)
