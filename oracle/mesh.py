"""Structured box mesh of Q_p hexahedra (oracle).

Box [0,Lx] x [0,Ly] x [0,Lz] split into nx x ny x nz equal cells.  The
global node grid has p*n_d + 1 points per axis and global node id
g = X + (p nx + 1) (Y + (p ny + 1) Z) (x fastest).  Cell (cx, cy, cz) owns
the nodes (p cx + i, p cy + j, p cz + k), local index i + n j + n^2 k with
n = p + 1.  Cells are numbered lexicographically, cx fastest.

Homogeneous Dirichlet conditions (the H^1_0 space of Sec. 3.1) are imposed on
the faces selected by a bit mask (bit 2d: x_d = 0, bit 2d+1: x_d = L_d): the
nodes there remain rows of the multivector, but the operator is restricted to
the other nodes, i.e. X is read as 0 and Y is 0 on them.

Curved cells (the general hexahedral meshes of Sec. 3.1): when ``nodes``
holds a physical position for every global node, each cell is the image of
the reference cube under the isoparametric map x(xi) = sum_k x_k N_k(xi) of
its own node positions, so cells may be rotated, sheared or curved.  The
node numbering, the faces and the box [0, L] stay those of the index grid,
which also defines batches, supports and the column order.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .fe1d import gauss_rule, gll_nodes


@dataclasses.dataclass
class BoxMesh:
    nx: int
    ny: int
    nz: int
    L: tuple
    p: int
    dirichlet: int = 0x3F
    nodes: np.ndarray | None = None  # (N, 3) physical node positions (curved cells), or None

    @property
    def curved(self) -> bool:
        return self.nodes is not None

    @property
    def n(self):
        return self.p + 1

    @property
    def cells(self):
        return (self.nx, self.ny, self.nz)

    @property
    def h(self):
        return tuple(self.L[d] / self.cells[d] for d in range(3))

    @property
    def nodes_per_axis(self):
        return tuple(self.p * self.cells[d] + 1 for d in range(3))

    @property
    def ndofs(self):
        a = self.nodes_per_axis
        return a[0] * a[1] * a[2]

    @property
    def ncells(self):
        return self.nx * self.ny * self.nz

    def cell_coords(self) -> np.ndarray:
        """(ncells, 3) integer coordinates, cx fastest."""
        cz, cy, cx = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx),
                                 indexing="ij")
        return np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)

    def cell_dofs(self, cells: np.ndarray | None = None) -> np.ndarray:
        """(ncells, n^3) global node ids of each cell, local index x fastest."""
        cc = self.cell_coords() if cells is None else np.asarray(cells).reshape(-1, 3)
        n, p = self.n, self.p
        a = self.nodes_per_axis
        k3, j3, i3 = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        li, lj, lk = i3.ravel(), j3.ravel(), k3.ravel()
        X = p * cc[:, 0:1] + li[None, :]
        Y = p * cc[:, 1:2] + lj[None, :]
        Z = p * cc[:, 2:3] + lk[None, :]
        return (X + a[0] * (Y + a[1] * Z)).astype(np.int64)

    def node_coords(self) -> np.ndarray:
        """(N, 3) integer grid coordinates of every global node."""
        a = self.nodes_per_axis
        g = np.arange(self.ndofs)
        return np.stack([g % a[0], (g // a[0]) % a[1], g // (a[0] * a[1])], axis=1)

    def node_points(self) -> np.ndarray:
        """(N, 3) physical node positions (GLL nodes inside each cell)."""
        if self.nodes is not None:
            return np.asarray(self.nodes, dtype=np.float64)
        xi = gll_nodes(self.p)
        pos = []
        for d in range(3):
            X = np.arange(self.nodes_per_axis[d])
            c = np.minimum(X // self.p, self.cells[d] - 1)
            loc = X - self.p * c
            pos.append((c + xi[loc]) * self.h[d])
        a = self.nodes_per_axis
        g = np.arange(self.ndofs)
        return np.stack([pos[0][g % a[0]], pos[1][(g // a[0]) % a[1]], pos[2][g // (a[0] * a[1])]],
                        axis=1)

    def qp_points(self, cells: np.ndarray | None = None, nq: int | None = None) -> np.ndarray:
        """(ncells, nq^3, 3) physical quadrature points, q = q1 + nq q2 + nq^2 q3."""
        cc = self.cell_coords() if cells is None else np.asarray(cells).reshape(-1, 3)
        m = self.n if nq is None else nq
        if self.nodes is not None:
            # x(xi_q) = sum_k x_k N_k(xi_q) over the cell's own nodes
            from .fe1d import basis_tables
            _, _, S, _ = basis_tables(self.p, m)
            N = np.kron(S, np.kron(S, S))                 # (m^3, n^3)
            lin = cc[:, 0] + self.nx * (cc[:, 1] + self.ny * cc[:, 2])
            xc = np.asarray(self.nodes)[self.cell_dofs()[lin]]   # (c, n^3, 3)
            return np.einsum("qk,cka->cqa", N, xc)
        xq, _ = gauss_rule(m)
        k3, j3, i3 = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
        h = self.h
        x = (cc[:, 0:1] + xq[i3.ravel()][None, :]) * h[0]
        y = (cc[:, 1:2] + xq[j3.ravel()][None, :]) * h[1]
        z = (cc[:, 2:3] + xq[k3.ravel()][None, :]) * h[2]
        return np.stack([x, y, z], axis=2)

    def dirichlet_mask(self) -> np.ndarray:
        """Boolean (N,) -- True on nodes of the selected Dirichlet faces."""
        nc = self.node_coords()
        a = self.nodes_per_axis
        m = np.zeros(self.ndofs, dtype=bool)
        for d in range(3):
            if self.dirichlet & (1 << (2 * d)):
                m |= nc[:, d] == 0
            if self.dirichlet & (1 << (2 * d + 1)):
                m |= nc[:, d] == a[d] - 1
        return m
