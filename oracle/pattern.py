"""BCSR pattern of the sparse multivector (oracle).

Rows (Alg. 1).  Coarse cells of level L are 2x2x2 batches of fine cells (the
experiments take L one coarser than the finest, Sec. 4).  Batches are sorted
by the Hilbert index of their integer batch coordinates (step 2).  Walking the
batches in that order, every node of a batch that no earlier batch has
claimed gets the next row number; the rows claimed by one batch form one row
block (steps 5-7).  Within a block, rows are in ascending global node id.

Columns (Alg. 2).  Each orbital centre is located in the batch that contains
it (floor(c_d * nb_d / L_d), clamped to the box); orbitals are sorted by the
Hilbert index of that batch (stable, ties kept in original id order) and cut
into column blocks (B with the remainder on the last block, or explicit
sizes).

Support (Sec. 4).  The patch of orbital alpha is the set of batches whose
centre lies within distance r of the orbital centre; a block (r, C) is stored
iff row block r's batch lies in the patch of some orbital of C.  Blocks are
numbered in CSR order and laid out back to back, each row-major with row
length |C| (no padding).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .hilbert import bits_for, hilbert_index
from .mesh import BoxMesh


@dataclasses.dataclass
class Pattern:
    mesh: BoxMesh
    batch_order: np.ndarray      # (nrb,) row block r -> batch id bx + nbx (by + nby bz)
    rb_start: np.ndarray         # (nrb+1,) first row of each row block
    dof_perm: np.ndarray         # (N,) row -> global node id
    node_row: np.ndarray         # (N,) global node id -> row
    node_rb: np.ndarray          # (N,) global node id -> row block
    col_perm: np.ndarray         # (M,) column position -> original orbital id
    col_pos: np.ndarray          # (M,) original orbital id -> column position
    cb_start: np.ndarray         # (ncb+1,) first column position of each column block
    orb_cb: np.ndarray           # (M,) original orbital id -> column block
    rowptr: np.ndarray           # (nrb+1,) CSR over row blocks
    colidx: np.ndarray           # (nnzb,) column block of each stored block, ascending per row
    block_offset: np.ndarray     # (nnzb+1,) value offset of each stored block
    stored: np.ndarray           # (nrb, ncb) bool

    @property
    def nrb(self):
        return len(self.rb_start) - 1

    @property
    def ncb(self):
        return len(self.cb_start) - 1

    @property
    def nvalues(self):
        return int(self.block_offset[-1])


def batch_grid(mesh: BoxMesh):
    nb = tuple(c // 2 for c in mesh.cells)
    if any(2 * b != c for b, c in zip(nb, mesh.cells)):
        raise ValueError("cell counts must be even (2x2x2 batches)")
    return nb


def order_batches(mesh: BoxMesh, hilbert: bool = True) -> np.ndarray:
    nb = batch_grid(mesh)
    ids = np.arange(nb[0] * nb[1] * nb[2])
    if not hilbert:
        return ids.astype(np.int64)
    bits = bits_for(max(nb))
    bx, by, bz = ids % nb[0], (ids // nb[0]) % nb[1], ids // (nb[0] * nb[1])
    keys = np.array([hilbert_index((x, y, z), bits) for x, y, z in zip(bx, by, bz)],
                    dtype=np.int64)
    return ids[np.argsort(keys, kind="stable")]


def batch_nodes(mesh: BoxMesh, b: int) -> np.ndarray:
    """Global ids (ascending) of the (2p+1)^3 nodes of batch b."""
    nb = batch_grid(mesh)
    bx, by, bz = b % nb[0], (b // nb[0]) % nb[1], b // (nb[0] * nb[1])
    p = mesh.p
    a = mesh.nodes_per_axis
    r = np.arange(2 * p + 1)
    Z, Y, X = np.meshgrid(2 * p * bz + r, 2 * p * by + r, 2 * p * bx + r, indexing="ij")
    return (X + a[0] * (Y + a[1] * Z)).ravel().astype(np.int64)


def row_blocks(mesh: BoxMesh, order: np.ndarray):
    """First-encounter row numbering along the batch order (Alg. 1 steps 5-7)."""
    N = mesh.ndofs
    node_rb = np.full(N, -1, dtype=np.int64)
    rows = []
    rb_start = [0]
    for r, b in enumerate(order):
        g = batch_nodes(mesh, int(b))
        new = g[node_rb[g] < 0]          # ascending, since g is ascending
        node_rb[new] = r
        rows.append(new)
        rb_start.append(rb_start[-1] + len(new))
    dof_perm = np.concatenate(rows)
    node_row = np.empty(N, dtype=np.int64)
    node_row[dof_perm] = np.arange(N)
    return np.asarray(rb_start, dtype=np.int64), dof_perm, node_row, node_rb


def batch_of_point(mesh: BoxMesh, c) -> tuple:
    nb = batch_grid(mesh)
    out = []
    for d in range(3):
        k = int(np.floor((c[d] * nb[d]) / mesh.L[d]))
        out.append(min(max(k, 0), nb[d] - 1))
    return tuple(out)


def order_columns(mesh: BoxMesh, centres: np.ndarray, hilbert: bool = True) -> np.ndarray:
    M = len(centres)
    if not hilbert:
        return np.arange(M, dtype=np.int64)
    nb = batch_grid(mesh)
    bits = bits_for(max(nb))
    keys = np.array([hilbert_index(batch_of_point(mesh, c), bits) for c in centres],
                    dtype=np.int64)
    return np.argsort(keys, kind="stable").astype(np.int64)


def patches(mesh: BoxMesh, centres: np.ndarray, radius) -> np.ndarray:
    """(M, nbatches) bool: batch centre within distance r of orbital centre."""
    nb = batch_grid(mesh)
    h = mesh.h
    ids = np.arange(nb[0] * nb[1] * nb[2])
    bx, by, bz = ids % nb[0], (ids // nb[0]) % nb[1], ids // (nb[0] * nb[1])
    cx = (2 * bx + 1) * h[0]
    cy = (2 * by + 1) * h[1]
    cz = (2 * bz + 1) * h[2]
    rad = np.broadcast_to(np.asarray(radius, dtype=np.float64), (len(centres),))
    out = np.zeros((len(centres), len(ids)), dtype=bool)
    for a, c in enumerate(centres):
        dx = cx - c[0]
        dy = cy - c[1]
        dz = cz - c[2]
        out[a] = (dx * dx + dy * dy) + dz * dz <= rad[a] * rad[a]
    return out


def build_pattern(mesh: BoxMesh, centres, radius, colblock_sizes,
                  hilbert_rows: bool = True, hilbert_cols: bool = True) -> Pattern:
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    M = len(centres)
    sizes = np.asarray(colblock_sizes, dtype=np.int64)
    if sizes.sum() != M or (sizes <= 0).any():
        raise ValueError("column block sizes must be positive and sum to M")
    order = order_batches(mesh, hilbert_rows)
    rb_start, dof_perm, node_row, node_rb = row_blocks(mesh, order)
    col_perm = order_columns(mesh, centres, hilbert_cols)
    col_pos = np.empty(M, dtype=np.int64)
    col_pos[col_perm] = np.arange(M)
    cb_start = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cb_of_pos = np.repeat(np.arange(len(sizes)), sizes)
    orb_cb = cb_of_pos[col_pos]
    P = patches(mesh, centres, radius)               # (M, nbatches) by batch id
    nrb, ncb = len(order), len(sizes)
    stored = np.zeros((nrb, ncb), dtype=bool)
    for a in range(M):
        hit = P[a][order]                            # by row block
        stored[hit, orb_cb[a]] = True
    rowptr = np.concatenate([[0], np.cumsum(stored.sum(axis=1))]).astype(np.int64)
    rr, cc = np.nonzero(stored)                      # row-major: ascending C per row
    rows_r = np.diff(rb_start)
    blk = rows_r[rr] * sizes[cc]
    block_offset = np.concatenate([[0], np.cumsum(blk)]).astype(np.int64)
    return Pattern(mesh, order, rb_start, dof_perm, node_row, node_rb, col_perm, col_pos,
                   cb_start, orb_cb, rowptr, cc.astype(np.int64), block_offset, stored)


def closure_pattern(pat: Pattern) -> Pattern:
    """Destination pattern that holds H X and M X entirely.

    Alg. 6 writes through the destination's accessor, and the text notes that
    the operator's result has a larger support than its argument.  This
    pattern is the support of that result: block (r, C) is stored iff some
    non-Dirichlet node of row block r shares a cell with a non-Dirichlet node
    whose block (r', C) is stored in ``pat``.  Rows, columns and column blocks
    are those of ``pat``; the stored blocks of ``pat`` are a subset.
    """
    mesh = pat.mesh
    dofs = mesh.cell_dofs()                          # (ncells, n^3)
    free = ~mesh.dirichlet_mask()[dofs]              # (ncells, n^3)
    rb = pat.node_rb[dofs]                           # row block of every cell node
    stored = np.zeros_like(pat.stored)
    for C in range(pat.ncb):
        touches = (pat.stored[rb, C] & free).any(axis=1)   # cells with a stored free node
        reached = rb[touches][free[touches]]
        stored[np.unique(reached), C] = True
    rowptr = np.concatenate([[0], np.cumsum(stored.sum(axis=1))]).astype(np.int64)
    rr, cc = np.nonzero(stored)
    rows_r = np.diff(pat.rb_start)
    sizes = np.diff(pat.cb_start)
    block_offset = np.concatenate([[0], np.cumsum(rows_r[rr] * sizes[cc])]).astype(np.int64)
    return dataclasses.replace(pat, rowptr=rowptr, colidx=cc.astype(np.int64),
                               block_offset=block_offset, stored=stored)


def entry_coords(pat: Pattern):
    """For every stored value position: (global node id, original orbital id)."""
    nodes = np.empty(pat.nvalues, dtype=np.int64)
    orbs = np.empty(pat.nvalues, dtype=np.int64)
    for r in range(pat.nrb):
        rows = pat.dof_perm[pat.rb_start[r]:pat.rb_start[r + 1]]
        for k in range(pat.rowptr[r], pat.rowptr[r + 1]):
            C = pat.colidx[k]
            cols = pat.col_perm[pat.cb_start[C]:pat.cb_start[C + 1]]
            o = pat.block_offset[k]
            m = len(rows) * len(cols)
            nodes[o:o + m] = np.repeat(rows, len(cols))
            orbs[o:o + m] = np.tile(cols, len(rows))
    return nodes, orbs


def entry_positions(pat: Pattern, node: np.ndarray, orb: np.ndarray) -> np.ndarray:
    """Value position of (node, orbital) pairs; -1 where the block is not stored."""
    node = np.asarray(node, dtype=np.int64)
    orb = np.asarray(orb, dtype=np.int64)
    r = pat.node_rb[node]
    C = pat.orb_cb[orb]
    ok = pat.stored[r, C]
    # block index of (r, C): rowptr[r] + rank of C among the stored columns of row r
    rank = np.cumsum(pat.stored, axis=1) - 1
    k = pat.rowptr[r] + rank[r, C]
    width = pat.cb_start[C + 1] - pat.cb_start[C]
    row_in = pat.node_row[node] - pat.rb_start[r]
    col_in = pat.col_pos[orb] - pat.cb_start[C]
    pos = pat.block_offset[np.where(ok, k, 0)] + row_in * width + col_in
    return np.where(ok, pos, -1)
