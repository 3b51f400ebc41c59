"""Cell-by-cell operator application, overlap matrix and trace (oracle).

Operator (eq. fe_matrices_cell_based):  H = sum_K P_K^T H_K P_K, with P_K
the gather of the cell's node values and H_K the explicit element matrix of
``oracle.element``.  Applying it to a multivector X (global node x orbital):

    Y = sum_K P_K^T (H_K (P_K X))

restricted to the nodes off the Dirichlet faces (X is read as 0 there and Y
is 0 there).  The BCSR result keeps only entries whose block is stored in the
pattern of X (Alg. 6 writes through the accessor of the destination, which
only reaches stored blocks; the destination here has the pattern of X):

    Y_bcsr = mask_P(Y)

Overlap (Alg. 8 / eq. inner2): S = X^T Y, and its trace sum_a X_a . Y_a
(eq. G_ops4 with D = X, G = Y).

With the closure pattern (``oracle.pattern.closure_pattern``) as the
destination, nothing of H X or M X is dropped, so X^T (H X) and X^T (M X) are
the projected matrices Hbar and Mbar of eq. energy, and the energy follows.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .element import (curved_matrices, hamiltonian_matrices, laplace_matrix, mass_matrix,
                      potential_matrices)
from .mesh import BoxMesh
from .pattern import Pattern


def _cell_nodes(mesh: BoxMesh, cells: np.ndarray) -> np.ndarray:
    """(c, n^3, 3) node positions of the listed cells (curved meshes)."""
    return np.asarray(mesh.nodes)[mesh.cell_dofs()[cells]]


def element_masses(mesh: BoxMesh, cells: np.ndarray) -> np.ndarray:
    """M_K for the listed cells (the same on every cell of a uniform box)."""
    if mesh.curved:
        return curved_matrices(mesh.p, _cell_nodes(mesh, cells), which="M")
    Mk = mass_matrix(mesh.p, mesh.h)
    return np.broadcast_to(Mk, (len(cells),) + Mk.shape)


def element_hamiltonians(mesh: BoxMesh, v_qp: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """H_K for the listed cells (indices into the lexicographic cell order)."""
    if mesh.curved:
        return curved_matrices(mesh.p, _cell_nodes(mesh, cells), np.asarray(v_qp)[cells], "H")
    return hamiltonian_matrices(mesh.p, mesh.h, np.asarray(v_qp)[cells])


def apply_hamiltonian(mesh: BoxMesh, v_qp: np.ndarray, Xg: np.ndarray,
                      chunk: int = 4096, op: str = "H") -> np.ndarray:
    """Y = H X (op "H") or Y = M X (op "M", the mass matrix of eq. fe_matrices)
    on the non-Dirichlet nodes for a dense (N, m) block of columns."""
    Xg = np.asarray(Xg, dtype=np.float64)
    if Xg.ndim == 1:
        Xg = Xg[:, None]
    dmask = mesh.dirichlet_mask()
    X = Xg.copy()
    X[dmask] = 0.0
    dofs = mesh.cell_dofs()
    nz_row = np.any(X != 0.0, axis=1)
    active = np.nonzero(nz_row[dofs].any(axis=1))[0]   # cells with a non-zero input
    Y = np.zeros_like(X)
    m = X.shape[1]
    for s in range(0, len(active), chunk):
        cells = active[s:s + chunk]
        H = element_hamiltonians(mesh, v_qp, cells) if op == "H" else element_masses(mesh, cells)
        idx = dofs[cells]                              # (c, n3)
        Yk = H @ X[idx]                                # (c, n3, m)
        np.add.at(Y, idx.ravel(), Yk.reshape(-1, m))
    Y[dmask] = 0.0
    return Y


def block_mask(pat: Pattern, orbs) -> np.ndarray:
    """(N, len(orbs)) bool: entry (i, alpha) lies in a stored block."""
    orbs = np.asarray(orbs, dtype=np.int64)
    return pat.stored[pat.node_rb[:, None], pat.orb_cb[orbs][None, :]]


def masked_apply(pat: Pattern, v_qp: np.ndarray, Xg: np.ndarray, orbs, op: str = "H") -> np.ndarray:
    """Y = mask_P(H X) (or mask_P(M X)) for the columns ``orbs`` of X (dense
    (N, len(orbs))); ``pat`` is the destination pattern."""
    Y = apply_hamiltonian(pat.mesh, v_qp, Xg, op=op)
    return np.where(block_mask(pat, orbs), Y, 0.0)


def dense_columns(N: int, node, orb, val, orbs) -> np.ndarray:
    """Dense (N, len(orbs)) block of a COO multivector, restricted to ``orbs``."""
    orbs = np.asarray(orbs, dtype=np.int64)
    where = {int(a): j for j, a in enumerate(orbs)}
    col = np.array([where.get(int(a), -1) for a in np.asarray(orb)], dtype=np.int64) \
        if len(orb) else np.zeros(0, dtype=np.int64)
    keep = col >= 0
    out = np.zeros((N, len(orbs)))
    np.add.at(out, (np.asarray(node)[keep], col[keep]), np.asarray(val)[keep])
    return out


def overlap(X: sp.spmatrix, Y: sp.spmatrix) -> np.ndarray:
    """S = X^T Y (dense M x M) from two sparse N x M multivectors."""
    return np.asarray((sp.csc_matrix(X).T @ sp.csc_matrix(Y)).todense())


def trace(S: np.ndarray) -> float:
    return float(np.trace(S))


def energy(Mbar: np.ndarray, Hbar: np.ndarray) -> float:
    """eq. energy: E = tr((2 I - Mbar) Hbar) with Mbar = X^T M X, Hbar = X^T H X."""
    return float(np.trace((2.0 * np.eye(len(Mbar)) - Mbar) @ Hbar))


def assemble(mesh: BoxMesh, v_qp: np.ndarray | None = None, which: str = "H") -> np.ndarray:
    """Dense global matrix by scatter-adding element matrices (pins only)."""
    N = mesh.ndofs
    dofs = mesh.cell_dofs()
    A = np.zeros((N, N))
    if mesh.curved:
        allc = np.arange(mesh.ncells)
        Ke = curved_matrices(mesh.p, _cell_nodes(mesh, allc),
                             None if v_qp is None else np.asarray(v_qp), which)
    elif which == "H":
        Ke = hamiltonian_matrices(mesh.p, mesh.h, v_qp)
    elif which == "K":
        Ke = np.broadcast_to(laplace_matrix(mesh.p, mesh.h), (mesh.ncells,) + (dofs.shape[1],) * 2)
    elif which == "M":
        Ke = np.broadcast_to(mass_matrix(mesh.p, mesh.h), (mesh.ncells,) + (dofs.shape[1],) * 2)
    elif which == "V":
        Ke = potential_matrices(mesh.p, mesh.h, v_qp)
    else:
        raise ValueError(which)
    for c in range(mesh.ncells):
        idx = dofs[c]
        A[np.ix_(idx, idx)] += Ke[c]
    return A


def mmult(A: np.ndarray, B: np.ndarray, dest_mask: np.ndarray) -> np.ndarray:
    """Alg. 7 with truncation: C = A B (A dense N x M, B dense M x M), kept
    only where the destination pattern stores an entry (``dest_mask``,
    N x M bool); the rest of the product is discarded."""
    return np.where(dest_mask, A @ B, 0.0)


def gradient(MX: np.ndarray, HX: np.ndarray, Mbar: np.ndarray, Hbar: np.ndarray,
             dest_mask: np.ndarray) -> np.ndarray:
    """eq. gradient on the pattern of X: G = -2 M X Hbar + 2 H X (2 I - Mbar),
    each product by Alg. 7 truncated to the destination pattern."""
    two_minus = 2.0 * np.eye(len(Mbar)) - Mbar
    return mmult(MX, -2.0 * Hbar, dest_mask) + mmult(HX, 2.0 * two_minus, dest_mask)
