"""Explicit element matrices of the Hamiltonian (oracle).

eq. fe_matrices (Sec. 3.1):

    M_ij = sum_K int_K N_i N_j dx
    H_ij = sum_K int_K [ 1/2 grad N_i . grad N_j + N_i V N_j ] dx

On an axis-aligned box cell K = x_K + [0,h_x] x [0,h_y] x [0,h_z] with
quadrature points x_q = x_K + h (.) xi_q and weights JxW_q = w_q1 w_q2 w_q3
h_x h_y h_z, the tensor-product shape function with local index
i = i1 + n i2 + n^2 i3 is N_i(x_q) = phi_i1(xi_q1) phi_i2(xi_q2) phi_i3(xi_q3)
and d/dx_1 N_i = phi'_i1 phi_i2 phi_i3 / h_x, and so on.  The element matrix
is assembled here as a plain sum over quadrature points -- no sum
factorisation -- so that it can be checked against the paper by eye:

    H_K = 1/2 sum_d G_d^T diag(JxW) G_d + N^T diag(JxW * V) N

On a curved cell (isoparametric map x(xi) = sum_k x_k N_k(xi)), the Jacobian
J_ab(q) = dx_a/dxi_b = sum_k x_k,a dN_k/dxi_b (xi_q), the physical gradient is
grad N_i = J^{-T} grad_xi N_i and JxW_q = w_q |det J(q)|, per cell.
"""

from __future__ import annotations

import numpy as np

from .fe1d import basis_tables


def tensor_tables(p: int, h, nq: int | None = None):
    """Values N[q,i], gradients G[d][q,i] and JxW[q] on one cell of size h.

    Local index i = i1 + n i2 + n^2 i3 (x fastest) and the same for q.
    """
    xq, wq, S, D = basis_tables(p, nq)
    hx, hy, hz = (float(v) for v in h)
    # kron(A3, kron(A2, A1))[(q3,q2,q1),(i3,i2,i1)] = A3[q3,i3] A2[q2,i2] A1[q1,i1]
    N = np.kron(S, np.kron(S, S))
    Gx = np.kron(S, np.kron(S, D)) / hx
    Gy = np.kron(S, np.kron(D, S)) / hy
    Gz = np.kron(D, np.kron(S, S)) / hz
    JxW = np.kron(wq, np.kron(wq, wq)) * (hx * hy * hz)
    return N, (Gx, Gy, Gz), JxW, xq


def laplace_matrix(p: int, h, nq: int | None = None) -> np.ndarray:
    """K_K[i,j] = sum_q JxW_q * 1/2 * sum_d dN_i/dx_d(q) dN_j/dx_d(q)."""
    N, G, JxW, _ = tensor_tables(p, h, nq)
    K = np.zeros((N.shape[1], N.shape[1]))
    for Gd in G:
        K += 0.5 * Gd.T @ (JxW[:, None] * Gd)
    return K


def mass_matrix(p: int, h, nq: int | None = None) -> np.ndarray:
    """M_K[i,j] = sum_q JxW_q N_i(q) N_j(q)."""
    N, _, JxW, _ = tensor_tables(p, h, nq)
    return N.T @ (JxW[:, None] * N)


def potential_matrices(p: int, h, v_qp: np.ndarray, nq: int | None = None) -> np.ndarray:
    """Batch of M_K[V][i,j] = sum_q JxW_q V(x_q) N_i(q) N_j(q) for cells K.

    ``v_qp`` has shape (ncells, nq^3): V at the quadrature points of each cell.
    """
    N, _, JxW, _ = tensor_tables(p, h, nq)
    v_qp = np.asarray(v_qp, dtype=np.float64)
    c = v_qp * JxW[None, :]                       # (ncells, nq3)
    NT_c = N.T[None, :, :] * c[:, None, :]        # (ncells, n3, nq3): N^T diag(c)
    return NT_c @ N


def hamiltonian_matrices(p: int, h, v_qp: np.ndarray, nq: int | None = None) -> np.ndarray:
    """H_K = K_K + M_K[V] for every cell (eq. fe_matrices)."""
    K = laplace_matrix(p, h, nq)
    return K[None, :, :] + potential_matrices(p, h, v_qp, nq)


def curved_tables(p: int, xcell: np.ndarray, nq: int | None = None):
    """Per cell of an isoparametric mesh: values N[q,i], physical gradients
    G[c,q,a,i] = (J^{-T} grad_xi N_i)_a and JxW[c,q] = w_q |det J|.

    ``xcell`` (c, n^3, 3): the cells' node positions in local order.
    """
    xq, wq, S, D = basis_tables(p, nq)
    N = np.kron(S, np.kron(S, S))
    # reference gradients d/dxi_1, d/dxi_2, d/dxi_3 on [0,1]^3
    Gr = np.stack([np.kron(S, np.kron(S, D)), np.kron(S, np.kron(D, S)), np.kron(D, np.kron(S, S))])
    J = np.einsum("bqk,cka->cqab", Gr, np.asarray(xcell, dtype=np.float64))
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    G = np.einsum("cqba,bqi->cqai", Jinv, Gr)         # J^{-T} grad_xi N_i
    W = np.kron(wq, np.kron(wq, wq))
    JxW = W[None, :] * np.abs(det)
    return N, G, JxW


def curved_matrices(p: int, xcell: np.ndarray, v_qp: np.ndarray | None = None,
                    which: str = "H", nq: int | None = None) -> np.ndarray:
    """Element matrices of curved cells, plain sums over quadrature points:
    "K" = 1/2 sum_q JxW grad N_i . grad N_j, "M" = sum_q JxW N_i N_j,
    "V" = sum_q JxW V N_i N_j, "H" = K + V."""
    N, G, JxW = curved_tables(p, xcell, nq)
    out = 0.0
    if which in ("K", "H"):
        out = out + 0.5 * np.einsum("cqai,cq,cqaj->cij", G, JxW, G)
    if which in ("V", "H"):
        c = JxW * np.asarray(v_qp, dtype=np.float64)
        out = out + np.einsum("qi,cq,qj->cij", N, c, N)
    if which == "M":
        out = np.einsum("qi,cq,qj->cij", N, JxW, N)
    return out
