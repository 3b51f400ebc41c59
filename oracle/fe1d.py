"""1D ingredients of the Q_p tensor-product basis (oracle).

Sec. 3.1 of the paper: shape functions are Lagrange polynomials on the
elements, continuous across element faces, with nodes where N_j(x_i) =
delta_ij.  The node family is not stated; this oracle takes the
Gauss-Lobatto-Legendre points (the usual choice of continuous Lagrange
elements).  The quadrature is the (p+1)-point Gauss-Legendre rule per
direction.  Everything lives on the reference interval [0, 1].
"""

from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as _leg


def gll_nodes(p: int) -> np.ndarray:
    """p+1 Gauss-Lobatto-Legendre nodes on [0, 1], ascending.

    The interior nodes are the roots of P_p'(t) on [-1, 1]; the end points
    are -1 and 1; the map t -> (1 + t) / 2 takes them to [0, 1].
    """
    if p < 1:
        raise ValueError("degree must be >= 1")
    if p == 1:
        t = np.array([-1.0, 1.0])
    else:
        c = np.zeros(p + 1)
        c[p] = 1.0
        roots = np.sort(np.real(_leg.legroots(_leg.legder(c))))
        t = np.concatenate([[-1.0], roots, [1.0]])
    return 0.5 * (1.0 + t)


def gauss_rule(n: int):
    """n-point Gauss-Legendre points (ascending) and weights on [0, 1]."""
    t, w = _leg.leggauss(n)
    return 0.5 * (1.0 + t), 0.5 * w


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """phi[q, k] = phi_k(x_q) for the Lagrange basis through ``nodes``."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(nodes)
    out = np.ones((len(x), m))
    for k in range(m):
        for j in range(m):
            if j != k:
                out[:, k] *= (x - nodes[j]) / (nodes[k] - nodes[j])
    return out


def lagrange_derivatives(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dphi[q, k] = phi_k'(x_q), by the product rule over the factors."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(nodes)
    out = np.zeros((len(x), m))
    for k in range(m):
        for j in range(m):
            if j == k:
                continue
            term = np.full(len(x), 1.0 / (nodes[k] - nodes[j]))
            for l in range(m):
                if l != k and l != j:
                    term *= (x - nodes[l]) / (nodes[k] - nodes[l])
            out[:, k] += term
    return out


def basis_tables(p: int, nq: int | None = None):
    """Return (xq, wq, S, D): Gauss points/weights and S[q,k]=phi_k(xq), D=phi_k'(xq)."""
    n = p + 1 if nq is None else nq
    xq, wq = gauss_rule(n)
    nodes = gll_nodes(p)
    return xq, wq, lagrange_values(nodes, xq), lagrange_derivatives(nodes, xq)
