"""Oracle: reference-element tabulation (Section II-B, eq. tensorDense).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The reference element is ``[-1, 1]^3``.  Nodes are the ``P = p + 1`` Gauss-Lobatto
points (end points plus roots of the derivative of the Legendre polynomial of degree
``p``); quadrature is ``Q``-point Gauss-Legendre.  The paper states that order 2 uses 27
quadrature points (Section V-B), so ``Q = p + 1`` is the default everywhere.  3D tables
are dense Kronecker products, built by explicit loops.
"""
from __future__ import annotations

import numpy as np


def gll_nodes(P: int) -> np.ndarray:
    """Gauss-Lobatto nodes on [-1, 1] (sorted)."""
    p = P - 1
    if p < 1:
        raise ValueError("P must be >= 2")
    if p == 1:
        return np.array([-1.0, 1.0])
    inner = np.sort(np.real(np.polynomial.legendre.Legendre.basis(p).deriv().roots()))
    return np.concatenate(([-1.0], inner, [1.0]))


def gauss(Q: int) -> tuple:
    """Gauss-Legendre points and weights on [-1, 1]."""
    x, w = np.polynomial.legendre.leggauss(Q)
    return x, w


def lagrange(nodes: np.ndarray, x: np.ndarray) -> tuple:
    """Values ``B[q, i] = l_i(x_q)`` and derivatives ``D[q, i] = l_i'(x_q)`` of the
    Lagrange polynomials on ``nodes``, by the product formula."""
    n = len(nodes)
    B = np.ones((len(x), n))
    D = np.zeros((len(x), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                B[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
        for k in range(n):
            if k == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[k]))
            for j in range(n):
                if j != i and j != k:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            D[:, i] += term
    return B, D


def tables_1d(P: int, Q: int) -> dict:
    """1D interpolation and derivative tables from GLL nodes to Gauss points."""
    nodes = gll_nodes(P)
    xq, wq = gauss(Q)
    B, D = lagrange(nodes, xq)
    return {"nodes": nodes, "xq": xq, "wq": wq, "B": B, "D": D}


def tensor_3d(P: int, Q: int) -> dict:
    """Dense 3D tables (eq. tensorDense): ``Phi[q, a]`` and ``dPhi[d, q, a]`` with
    ``q = q1 + Q q2 + Q^2 q3`` and ``a = a1 + P a2 + P^2 a3``, and weights ``w3[q]``."""
    t = tables_1d(P, Q)
    B, D, w = t["B"], t["D"], t["wq"]
    Q3, P3 = Q ** 3, P ** 3
    Phi = np.zeros((Q3, P3))
    dPhi = np.zeros((3, Q3, P3))
    w3 = np.zeros(Q3)
    for q3 in range(Q):
        for q2 in range(Q):
            for q1 in range(Q):
                q = q1 + Q * q2 + Q * Q * q3
                w3[q] = w[q1] * w[q2] * w[q3]
                for a3 in range(P):
                    for a2 in range(P):
                        for a1 in range(P):
                            a = a1 + P * a2 + P * P * a3
                            Phi[q, a] = B[q1, a1] * B[q2, a2] * B[q3, a3]
                            dPhi[0, q, a] = D[q1, a1] * B[q2, a2] * B[q3, a3]
                            dPhi[1, q, a] = B[q1, a1] * D[q2, a2] * B[q3, a3]
                            dPhi[2, q, a] = B[q1, a1] * B[q2, a2] * D[q3, a3]
    return {"Phi": Phi, "dPhi": dPhi, "w3": w3, "P": P, "Q": Q, **t}


def node_positions_3d(P: int) -> np.ndarray:
    """Reference coordinates ``[P^3][3]`` of the element's nodes, lexicographic."""
    r = gll_nodes(P)
    out = np.zeros((P ** 3, 3))
    for a3 in range(P):
        for a2 in range(P):
            for a1 in range(P):
                out[a1 + P * a2 + P * P * a3] = (r[a1], r[a2], r[a3])
    return out


def eval_3d(P: int, xi: np.ndarray) -> np.ndarray:
    """Values ``[n_pts][P^3]`` of the 3D nodal basis of order ``P - 1`` at reference
    points ``xi [n_pts][3]`` (Kronecker product of 1D Lagrange values)."""
    nodes = gll_nodes(P)
    B1, _ = lagrange(nodes, xi[:, 0])
    B2, _ = lagrange(nodes, xi[:, 1])
    B3, _ = lagrange(nodes, xi[:, 2])
    out = np.zeros((xi.shape[0], P ** 3))
    for a3 in range(P):
        for a2 in range(P):
            for a1 in range(P):
                out[:, a1 + P * a2 + P * P * a3] = B1[:, a1] * B2[:, a2] * B3[:, a3]
    return out
