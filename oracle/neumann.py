"""Neumann-Neumann preconditioner of the vertex Schur system (oracle, FP64).

Test infrastructure only: the plain definitions that the GPU preconditioner
is checked against.

Paper passages followed (section "Algorithmic Implementation", subsection
"Phase 4: The Inside Loop (PCG solver)", "The Neumann Step"):

* eq. distribute_dv: the vertex residual r is shared out over the edge ends
  at each vertex v, every end receiving r_v / d_v (d_v = number of edge ends
  at v, so a self-loop counts twice).
* eq. neumann_block: on each edge, the full local system of that edge's
  elements, with zero load on the interior nodes and the shared residual on
  its two end nodes, is solved for the displacements delta.
* The permutation P of that passage puts the nodes in their order along the
  edge ([left end, interior, right end]), which makes the local matrix
  tridiagonal; it is solved with the Thomas algorithm.
* eq. induced_displacements: the two end displacements are scaled by 1/d_v
  again and summed over the edges at each vertex.
* The closing remark of the subsection: the step is the operator
  D^{-1} (sum_e S_e^{-1}) D^{-1} with D = diag(d_v) and S_e the edge's 2x2
  Schur complement (eq. local_reduced_schur), each S_e^{-1} placed at the
  edge's two vertices.

``neumann_step`` follows the steps in that order; ``nn_matrix`` is the closed
form.  The local element matrices are the lumped-mass ones of the shifted
system A = (c_I + c_L kappa^2) M_L + c_L G (Phase 2): alpha h_e/2 + c_L/h_e at
each end node, alpha h_e + 2 c_L/h_e inside, -c_L/h_e between neighbours.

Parity pins (tests/test_oracle_neumann.py): the local matrices summed over
the edges equal the assembled shifted matrix; the Schur complement of each
local matrix equals the edge blocks of the learned-preconditioner oracle;
``neumann_step`` equals ``nn_matrix`` applied to r (the paper's equivalence);
on a single edge the preconditioner is S^{-1} and PCG ends after one step;
with decoupled, equal edges it reduces to Jacobi; it is symmetric positive
definite.
"""

from __future__ import annotations

import numpy as np

from . import mesh as _mesh


def _alpha(kappa_e: float, c_I: float, c_L: float) -> float:
    return c_I + c_L * kappa_e * kappa_e


def edge_tridiag(m: _mesh.Mesh, e: int, kappa_e: float, c_I: float, c_L: float):
    """Diagonals (sub, main, super) of edge e's local matrix P A_e P^T, nodes
    ordered [tail vertex, interior 1..m, head vertex] (length m + 2)."""
    h = float(m.h_e[e])
    a = _alpha(kappa_e, c_I, c_L)
    n = m.m(e) + 2
    main = np.full(n, a * h + 2.0 * c_L / h)
    main[0] = main[-1] = a * h / 2.0 + c_L / h
    off = np.full(n - 1, -c_L / h)
    return off.copy(), main, off


def thomas(sub: np.ndarray, main: np.ndarray, sup: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Textbook Thomas algorithm for a tridiagonal system (no pivoting)."""
    n = main.shape[0]
    c = np.zeros(n)
    d = np.zeros(n)
    c[0] = sup[0] / main[0] if n > 1 else 0.0
    d[0] = rhs[0] / main[0]
    for i in range(1, n):
        den = main[i] - sub[i - 1] * c[i - 1]
        c[i] = sup[i] / den if i < n - 1 else 0.0
        d[i] = (rhs[i] - sub[i - 1] * d[i - 1]) / den
    x = np.zeros(n)
    x[-1] = d[-1]
    for i in range(n - 2, -1, -1):
        x[i] = d[i] - c[i] * x[i + 1]
    return x


def degrees(m: _mesh.Mesh) -> np.ndarray:
    """d_v: edge ends at each vertex (a self-loop contributes two)."""
    return np.bincount(m.edges.ravel(), minlength=m.n_vertices).astype(np.float64)


def neumann_step(m: _mesh.Mesh, kappa_e: np.ndarray, c_I: float, c_L: float, r: np.ndarray) -> np.ndarray:
    """The Neumann step applied to the vertex residual r: share out by 1/d_v,
    solve every edge's local system with the shared residual on its ends,
    scale the end displacements by 1/d_v and sum them at the vertices."""
    d = degrees(m)
    rt = r / d                                      # eq. distribute_dv
    w = np.zeros(m.n_vertices)
    for e in range(m.n_edges):
        u, v = int(m.edges[e, 0]), int(m.edges[e, 1])
        sub, main, sup = edge_tridiag(m, e, float(kappa_e[e]), c_I, c_L)
        rhs = np.zeros(main.shape[0])
        rhs[0], rhs[-1] = rt[u], rt[v]              # zero load on the interior nodes
        delta = thomas(sub, main, sup, rhs)         # eq. neumann_block, permuted
        w[u] += delta[0] / d[u]                     # eq. induced_displacements
        w[v] += delta[-1] / d[v]
    return w


def nn_matrix(n_vertices: int, edges: np.ndarray, sd: np.ndarray, so: np.ndarray) -> np.ndarray:
    """Dense D^{-1} (sum_e S_e^{-1}) D^{-1}, S_e = [[sd_e, so_e], [so_e, sd_e]]."""
    d = np.bincount(np.asarray(edges).ravel(), minlength=n_vertices).astype(np.float64)
    Sinv = np.zeros((n_vertices, n_vertices))
    for e, (u, v) in enumerate(edges):
        Se = np.array([[sd[e], so[e]], [so[e], sd[e]]])
        Ie = np.linalg.inv(Se)
        for i, a in enumerate((u, v)):
            for j, b in enumerate((u, v)):
                Sinv[a, b] += Ie[i, j]
    Dinv = np.diag(1.0 / d)
    return Dinv @ Sinv @ Dinv
