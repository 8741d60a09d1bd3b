"""Mesh, DOF numbering and FEM assembly on a metric graph (oracle, FP64).

Paper passages followed:

* Phase 1 (section "Algorithmic Implementation", subsection "Phase 1:
  Initialization"): every edge of length l_e gets n_e uniform elements with
  n_e = ceil(l_e / h), local size h_e = l_e / n_e, N_e = n_e + 1 nodes, and
  N = |V| + sum_e (N_e - 2) global nodes.
* Phase 2 (subsection "Phase 2: Global Setup and Noise Generation"): the
  consistent mass entries (2h/3 interior diagonal, h/6 couplings, sum h/3 at
  a vertex), the lumped mass (row sums: h_e inside an edge, sum of h_e/2 at a
  vertex) and the stiffness entries (2/h, -1/h, sum 1/h, -1/h), and the
  partition of the DOF vector into per-edge interior blocks followed by the
  vertex block ([W_I,1 ... W_I,|E| W_Gamma]).

Readings where the paper is silent:

* ``rule="round"`` uses n_e = floor(l_e/h + 1/2) (half-up) instead of the
  ceiling; both clamp n_e >= 1, and a self-loop gets n_e >= 2.
* Within an edge, interior node i = 1..n_e-1 runs from the tail vertex u_e
  (x = 0) to the head vertex v_e (x = l_e).
* Vertex lumped masses are summed over edges in increasing edge index, adding
  the tail end before the head end.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Mesh:
    n_vertices: int
    edges: np.ndarray  # [E, 2] int64
    lengths: np.ndarray  # [E] float64
    h: float
    n_el: np.ndarray  # [E] int64, elements per edge
    h_e: np.ndarray  # [E] float64, local mesh size
    offsets: np.ndarray  # [E+1] int64, first interior DOF of each edge

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    @property
    def n_interior(self) -> int:
        return int(self.offsets[-1])

    @property
    def n_dof(self) -> int:
        return self.n_interior + self.n_vertices

    def m(self, e: int) -> int:
        """Interior DOF count of edge e (N_e - 2)."""
        return int(self.n_el[e]) - 1

    def node(self, e: int, j: int) -> int:
        """Global DOF of local node j = 0..n_e on edge e (0 = tail vertex)."""
        n = int(self.n_el[e])
        if j == 0:
            return self.n_interior + int(self.edges[e, 0])
        if j == n:
            return self.n_interior + int(self.edges[e, 1])
        return int(self.offsets[e]) + j - 1

    def element_nodes(self) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
        """(a, b, h) for every element of every edge, a = left node, b = right."""
        a_list, b_list, h_list = [], [], []
        NI = self.n_interior
        for e in range(self.n_edges):
            n = int(self.n_el[e])
            nodes = np.empty(n + 1, dtype=np.int64)
            nodes[0] = NI + self.edges[e, 0]
            nodes[n] = NI + self.edges[e, 1]
            nodes[1:n] = self.offsets[e] + np.arange(n - 1)
            a_list.append(nodes[:-1])
            b_list.append(nodes[1:])
            h_list.append(np.full(n, self.h_e[e]))
        return np.concatenate(a_list), np.concatenate(b_list), np.concatenate(h_list)


def element_count(length: float, h: float, rule: str, self_loop: bool) -> int:
    """n_e for one edge: ceil(l/h) (paper, Phase 1) or floor(l/h + 1/2)."""
    q = length / h
    if rule == "ceil":
        n = math.ceil(q)
    elif rule == "round":
        n = math.floor(q + 0.5)
    else:
        raise ValueError(rule)
    return max(2 if self_loop else 1, int(n))


def build_mesh(n_vertices: int, edges: np.ndarray, lengths: np.ndarray, h: float, rule: str = "ceil") -> Mesh:
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    lengths = np.asarray(lengths, dtype=np.float64)
    if not (h > 0 and math.isfinite(h)):
        raise ValueError("h must be positive and finite")
    if not np.all(np.isfinite(lengths)) or np.any(lengths <= 0):
        raise ValueError("edge lengths must be positive and finite")
    if edges.size and (edges.min() < 0 or edges.max() >= n_vertices):
        raise ValueError("edge endpoint out of range")
    deg = np.bincount(edges.ravel(), minlength=n_vertices)
    if n_vertices <= 0 or np.any(deg == 0):
        raise ValueError("isolated vertex: its lumped mass is zero and the system is singular")
    n_el = np.array([element_count(float(lengths[e]), h, rule, bool(edges[e, 0] == edges[e, 1]))
                     for e in range(edges.shape[0])], dtype=np.int64)
    h_e = lengths / n_el.astype(np.float64)
    offsets = np.zeros(edges.shape[0] + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(n_el - 1)
    return Mesh(int(n_vertices), edges, lengths, float(h), n_el, h_e, offsets)


def lumped_mass(mesh: Mesh) -> np.ndarray:
    """Diagonal of the lumped mass matrix (paper, Phase 2, lumped case):
    h_e at every interior node of edge e, sum over incident edge ends of
    h_e/2 at a vertex."""
    NI = mesh.n_interior
    M = np.zeros(mesh.n_dof, dtype=np.float64)
    for e in range(mesh.n_edges):
        M[mesh.offsets[e]:mesh.offsets[e + 1]] = mesh.h_e[e]
    for e in range(mesh.n_edges):
        half = mesh.h_e[e] * 0.5
        M[NI + mesh.edges[e, 0]] += half
        M[NI + mesh.edges[e, 1]] += half
    return M


def _assemble(mesh: Mesh, k_aa: np.ndarray, k_ab: np.ndarray) -> sp.csr_matrix:
    a, b, _ = mesh.element_nodes()
    rows = np.concatenate([a, b, a, b])
    cols = np.concatenate([a, b, b, a])
    vals = np.concatenate([k_aa, k_aa, k_ab, k_ab])
    N = mesh.n_dof
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def stiffness(mesh: Mesh) -> sp.csr_matrix:
    """Global stiffness G: element matrices (1/h_e)[[1,-1],[-1,1]] summed,
    giving 2/h_e inside an edge, -1/h_e couplings, sum 1/h_e at a vertex."""
    _, _, he = mesh.element_nodes()
    return _assemble(mesh, 1.0 / he, -1.0 / he)


def consistent_mass(mesh: Mesh) -> sp.csr_matrix:
    """Global consistent mass M: element matrices (h_e/6)[[2,1],[1,2]],
    giving 2h_e/3 inside an edge, h_e/6 couplings, sum h_e/3 at a vertex."""
    _, _, he = mesh.element_nodes()
    return _assemble(mesh, he / 3.0, he / 6.0)
