"""Pins for the oracle's mesh and assembly (CPU only).

Checked against: the DOF counts printed in the paper's performance tables
(tests/golden/paper_ba_dofs.txt), the closed-form matrix entries and the
lumping identities of Phase 2, and conservation identities (G 1 = 0, row sums
of the consistent mass equal the lumped mass, total mass = total length).
"""

import os

import numpy as np
import pytest

from oracle import mesh
from workloads import lattice, preferential_attachment

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(x) for x in line.split()])
    return np.array(rows)


def test_c1_lattice_counts():
    g = lattice(4, 4)
    m = mesh.build_mesh(g.n_vertices, g.edges, g.lengths, 1 / 64, "ceil")
    assert g.n_edges == 24
    assert np.all(m.n_el == 64)
    assert m.n_interior == 24 * 63 and m.n_dof == 1528


@pytest.mark.parametrize("row", range(6))  # the two largest graphs are slow to generate
def test_paper_ba_dof_counts(row):
    n, n_printed = _golden("paper_ba_dofs.txt")[row]
    n = int(n)
    g = preferential_attachment(n, 2, seed=row)
    assert g.n_edges == 2 * (n - 2)
    m = mesh.build_mesh(g.n_vertices, g.edges, g.lengths, 2.0 ** -6, "ceil")
    # N = |V| + sum_e (N_e - 2) (Phase 1); the printed N counts interior DOFs only
    assert m.n_interior == int(n_printed)
    assert m.n_dof == int(n_printed) + n


def test_mesh_rules():
    e = np.array([[0, 1], [1, 2], [2, 2]], dtype=np.int64)
    L = np.array([1.0, 0.30, 0.05])
    mc = mesh.build_mesh(3, e, L, 0.25, "ceil")
    mr = mesh.build_mesh(3, e, L, 0.25, "round")
    assert mc.n_el.tolist() == [4, 2, 2]  # ceil(1.2)=2; self-loop clamped to 2
    assert mr.n_el.tolist() == [4, 1, 2]  # floor(1.2+0.5)=1
    assert np.allclose(mr.h_e, L / mr.n_el)
    assert mr.offsets.tolist() == [0, 3, 3, 4]
    with pytest.raises(ValueError):
        mesh.build_mesh(4, e, L, 0.25)  # vertex 3 isolated
    with pytest.raises(ValueError):
        mesh.build_mesh(3, e, np.array([1.0, -1.0, 1.0]), 0.25)


def _small_graph():
    g = lattice(3, 2, lengths=(0.3, 1.2), seed=5)
    # add a multi-edge and a self-loop
    edges = np.vstack([g.edges, [[0, 1], [4, 4]]])
    lengths = np.concatenate([g.lengths, [0.7, 0.9]])
    return mesh.build_mesh(g.n_vertices, edges, lengths, 0.1, "round")


def test_lumped_mass_entries():
    m = _small_graph()
    ML = mesh.lumped_mass(m)
    NI = m.n_interior
    for e in range(m.n_edges):
        assert np.all(ML[m.offsets[e]:m.offsets[e + 1]] == m.h_e[e])
    for v in range(m.n_vertices):
        ends = [m.h_e[e] / 2 for e in range(m.n_edges) for side in (0, 1) if m.edges[e, side] == v]
        assert np.isclose(ML[NI + v], sum(ends), rtol=1e-15)
    assert np.isclose(ML.sum(), m.lengths.sum(), rtol=1e-13)


def test_consistent_mass_and_stiffness_entries():
    m = _small_graph()
    M = mesh.consistent_mass(m).toarray()
    G = mesh.stiffness(m).toarray()
    ML = mesh.lumped_mass(m)
    NI = m.n_interior
    assert np.allclose(M.sum(axis=1), ML, rtol=1e-13)  # lumping = row sums
    assert np.allclose(G.sum(axis=1), 0.0, atol=1e-9 * np.abs(G).max())
    assert np.allclose(M, M.T) and np.allclose(G, G.T)
    e = 0
    i0 = int(m.offsets[e]) + 1  # an interior node with interior neighbours
    he = m.h_e[e]
    assert np.isclose(M[i0, i0], 2 * he / 3) and np.isclose(M[i0, i0 + 1], he / 6)
    assert np.isclose(G[i0, i0], 2 / he) and np.isclose(G[i0, i0 + 1], -1 / he)
    u = NI + int(m.edges[e, 0])
    first = int(m.offsets[e])
    assert np.isclose(M[u, first], he / 6) and np.isclose(G[u, first], -1 / he)
    for v in range(m.n_vertices):
        inc = [m.h_e[k] for k in range(m.n_edges) for side in (0, 1) if m.edges[k, side] == v]
        loops = [k for k in range(m.n_edges) if m.edges[k, 0] == v and m.edges[k, 1] == v]
        assert np.isclose(M[NI + v, NI + v], sum(h / 3 for h in inc))
        if not loops:
            assert np.isclose(G[NI + v, NI + v], sum(1 / h for h in inc))
