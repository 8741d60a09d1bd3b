"""Pins of the Neumann-Neumann preconditioner oracle (CPU, FP64)."""

import numpy as np
import pytest

from oracle import learned as ol
from oracle import mesh as omesh
from oracle import neumann as onn
from oracle import solve as osolve
from workloads import lattice, preferential_attachment

SHIFTS = [(4.0, 0.7, 1.9), (1.0, 1e3, 1e-2), (10.0, 1e-3, 1e2), (2.0, 1.0, 1e6)]


def _ragged():
    """Tree plus a multi-edge, a self-loop and a pendant vertex; ragged lengths."""
    g = preferential_attachment(12, 2, lengths=(0.05, 1.7), seed=11)
    edges = np.vstack([g.edges, [[0, 1], [5, 5], [3, 12]]])
    lengths = np.concatenate([g.lengths, [0.013, 0.9, 0.31]])
    return 13, edges, lengths


def test_thomas_solves_tridiagonal():
    rng = np.random.default_rng(0)
    for n in (1, 2, 3, 17):
        sub, sup = rng.uniform(-1, 1, n - 1), rng.uniform(-1, 1, n - 1)
        main = 3.0 + rng.uniform(0, 1, n)
        A = np.diag(main) + np.diag(sub, -1) + np.diag(sup, 1)
        b = rng.standard_normal(n)
        assert np.allclose(onn.thomas(sub, main, sup, b), np.linalg.solve(A, b), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kappa,cI,cL", SHIFTS)
def test_local_matrices_sum_to_shifted_matrix(kappa, cI, cL):
    V, E, L = _ragged()
    m = omesh.build_mesh(V, E, L, 0.05, "round")
    A = np.zeros((m.n_dof, m.n_dof))
    NI = m.n_interior
    for e in range(m.n_edges):
        sub, main, sup = onn.edge_tridiag(m, e, kappa, cI, cL)
        nodes = np.concatenate([[NI + E[e, 0]], m.offsets[e] + np.arange(m.m(e)), [NI + E[e, 1]]])
        for i, a in enumerate(nodes):
            A[a, a] += main[i]
            if i + 1 < len(nodes):
                A[a, nodes[i + 1]] += sup[i]
                A[nodes[i + 1], a] += sub[i]
    A_ref = osolve.shifted_matrix(m, kappa, cI, cL).toarray()
    assert np.abs(A - A_ref).max() <= 1e-12 * np.abs(A_ref).max()


@pytest.mark.parametrize("kappa,cI,cL", SHIFTS)
def test_local_schur_is_edge_block(kappa, cI, cL):
    V, E, L = _ragged()
    m = omesh.build_mesh(V, E, L, 0.05, "round")
    sd, so = ol.edge_schur(m, np.full(len(E), kappa), cI, cL)
    for e in range(m.n_edges):
        sub, main, sup = onn.edge_tridiag(m, e, kappa, cI, cL)
        A = np.diag(main) + np.diag(sub, -1) + np.diag(sup, 1)
        ends, inner = [0, len(main) - 1], list(range(1, len(main) - 1))
        Sl = A[np.ix_(ends, ends)]
        if inner:
            Sl = Sl - A[np.ix_(ends, inner)] @ np.linalg.solve(A[np.ix_(inner, inner)], A[np.ix_(inner, ends)])
        ref = np.array([[sd[e], so[e]], [so[e], sd[e]]])
        assert np.abs(Sl - ref).max() <= 1e-11 * np.abs(ref).max(), e


@pytest.mark.parametrize("kappa,cI,cL", SHIFTS)
def test_neumann_step_is_closed_form(kappa, cI, cL):
    V, E, L = _ragged()
    m = omesh.build_mesh(V, E, L, 0.05, "round")
    ke = np.linspace(0.5, 1.5, len(E)) * kappa  # per-edge kappa
    sd, so = ol.edge_schur(m, ke, cI, cL)
    P = onn.nn_matrix(V, E, sd, so)
    rng = np.random.default_rng(2)
    for _ in range(3):
        r = rng.standard_normal(V)
        z = onn.neumann_step(m, ke, cI, cL, r)
        zr = P @ r
        assert np.linalg.norm(z - zr) <= 1e-11 * np.linalg.norm(zr)


@pytest.mark.parametrize("kappa,cI,cL", SHIFTS)
def test_single_edge_is_exact(kappa, cI, cL):
    m = omesh.build_mesh(2, np.array([[0, 1]]), np.array([0.83]), 0.05, "round")
    sd, so = ol.edge_schur(m, np.array([kappa]), cI, cL)
    S = ol.schur_matrix(2, m.edges, sd, so)
    P = onn.nn_matrix(2, m.edges, sd, so)
    assert np.abs(P @ S - np.eye(2)).max() <= 1e-12
    g = np.array([0.3, -1.7])
    x, it = ol.pcg(S, g, P, np.zeros(2), 1e-12)
    assert it == 1
    assert np.allclose(x, np.linalg.solve(S, g), rtol=1e-12)


def test_jacobi_limit():
    """With no stiffness (c_L = 0) the edges decouple, S_e = diag(sd_e), and on a
    lattice of unit edges every vertex sees equal sd_e: then
    D^{-1} (sum_e S_e^{-1}) D^{-1} = diag(1 / (d_v sd)) = diag(S)^{-1}."""
    g = lattice(4, 5)
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, 0.1, "ceil")
    sd, so = ol.edge_schur(m, np.full(len(g.edges), 3.0), 2.0, 0.0)
    S = ol.schur_matrix(g.n_vertices, g.edges, sd, so)
    P = onn.nn_matrix(g.n_vertices, g.edges, sd, so)
    assert np.abs(P - np.diag(1.0 / np.diag(S))).max() <= 1e-13 * np.abs(P).max()
    # with unequal lengths the two differ (harmonic against arithmetic mean)
    g2 = lattice(4, 5, lengths=(0.5, 1.5), seed=3)
    m2 = omesh.build_mesh(g2.n_vertices, g2.edges, g2.lengths, 0.1, "ceil")
    sd2, so2 = ol.edge_schur(m2, np.full(len(g2.edges), 3.0), 2.0, 0.0)
    S2 = ol.schur_matrix(g2.n_vertices, g2.edges, sd2, so2)
    P2 = onn.nn_matrix(g2.n_vertices, g2.edges, sd2, so2)
    assert np.all(np.diag(P2) >= 1.0 / np.diag(S2) * (1 - 1e-14))
    assert np.abs(np.diag(P2) - 1.0 / np.diag(S2)).max() > 1e-3 * np.abs(np.diag(P2)).max()


@pytest.mark.parametrize("kappa,cI,cL", SHIFTS)
def test_spd_and_convergence(kappa, cI, cL):
    V, E, L = _ragged()
    m = omesh.build_mesh(V, E, L, 0.05, "round")
    sd, so = ol.edge_schur(m, np.full(len(E), kappa), cI, cL)
    S = ol.schur_matrix(V, E, sd, so)
    P = onn.nn_matrix(V, E, sd, so)
    assert np.abs(P - P.T).max() <= 1e-14 * np.abs(P).max()
    assert np.linalg.eigvalsh(P).min() > 0
    g = np.random.default_rng(4).standard_normal(V)
    x, it = ol.pcg(S, g, P, np.zeros(V), 1e-12)
    assert it <= 2 * V  # finite termination holds up to rounding only
    assert np.linalg.norm(S @ x - g) <= 1e-11 * np.linalg.norm(g)
