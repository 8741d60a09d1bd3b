"""Neumann-Neumann preconditioner of the vertex Schur PCG through the C ABI.

* exactness: on k parallel edges of equal length between two vertices,
  D^{-1} (sum_e S_e^{-1}) D^{-1} = (k S_e)^{-1} = S^{-1}, so every system ends
  after one PCG step (Jacobi needs more: the components' scaled blocks have
  different eigenvalues, and CG runs on their union);
* the sample of the 4x4 lattice workload (16 vertices, h = 1/64, 55 shifts,
  16 samples) equals the FP64 oracle to 1e-10 in the lumped-mass norm, and
  the PCG iteration totals with Jacobi and with Neumann-Neumann each lie
  within 10% of the oracle's PCG with the same preconditioner on the same
  systems (the oracle halves the count: 4464 against 2320);
* a shifted solve on a ragged graph (self-loop, multi-edge, vertices of
  degree above four) equals the oracle's direct solve, with an iteration
  total within 10% of the oracle's.
"""

import numpy as np
import pytest

from oracle import learned as ol
from oracle import mesh as omesh
from oracle import neumann as onn
from oracle import noise as onoise
from oracle import quadrature as oquad
from oracle import solve as osolve
from workloads import config_c1, preferential_attachment

pytestmark = pytest.mark.gpu


def _rel_ml(u, ref, ML):
    """Worst sample's relative error, the larger of the lumped-mass norm
    ||u - ref||_{M_L} / ||ref||_{M_L} and the element-wise max |u - ref| / max |ref|
    (a local error that the norm would dilute fails the second)."""
    num = np.sqrt(((u - ref) ** 2 * ML).sum(axis=-1))
    den = np.sqrt((ref ** 2 * ML).sum(axis=-1))
    el = np.abs(u - ref).max(axis=-1) / np.abs(ref).max(axis=-1)
    return float(max(np.max(num / den), np.max(el)))


def _ragged():
    g = preferential_attachment(12, 2, lengths=(0.05, 1.7), seed=11)
    edges = np.vstack([g.edges, [[0, 1], [5, 5], [3, 12]]])
    lengths = np.concatenate([g.lengths, [0.013, 0.9, 0.31]])
    return 13, edges, lengths


def _oracle_iterations(m, kappa, cI, cL, B, tol):
    """Total PCG iterations (Jacobi, Neumann-Neumann) of the oracle on the vertex
    Schur systems of the rows of B (condensed with dense solves)."""
    V, ni = m.n_vertices, m.n_interior
    A = osolve.shifted_matrix(m, kappa, cI, cL).toarray()
    Aii, Aiv, Avv = A[:ni, :ni], A[:ni, ni:], A[ni:, ni:]
    Y = np.linalg.solve(Aii, np.hstack([Aiv, B[:, :ni].T])) if ni else np.zeros((0, V + B.shape[0]))
    S = Avv - Aiv.T @ Y[:, :V]
    G = B[:, ni:] - (Aiv.T @ Y[:, V:]).T
    sd, so = ol.edge_schur(m, np.full(m.n_edges, kappa), cI, cL)
    P = onn.nn_matrix(V, m.edges, sd, so)
    J = np.diag(1.0 / np.diag(S))
    tj = sum(ol.pcg(S, g, J, np.zeros(V), tol)[1] for g in G)
    tn = sum(ol.pcg(S, g, P, np.zeros(V), tol)[1] for g in G)
    return tj, tn


def test_nn_exact_on_parallel_edges(grf):
    # components: one edge; two equal parallel edges; three equal parallel edges
    edges = np.array([[0, 1], [2, 3], [2, 3], [4, 5], [5, 4], [4, 5]])
    lengths = np.array([0.83, 1.3, 1.3, 0.6, 0.6, 0.6])
    G = grf.Graph(6, edges, lengths, 1.0 / 32, "round")
    m = omesh.build_mesh(6, edges, lengths, 1.0 / 32, "round")
    ML = omesh.lumped_mass(m)
    kappa, beta, k, S, seed = 3.0, 0.7, 0.4, 8, 21
    ref = osolve.sample(m, kappa, beta, k, onoise.white_noise(ML, seed, S))
    u, st = G.sample(kappa, beta, k, S, seed, precond="nn")
    print(f"NN: max iterations {st['max_iterations']}, total {st['total_iterations']} / {st['n_systems']}", flush=True)
    assert st["n_unconverged"] == 0
    assert st["max_iterations"] == 1
    assert _rel_ml(u.cpu().numpy(), ref, ML) <= 1e-10
    _, stj = G.sample(kappa, beta, k, S, seed)
    assert stj["max_iterations"] >= 2


def test_nn_c1_matches_oracle(grf):
    cfg = config_c1()
    g = cfg["graph"]
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    ML = omesh.lumped_mass(m)
    W = onoise.white_noise(ML, cfg["seed"], cfg["n_samples"])
    ref = osolve.sample(m, cfg["kappa"], cfg["beta"], cfg["quad_step"], W)
    tj = tn = 0
    for _, cI, cL in zip(*oquad.shifts(cfg["beta"], cfg["quad_step"])):
        a, b = _oracle_iterations(m, cfg["kappa"], cI, cL, W, cfg["tol"])
        tj, tn = tj + a, tn + b
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    args = (cfg["kappa"], cfg["beta"], cfg["quad_step"], cfg["n_samples"], cfg["seed"])
    u, st = G.sample(*args, tol=cfg["tol"], precond="nn")
    uj, stj = G.sample(*args, tol=cfg["tol"])
    print(f"iterations: oracle Jacobi {tj}, NN {tn}; GPU Jacobi {stj['total_iterations']}, "
          f"NN {st['total_iterations']} over {st['n_systems']} systems", flush=True)
    assert st["n_unconverged"] == 0
    assert _rel_ml(u.cpu().numpy(), ref, ML) <= 1e-10
    assert _rel_ml(uj.cpu().numpy(), ref, ML) <= 1e-10
    assert abs(st["total_iterations"] - tn) <= 0.1 * tn
    assert abs(stj["total_iterations"] - tj) <= 0.1 * tj


def test_nn_solve_shifted_ragged(grf):
    import torch

    V, E, L = _ragged()
    m = omesh.build_mesh(V, E, L, 0.07, "round")
    assert np.bincount(E.ravel(), minlength=V).max() > 4  # ELL overflow slots in use
    G = grf.Graph(V, E, L, 0.07, "round")
    B = np.random.default_rng(5).standard_normal((67, m.n_dof))
    for kappa, cI, cL in [(3.0, 1e-3, 5e3), (8.0, 1.0, 1.0), (2.0, 1e2, 1e-6)]:
        x, st = G.solve_shifted(kappa, cI, cL, torch.from_numpy(B).cuda(), precond="nn")
        ref = osolve.solve_shifted(m, kappa, cI, cL, B)
        _, tn = _oracle_iterations(m, kappa, cI, cL, B, 1e-12)
        print(f"kappa {kappa} c_I {cI} c_L {cL}: GPU {st['total_iterations']}, oracle {tn}", flush=True)
        assert st["n_unconverged"] == 0
        assert _rel_ml(x.cpu().numpy(), ref, omesh.lumped_mass(m)) <= 1e-10
        assert abs(st["total_iterations"] - tn) <= 0.1 * tn + 2
