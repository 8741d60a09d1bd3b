"""Pins of the learned-preconditioner oracle (CPU, FP64)."""

import math

import numpy as np
import pytest

from oracle import learned as ol
from oracle import mesh as omesh
from workloads import lattice, preferential_attachment
from workloads.learned_init import N_PARAMS, init_params


def _ragged():
    g = preferential_attachment(12, 2, lengths=(0.05, 1.7), seed=11)
    edges = np.vstack([g.edges, [[0, 1], [5, 5], [3, 12]]])
    lengths = np.concatenate([g.lengths, [0.013, 0.9, 0.31]])
    return 13, edges, lengths


def _system(V, edges, lengths, h=0.05, kappa=4.0, cI=0.7, cL=1.9):
    m = omesh.build_mesh(V, edges, lengths, h, "round")
    sd, so = ol.edge_schur(m, np.full(len(edges), kappa), cI, cL)
    f, w, D = ol.features(m, edges, lengths, sd, so, cI, cL, np.full(V, kappa))
    return m, sd, so, f, w, D


def test_layout_matches_init():
    assert ol.N_PARAMS == N_PARAMS


def test_edge_schur_matches_dense_schur():
    V, E, L = _ragged()
    m = omesh.build_mesh(V, E, L, 0.05, "round")
    for kappa, cI, cL in [(4.0, 0.7, 1.9), (1.0, 1e3, 1e-2), (10.0, 1e-3, 1e2)]:
        sd, so = ol.edge_schur(m, np.full(len(E), kappa), cI, cL)
        S = ol.schur_matrix(V, E, sd, so)
        S_ref = ol.dense_schur(m, kappa, cI, cL)
        assert np.abs(S - S_ref).max() <= 1e-10 * np.abs(S_ref).max()


def test_autograd_matches_finite_differences():
    V, E, L = _ragged()
    m, sd, so, f, w, D = _system(V, E, L)
    S = ol.schur_matrix(V, E, sd, so)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, V))
    G = X @ S  # S symmetric: rows g = S x
    theta = ol.effective_params(init_params(3, head_scale=0.3))
    L0, grad = ol.loss_and_grad(theta, f, w, E, V, D, G, X)
    import torch

    for _ in range(6):
        d = rng.standard_normal(theta.size)
        d /= np.linalg.norm(d)
        eps = 1e-6
        lp = float(ol.loss(torch.tensor(theta + eps * d), f, w, E, V, D, G, X))
        lm = float(ol.loss(torch.tensor(theta - eps * d), f, w, E, V, D, G, X))
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grad @ d) <= 1e-6 * max(1.0, abs(fd))


def test_preconditioner_is_spd_for_random_parameters():
    V, E, L = _ragged()
    m, sd, so, f, w, D = _system(V, E, L)
    for seed in range(4):
        theta = ol.effective_params(init_params(seed, head_scale=1.0))
        P, Q = ol.preconditioner(theta, f, w, E, V, D)
        assert np.allclose(P, P.T)
        assert np.linalg.eigvalsh(P).min() > 0


def test_jacobi_limit():
    """Zero head weights, delta = softplus(c_d) = 1 (c_d stored in float32: 1 to ~1e-8),
    p -> 0, gamma = 1, eta = 0: P = Q = D^{-1}."""
    V, E, L = _ragged()
    m, sd, so, f, w, D = _system(V, E, L)
    theta = init_params(0)
    P_ = ol.unpack(theta)
    for k in ("a_d", "a_g", "a_p1", "a_p2", "a_r", "a_e"):
        P_[k][:] = 0.0
    P_["c_p"][:] = -60.0
    P, Q = ol.preconditioner(ol.effective_params(theta), f, w, E, V, D)
    assert np.allclose(P, np.diag(1.0 / D), rtol=1e-7, atol=1e-25)
    assert np.allclose(Q, np.diag(1.0 / D), rtol=1e-14, atol=1e-30)


def test_reference_pcg_solves_with_learned_operators():
    g = lattice(4, 4, lengths=(0.5, 1.5), seed=2)
    m, sd, so, f, w, D = _system(g.n_vertices, g.edges, g.lengths, h=1 / 16)
    S = ol.schur_matrix(g.n_vertices, g.edges, sd, so)
    P, Q = ol.preconditioner(ol.effective_params(init_params(5, head_scale=0.5)), f, w, g.edges, g.n_vertices, D)
    b = np.random.default_rng(0).standard_normal(g.n_vertices)
    x, it = ol.pcg(S, b, P, Q @ b, 1e-12)
    assert it <= 200 and np.linalg.norm(S @ x - b) <= 1e-11 * np.linalg.norm(b)


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, -3.14159265, 1e-30], dtype=np.float32)
    r = ol.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0  # 1 + 2^-8 is a tie: rounds to even (1.0)
    assert r[2] == np.float32(1.0078125)  # above the tie: rounds up
    assert abs(r[3] + 3.140625) < 1e-7
    bits = r.view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)
    assert math.isclose(float(r[4]), 1e-30, rel_tol=1e-2)
