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


def test_features_hand_computed():
    """Features on a 4-vertex graph with a multi-edge (0-1 twice, opposite
    orientations) and a self-loop at vertex 2, with chosen edge Schur blocks.
    Every expected value below is worked out by hand from the definitions:
    a self-loop is two edge ends at its vertex (degree, length statistics and
    coupling sum count it twice), and its 2x2 block [[s_d, s_o], [s_o, s_d]]
    adds 2 s_d + 2 s_o to the diagonal of S."""
    edges = np.array([[0, 1], [1, 0], [1, 2], [2, 2], [2, 3]])
    lengths = np.array([1.0, 2.0, 0.5, 1.5, 1.0])
    sd = np.array([2.0, 3.0, 4.0, 5.0, 6.0])
    so = np.array([-1.0, -1.0, -0.5, -1.0, -2.0])
    m = omesh.build_mesh(4, edges, lengths, 0.25, "round")
    cI, cL = 0.5, 4.0
    kap = np.array([2.0, 2.0, 2.0, 2.0])
    f, w, D = ol.features(m, edges, lengths, sd, so, cI, cL, kap)
    # D_0 = 2 + 3, D_1 = 2 + 3 + 4, D_2 = 4 + 2*5 + 2*(-1) + 6, D_3 = 6
    assert np.array_equal(D, [5.0, 9.0, 18.0, 6.0])
    s45, s162, s108 = math.sqrt(45.0), math.sqrt(162.0), math.sqrt(108.0)
    w_ref = [1 / s45, 1 / s45, 0.5 / s162, 1 / 18, 2 / s108]
    assert np.allclose(w, w_ref, rtol=1e-15, atol=0)
    ref = np.array([
        # log(1 + deg), mean length, min, max, log(cL/cI)/10, log(kappa)/3, sum of w, 1
        [math.log(3), 1.5, 1.0, 2.0, math.log(8) / 10, math.log(2) / 3, 2 / s45, 1.0],
        [math.log(4), 3.5 / 3, 0.5, 2.0, math.log(8) / 10, math.log(2) / 3, 2 / s45 + 0.5 / s162, 1.0],
        [math.log(5), 4.5 / 4, 0.5, 1.5, math.log(8) / 10, math.log(2) / 3, 0.5 / s162 + 2 / 18 + 2 / s108,
         1.0],
        [math.log(2), 1.0, 1.0, 1.0, math.log(8) / 10, math.log(2) / 3, 2 / s108, 1.0],
    ])
    assert np.allclose(f, ref, rtol=1e-14, atol=0)


def test_reference_pcg_stops_on_true_residual():
    """The stopping decision uses g - S x recomputed from x: with an SPD S and
    the identity preconditioner, the returned iterate meets the bar, the one
    before it does not, and the iteration count equals that of a plain CG
    written out here step by step with the true residual tested."""
    rng = np.random.default_rng(7)
    A = rng.standard_normal((30, 30))
    S = A @ A.T + 30 * np.eye(30)
    g = rng.standard_normal(30)
    tol = 1e-9
    x, it = ol.pcg(S, g, np.eye(30), np.zeros(30), tol)
    assert np.linalg.norm(g - S @ x) <= tol * np.linalg.norm(g)
    # plain CG, iterate by iterate
    xs, r = np.zeros(30), g.copy()
    p, k = r.copy(), 0
    while np.linalg.norm(g - S @ xs) > tol * np.linalg.norm(g):
        q = S @ p
        a = (r @ r) / (p @ q)
        xs = xs + a * p
        rn = r - a * q
        p = rn + ((rn @ rn) / (r @ r)) * p
        r = rn
        k += 1
    assert it == k and k > 3
    assert np.allclose(x, xs, rtol=1e-12, atol=1e-14)
    # zero right-hand side: x = 0 after 0 iterations
    x0, it0 = ol.pcg(S, np.zeros(30), np.eye(30), np.ones(30), tol)
    assert it0 == 0 and not x0.any()
    # non-convergence is flagged as maxit + 1
    _, itm = ol.pcg(S, g, np.eye(30), np.zeros(30), 1e-30, maxit=5)
    assert itm == 6


def test_reference_pcg_falls_back_to_jacobi():
    """A preconditioner that ruins the conditioning (diagonal entries spread
    over eight decades) is replaced by the fallback after maxit // 2
    iterations, from the current iterate; the iteration then converges as
    Jacobi-PCG does, while without the fallback it does not within maxit."""
    n = 200
    rng = np.random.default_rng(3)
    A = rng.standard_normal((n, n))
    S = A @ A.T / n + np.eye(n)
    g = rng.standard_normal(n)
    J = np.diag(1.0 / np.diag(S))
    bad = np.diag(rng.permutation(np.logspace(-8, 0, n)))
    maxit = 80
    _, it_j = ol.pcg(S, g, J, np.zeros(n), 1e-10, maxit=maxit)
    assert it_j < maxit // 2
    x, it = ol.pcg(S, g, bad, np.zeros(n), 1e-10, maxit=maxit, fallback=J)
    assert np.linalg.norm(g - S @ x) <= 1e-10 * np.linalg.norm(g)
    assert maxit // 2 < it <= maxit // 2 + it_j
    _, it_nf = ol.pcg(S, g, bad, np.zeros(n), 1e-10, maxit=maxit)
    assert it_nf == maxit + 1


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, -3.14159265, 1e-30], dtype=np.float32)
    r = ol.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0  # 1 + 2^-8 is a tie: rounds to even (1.0)
    assert r[2] == np.float32(1.0078125)  # above the tie: rounds up
    assert abs(r[3] + 3.140625) < 1e-7
    bits = r.view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)
    assert math.isclose(float(r[4]), 1e-30, rel_tol=1e-2)
