"""Pins for the oracle's quadrature and solves (CPU only).

Checked against: the scalar sinc-quadrature error law, brute-force dense
solves, the generalised eigen-route, the closed-form Neumann cosine expansion
on one interval, conservation and Kirchhoff identities, the exact method
covariance (Monte Carlo), and the convergence rates of the paper's Table 1
(tests/golden/paper_table1_rates.txt) reproduced on a scaled-down interval
experiment.
"""

import math
import os

import numpy as np
import pytest

from oracle import mesh, noise, quadrature, solve, spectral
from workloads import interval, lattice, preferential_attachment

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_limits_c1():
    # k = 0.5, beta = 0.75: K^- = ceil(pi^2/0.75) = 14, K^+ = ceil(pi^2/0.25) = 40
    assert quadrature.limits(0.75, 0.5) == (14, 40)
    l, cI, cL = quadrature.shifts(0.75, 0.5)
    assert l[0] == -14 and l[-1] == 40 and l.size == 55
    c_const = math.pi / (2 * 0.5 * math.sin(0.75 * math.pi))
    i0 = 14  # l = 0
    assert cI[i0] == pytest.approx(c_const) and cL[i0] == pytest.approx(c_const)
    assert cL[i0 + 1] / cI[i0 + 1] == pytest.approx(math.exp(2 * 0.5))


@pytest.mark.parametrize("beta", [0.3, 0.55, 0.75, 0.9])
@pytest.mark.parametrize("k", [0.5, 0.3, 0.2])
def test_scalar_quadrature_error_law(beta, k):
    # sum_l 1/(c_I + c_L lam) -> lam^{-beta} with absolute error O(exp(-pi^2/(2k)))
    lam = np.geomspace(1.0, 1e6, 200)
    err = np.abs(quadrature.q_k(lam, beta, k) - lam ** -beta)
    assert err.max() <= 4.0 * math.exp(-math.pi ** 2 / (2 * k))


def test_paper_step_rule():
    assert quadrature.paper_step(0.75, 1 / 128) == pytest.approx(0.2748, abs=1e-4)
    assert quadrature.paper_step(0.75, 1 / 256) == pytest.approx(0.2404, abs=1e-4)


def _graphs():
    g1 = lattice(2, 3, lengths=(0.4, 1.3), seed=2)
    g2 = preferential_attachment(7, 2, lengths=(0.2, 1.0), seed=3)
    e = np.vstack([g1.edges, [[0, 1], [3, 3]]])
    L = np.concatenate([g1.lengths, [0.6, 0.8]])
    return [(g1.n_vertices, g1.edges, g1.lengths), (g2.n_vertices, g2.edges, g2.lengths),
            (g1.n_vertices, e, L)]


@pytest.mark.parametrize("gi", range(3))
def test_dense_sparse_eig_agree(gi):
    V, E, L = _graphs()[gi]
    m = mesh.build_mesh(V, E, L, 0.09, "round")
    W = noise.white_noise(mesh.lumped_mass(m), 4, 3)
    kappa, beta, k = 3.0, 0.65, 0.4
    us = solve.sample(m, kappa, beta, k, W, method="sparse")
    ud = solve.sample(m, kappa, beta, k, W, method="dense")
    ue = spectral.eig_sample(m, kappa, beta, k, W)
    scale = np.abs(ud).max()
    assert np.abs(us - ud).max() <= 1e-13 * scale
    assert np.abs(ue - ud).max() <= 1e-10 * scale


@pytest.mark.parametrize("length,h,kappa,beta,k", [(1.0, 1 / 64, 5.0, 0.75, 0.5),
                                                   (2.3, 0.05, 1.0, 0.4, 0.3),
                                                   (0.7, 0.01, 12.0, 0.9, 0.25)])
def test_interval_closed_form(length, h, kappa, beta, k):
    g = interval(length)
    m = mesh.build_mesh(2, g.edges, g.lengths, h, "ceil")
    W = noise.white_noise(mesh.lumped_mass(m), 9, 4)
    u = solve.sample(m, kappa, beta, k, W, method="sparse")
    uc = spectral.interval_sample(length, int(m.n_el[0]), kappa, beta, k, W)
    assert np.abs(u - uc).max() <= 1e-11 * np.abs(uc).max()


@pytest.mark.parametrize("length,h,kappa,beta,k", [(1.0, 1 / 32, 3.0, 0.75, 0.4), (2.5, 0.1, 0.7, 0.55, 0.3),
                                                   (0.3, 0.05, 25.0, 0.85, 0.5)])
def test_interval_closed_form_consistent_mass(length, h, kappa, beta, k):
    """Consistent mass in the shifted systems (the paper's Phase 2 consistent
    entries): the direct solves equal the cosine expansion with the consistent
    eigenvalue ratio c_n = (2 + cos theta_n)/3.  The shifts span matrices whose
    interior coupling alpha h/6 - gamma/h takes both signs."""
    g = interval(length)
    m = mesh.build_mesh(2, g.edges, g.lengths, h, "ceil")
    W = noise.white_noise(mesh.lumped_mass(m), 4, 3)
    u = solve.sample(m, kappa, beta, k, W, method="sparse", mass="consistent")
    uc = spectral.interval_sample(length, int(m.n_el[0]), kappa, beta, k, W, mass="consistent")
    assert np.abs(u - uc).max() <= 1e-11 * np.abs(uc).max()
    ul = spectral.interval_sample(length, int(m.n_el[0]), kappa, beta, k, W)
    assert np.abs(ul - uc).max() > 1e-6 * np.abs(uc).max()  # the two systems differ
    _, cI, cL = quadrature.shifts(beta, k)
    hh = length / int(m.n_el[0])
    b = (cI + cL * kappa * kappa) * hh / 6.0 - cL / hh
    assert (b > 0).any() and (b < 0).any()


def test_conservation_per_shift_and_sum():
    V, E, L = _graphs()[2]
    m = mesh.build_mesh(V, E, L, 0.07, "round")
    ML = mesh.lumped_mass(m)
    W = noise.white_noise(ML, 5, 2)
    kappa, beta, k = 2.0, 0.6, 0.45
    u, parts = solve.sample(m, kappa, beta, k, W, per_shift=True)
    _, cI, cL = quadrature.shifts(beta, k)
    for ul, ci, cl in zip(parts, cI, cL):
        lhs = (ul * ML).sum(axis=1)
        rhs = W.sum(axis=1) / (ci + cl * kappa ** 2)
        assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-14 * np.abs(rhs).max())
    q = quadrature.q_k(kappa ** 2, beta, k)
    assert np.allclose((u * ML).sum(axis=1), q * W.sum(axis=1), rtol=1e-11)


def test_kirchhoff_vertex_balance():
    # vertex rows of A u = W written as a discrete flux balance, walking edges:
    # gamma * sum_{edge ends at v} (u_v - u_adj)/h_e = W_v - alpha * M_vv * u_v
    V, E, L = _graphs()[2]
    m = mesh.build_mesh(V, E, L, 0.07, "round")
    ML = mesh.lumped_mass(m)
    W = noise.white_noise(ML, 6, 1)[0]
    kappa, cI, cL = 2.5, 0.8, 1.7
    u = solve.solve_shifted(m, kappa, cI, cL, W)
    alpha, gamma = cI + cL * kappa ** 2, cL
    NI = m.n_interior
    flux = np.zeros(V)
    for e in range(m.n_edges):
        n = int(m.n_el[e])
        a, b = m.node(e, 0), m.node(e, 1)
        flux[m.edges[e, 0]] += (u[a] - u[b]) / m.h_e[e]
        a, b = m.node(e, n), m.node(e, n - 1)
        flux[m.edges[e, 1]] += (u[a] - u[b]) / m.h_e[e]
    res = gamma * flux - (W[NI:] - alpha * ML[NI:] * u[NI:])
    assert np.abs(res).max() <= 1e-10 * np.abs(W).max()


def test_method_covariance_monte_carlo():
    g = interval(1.0)
    m = mesh.build_mesh(2, g.edges, g.lengths, 0.25, "ceil")  # N = 5
    kappa, beta, k = 1.5, 0.7, 0.5
    S = 20000
    W = noise.white_noise(mesh.lumped_mass(m), 21, S)
    u = spectral.eig_sample(m, kappa, beta, k, W)
    C = spectral.eig_covariance(m, kappa, beta, k)
    Cs = u.T @ u / S
    sd = np.sqrt((np.outer(np.diag(C), np.diag(C)) + C * C) / S)
    assert np.all(np.abs(Cs - C) <= 5 * sd)


# ---- convergence rates (paper Table 1), scaled down -------------------------

def _prolong(nc, nf):
    r = nf // nc
    P = np.zeros((nf + 1, nc + 1))
    for f in range(nf + 1):
        c, t = divmod(f, r)
        if c == nc:
            P[f, nc] = 1.0
        else:
            P[f, c] += 1 - t / r
            P[f, c + 1] += t / r
    return P


def _order(n):
    return np.concatenate([np.arange(1, n), [0, n]])


def _interval_op(n, kappa, beta, k):
    """Node-order load vector -> node-order solution, closed form."""
    o = _order(n)
    I = np.eye(n + 1)
    sol = spectral.interval_sample(1.0, n, kappa, beta, k, I[:, o])  # row r = unit load at node r
    out = np.zeros((n + 1, n + 1))
    out[:, o] = sol
    return out.T


def _rates(beta, kappa=1.0, pf=11, pc=10, levels=(3, 4, 5, 6), R=100):
    nf = 2 ** pf
    hf = 1.0 / nf
    wf = np.full(nf + 1, hf)
    wf[0] = wf[-1] = hf / 2
    rng = np.random.default_rng(0)
    Wn = rng.standard_normal((R, nf + 1)) * np.sqrt(wf)
    o = _order(nf)
    uf = np.zeros_like(Wn)
    uf[:, o] = spectral.interval_sample(1.0, nf, kappa, beta, quadrature.paper_step(beta, hf), Wn[:, o])
    nr = 2 ** pc  # covariance reference mesh
    Ff = _interval_op(nr, kappa, beta, quadrature.paper_step(beta, 1.0 / nr))
    wr = np.full(nr + 1, 1.0 / nr)
    wr[0] = wr[-1] = 0.5 / nr
    Cf = Ff @ np.diag(wr) @ Ff.T
    strong, cov, hs = [], [], []
    for lv in levels:
        nc = 2 ** lv
        hc = 1.0 / nc
        kc = quadrature.paper_step(beta, hc)
        P = _prolong(nc, nf)
        Wc = Wn @ P  # noise projected from the overkill mesh
        oc = _order(nc)
        uc = np.zeros((R, nc + 1))
        uc[:, oc] = spectral.interval_sample(1.0, nc, kappa, beta, kc, Wc[:, oc])
        e = uf - uc @ P.T
        strong.append(math.sqrt(((e * e) * wf).sum(axis=1).mean()))
        Pr = _prolong(nc, nr)
        G = Pr @ _interval_op(nc, kappa, beta, kc) @ Pr.T
        D = Cf - G @ np.diag(wr) @ G.T
        cov.append(math.sqrt((D * D * wr[:, None] * wr[None, :]).sum()))
        hs.append(hc)
    lh = np.log(hs)
    return np.polyfit(lh, np.log(strong), 1)[0], np.polyfit(lh, np.log(cov), 1)[0]


def _table1():
    rows = []
    with open(os.path.join(GOLDEN, "paper_table1_rates.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(x) for x in line.split()])
    return rows


@pytest.mark.parametrize("row", range(5))
def test_convergence_rates_table1(row):
    beta, strong_paper, cov_paper, strong_th, cov_th = _table1()[row]
    strong, cov = _rates(beta)
    # strong rate: the paper measures within 0.01 of 2 beta - 1/2; the
    # scaled-down interval experiment (2^3..2^6 elements) lands within 0.03
    # of both
    assert abs(strong - strong_th) <= 0.04
    assert abs(strong - strong_paper) <= 0.04
    # covariance rate: within 0.1 of the theoretical min(4 beta - 1/2, 2) and
    # of the paper's measurement (which itself sits up to 0.09 off theory);
    # measured 1.02, 1.55, 1.92, 2.01, 2.03 against a 2^10 reference mesh
    assert abs(cov - cov_th) <= 0.1
    assert abs(cov - cov_paper) <= 0.1
