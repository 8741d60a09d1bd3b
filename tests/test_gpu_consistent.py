"""Consistent mass in the shifted systems (GRF_MASS_CONSISTENT_SYS; paper
Phase 2, consistent mass entries), through the C ABI, against the FP64 oracle.

The interior coupling b = alpha h/6 - gamma/h of a consistent-mass system
changes sign across the quadrature shifts; the library runs the streamed
Thomas sweeps with a sign-alternating similarity where b > 0 and a diagonal
interior block where b = 0.  Bar: 1e-10 relative in the lumped-mass norm per
sample, and max |u - ref| <= 1e-10 max |ref| element by element, with the
vertex PCG at tol 1e-12.  The noise is the lumped Philox noise in both.
"""

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import noise as onoise
from oracle import quadrature as oquad
from oracle import solve as osolve
from workloads import config_c1, interval, lattice, preferential_attachment

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _rel_ml(u, ref, ML):
    """Worst sample's relative error, the larger of the lumped-mass norm
    ||u - ref||_{M_L} / ||ref||_{M_L} and the element-wise max |u - ref| / max |ref|
    (a local error that the norm would dilute fails the second)."""
    num = np.sqrt(((u - ref) ** 2 * ML).sum(axis=-1))
    den = np.sqrt((ref ** 2 * ML).sum(axis=-1))
    el = np.abs(u - ref).max(axis=-1) / np.abs(ref).max(axis=-1)
    return float(max(np.max(num / den), np.max(el)))


def _elem(u, ref):
    return float(np.abs(u - ref).max() / np.abs(ref).max())


def _ragged_graph():
    g = preferential_attachment(12, 2, lengths=(0.05, 1.7), seed=11)
    edges = np.vstack([g.edges, [[0, 1], [5, 5], [3, 12]]])
    lengths = np.concatenate([g.lengths, [0.013, 0.9, 0.31]])
    return 13, edges, lengths


def _b_signs(m, kappa, cI, cL):
    he = np.asarray(m.h_e)
    b = (cI[:, None] + cL[:, None] * kappa * kappa) * he[None, :] / 6.0 - cL[:, None] / he[None, :]
    return (b > 0).any(), (b < 0).any()


@pytest.mark.parametrize("precond", ["jacobi", "nn"])
def test_consistent_sample_c1(grf, precond):
    cfg = config_c1()
    g = cfg["graph"]
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"], mass="consistent")
    S = 8
    u, st = G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"], precond=precond)
    assert st["sweep_block"] > 0 and st["n_unconverged"] == 0  # the streamed sweeps ran
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    ML = omesh.lumped_mass(m)
    W = onoise.white_noise(ML, cfg["seed"], S)
    ref = osolve.sample(m, cfg["kappa"], cfg["beta"], cfg["quad_step"], W, mass="consistent")
    _, cI, cL = oquad.shifts(cfg["beta"], cfg["quad_step"])
    assert all(_b_signs(m, cfg["kappa"], cI, cL))  # both signs of b occur
    u = u.cpu().numpy()
    err, eel = _rel_ml(u, ref, ML), _elem(u, ref)
    print(f"consistent C1 ({precond}): rel err {err:.2e}, element-wise {eel:.2e}")
    assert err <= TOL and eel <= TOL
    lumped = osolve.sample(m, cfg["kappa"], cfg["beta"], cfg["quad_step"], W)
    assert _rel_ml(u, lumped, ML) > 1e-4  # not the lumped system


@pytest.mark.parametrize("sweep_block", [0, 8, 64])
def test_consistent_sample_ragged(grf, sweep_block):
    V, E, L = _ragged_graph()
    h, rule, kappa, beta, k = 0.07, "round", 3.0, 0.7, 0.45
    G = grf.Graph(V, E, L, h, rule, mass="consistent")
    S = 70
    u, st = G.sample(kappa, beta, k, S, 3, sweep_block=sweep_block)
    m = omesh.build_mesh(V, E, L, h, rule)
    ML = omesh.lumped_mass(m)
    W = onoise.white_noise(ML, 3, S)
    ref = osolve.sample(m, kappa, beta, k, W, mass="consistent")
    u = u.cpu().numpy()
    err, eel = _rel_ml(u, ref, ML), _elem(u, ref)
    print(f"consistent ragged (sweep_block {sweep_block} -> {st['sweep_block']}): rel err {err:.2e}, "
          f"element-wise {eel:.2e}")
    assert err <= TOL and eel <= TOL


@pytest.mark.parametrize("kappa,cI,cL", [(3.0, 1.0, 1.0), (3.0, 1e-9, 1e9), (3.0, 1e9, 1e-9), (20.0, 5e3, 1e-3),
                                         (0.0, 96.0, 1.0)])
def test_consistent_solve_shifted(grf, kappa, cI, cL):
    """Single shifts with b < 0, b > 0 and, for (0, 96, 1) on edges of length 1
    meshed with h = 1/4, b = 96/24 - 1/(1/4) = 0 exactly on the unit edges."""
    g = lattice(3, 3, lengths=None, seed=0)
    Lg = np.concatenate([np.ones(g.edges.shape[0] - 3), [0.6, 1.35, 0.21]])
    G = grf.Graph(g.n_vertices, g.edges, Lg, 0.25, "ceil", mass="consistent")
    m = omesh.build_mesh(g.n_vertices, g.edges, Lg, 0.25, "ceil")
    rng = np.random.default_rng(7)
    B = rng.standard_normal((5, m.n_dof))
    import torch

    x, _ = G.solve_shifted(kappa, cI, cL, torch.from_numpy(B).cuda())
    ref = osolve.solve_shifted(m, kappa, cI, cL, B, mass="consistent")
    ML = omesh.lumped_mass(m)
    x = x.cpu().numpy()
    err, eel = _rel_ml(x, ref, ML), _elem(x, ref)
    print(f"consistent shift kappa={kappa} c_I={cI:g} c_L={cL:g}: rel err {err:.2e}, element-wise {eel:.2e}")
    assert err <= TOL and eel <= TOL


def test_consistent_batched_matches_single(grf):
    specs = [_ragged_graph(), (lambda g: (g.n_vertices, g.edges, g.lengths))(lattice(4, 3, lengths=(0.3, 1.2),
                                                                                        seed=2))]
    h, rule, beta, k = 0.07, "round", 0.7, 0.45
    Gs = [grf.Graph(V, E, L, h, rule, mass="consistent") for V, E, L in specs]
    kappas = [3.0, 8.0]
    outs, _ = grf.sample_batched(Gs, kappas, beta, k, 5, 2)
    for (V, E, L), G, kap, u in zip(specs, Gs, kappas, outs):
        m = omesh.build_mesh(V, E, L, h, rule)
        ML = omesh.lumped_mass(m)
        W = onoise.white_noise(ML, 2, 5)
        ref = osolve.sample(m, kap, beta, k, W, mass="consistent")
        assert _rel_ml(u.cpu().numpy(), ref, ML) <= TOL and _elem(u.cpu().numpy(), ref) <= TOL
    lumped = grf.Graph(*specs[0], h, rule)
    with pytest.raises(grf.GrfError) as ei:  # a batch shares the mass matrix
        grf.sample_batched([Gs[0], lumped], kappas, beta, k, 5, 2)
    assert ei.value.code == grf.GRF_EINVAL


def test_consistent_mixed_unsupported(grf):
    g = interval(1.0)
    G = grf.Graph(2, g.edges, g.lengths, 0.1, "ceil", mass="consistent")
    with pytest.raises(grf.GrfError) as ei:
        G.sample(2.0, 0.75, 0.5, 2, 0, precision="mixed")
    assert ei.value.code == grf.GRF_EUNSUP


# ---- consistent-mass noise (GRF_NOISE_CONSISTENT; eq. wh_def with the element factors) ----


@pytest.mark.parametrize("S,offset", [(20, 0), (70, 5), (1, 3)])
def test_consistent_noise_bit_identical(grf, S, offset):
    """Every DOF (interior, vertex, self-loop and multi-edge ends) and every sample
    lane (16-, 32- and 64-lane groups, a ragged second block) bit for bit."""
    V, E, L = _ragged_graph()
    h, rule = 0.07, "round"
    G = grf.Graph(V, E, L, h, rule, noise="consistent")
    w = G.noise(S, 9, sample_offset=offset).cpu().numpy()
    m = omesh.build_mesh(V, E, L, h, rule)
    ref = onoise.consistent_white_noise(m, 9, S, sample_offset=offset)
    assert np.array_equal(w.view(np.uint64), ref.view(np.uint64))
    lumped = onoise.white_noise(omesh.lumped_mass(m), 9, S, sample_offset=offset)
    assert not np.allclose(w, lumped)


@pytest.mark.parametrize("mass", ["lumped", "consistent"])
def test_consistent_noise_sample(grf, mass):
    """The full consistent arm (consistent system and noise) and consistent noise on
    the lumped system (blocked matrix-core sweeps) against the oracle."""
    cfg = config_c1()
    g = cfg["graph"]
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"], mass=mass, noise="consistent")
    S = 8
    u, st = G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"])
    assert st["n_unconverged"] == 0
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    ML = omesh.lumped_mass(m)
    W = onoise.consistent_white_noise(m, cfg["seed"], S)
    ref = osolve.sample(m, cfg["kappa"], cfg["beta"], cfg["quad_step"], W, mass=mass)
    u = u.cpu().numpy()
    err, eel = _rel_ml(u, ref, ML), _elem(u, ref)
    print(f"consistent noise, {mass} system: rel err {err:.2e}, element-wise {eel:.2e}")
    assert err <= TOL and eel <= TOL


def test_consistent_noise_batched_matches_single(grf):
    specs = [_ragged_graph(), (lambda g: (g.n_vertices, g.edges, g.lengths))(lattice(4, 3, lengths=(0.3, 1.2),
                                                                                        seed=2))]
    h, rule, beta, k = 0.07, "round", 0.7, 0.45
    Gs = [grf.Graph(V, E, L, h, rule, noise="consistent") for V, E, L in specs]
    for G, (V, E, L) in zip(Gs, specs):  # the batch draws each graph's own stream
        m = omesh.build_mesh(V, E, L, h, rule)
        assert np.array_equal(G.noise(5, 2).cpu().numpy(), onoise.consistent_white_noise(m, 2, 5))
    kappas = [3.0, 8.0]
    outs, _ = grf.sample_batched(Gs, kappas, beta, k, 5, 2)
    for G, kap, u in zip(Gs, kappas, outs):
        single, _ = G.sample(kap, beta, k, 5, 2)
        assert _elem(u.cpu().numpy(), single.cpu().numpy()) <= 1e-12
