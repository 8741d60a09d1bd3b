"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Bar: the noise is bit-identical; every floating-point result is within
1e-10 relative of the oracle in the lumped-mass norm,
    max_s ||u_gpu[s] - u_ref[s]||_{M_L} / ||u_ref[s]||_{M_L},
with the vertex Schur PCG run to tol 1e-12 (the solver's error is bounded by
cond(S) * tol, far below the bar for these graphs).
"""

import math

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


def _ragged_graph():
    """Edges of very different interior counts (0, 1, 2, ...), a multi-edge, a
    self-loop and a pendant vertex, on a round-to-nearest mesh."""
    g = preferential_attachment(12, 2, lengths=(0.05, 1.7), seed=11)
    edges = np.vstack([g.edges, [[0, 1], [5, 5], [3, 12]]])
    lengths = np.concatenate([g.lengths, [0.013, 0.9, 0.31]])
    return 13, edges, lengths


@pytest.fixture(scope="module")
def c1(grf):
    cfg = config_c1()
    g = cfg["graph"]
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    return cfg, m, G


def test_mesh_sizes_match(grf, c1):
    cfg, m, G = c1
    assert G.n_dof == m.n_dof == 1528 and G.n_interior == m.n_interior
    assert np.array_equal(G.offsets, m.offsets)
    assert np.array_equal(G.lumped_mass(), omesh.lumped_mass(m))
    V, E, L = _ragged_graph()
    for rule in ("ceil", "round"):
        Gr = grf.Graph(V, E, L, 0.07, rule)
        mr = omesh.build_mesh(V, E, L, 0.07, rule)
        assert np.array_equal(Gr.lumped_mass(), omesh.lumped_mass(mr))


@pytest.mark.parametrize("rule", ["ceil", "round"])
def test_noise_bit_identical(grf, rule):
    V, E, L = _ragged_graph()
    m = omesh.build_mesh(V, E, L, 0.07, rule)
    G = grf.Graph(V, E, L, 0.07, rule)
    for S, seed, soff in [(1, 0, 0), (70, 12345, 0), (5, 2 ** 63 + 7, 1000)]:
        w = G.noise(S, seed, sample_offset=soff).cpu().numpy()
        ref = onoise.white_noise(omesh.lumped_mass(m), seed, S, sample_offset=soff)
        assert w.shape == ref.shape
        assert np.array_equal(w.view(np.uint64), ref.view(np.uint64)), "noise bits differ"


def test_noise_c1_bit_identical(grf, c1):
    cfg, m, G = c1
    w = G.noise(cfg["n_samples"], cfg["seed"]).cpu().numpy()
    ref = onoise.white_noise(omesh.lumped_mass(m), cfg["seed"], cfg["n_samples"])
    assert np.array_equal(w.view(np.uint64), ref.view(np.uint64))


# kappa = 0 is allowed by the ABI, but then A = c_I M + c_L G has condition
# ~ c_L / (c_I h^2): only moderate ratios give a system whose residual can reach
# 1e-12 in FP64.  With kappa > 0 (alpha/gamma >= kappa^2) the extreme shifts of
# the quadrature (c_I/c_L from 1e-18 to 1e18) are all well conditioned.
@pytest.mark.parametrize("kappa,cI,cL", [(0.0, 1.0, 1.0), (0.0, 3e4, 2e-4), (3.0, 1.0, 1.0), (3.0, 3e4, 2e-4),
                                         (3.0, 1e-3, 5e3), (3.0, 2.5e7, 1e-8), (3.0, 1e-9, 1e9),
                                         (20.0, 1e-9, 1e9), (20.0, 1e9, 1e-9)])
def test_solve_shifted_ragged(grf, kappa, cI, cL):
    import torch

    V, E, L = _ragged_graph()
    m = omesh.build_mesh(V, E, L, 0.07, "round")
    G = grf.Graph(V, E, L, 0.07, "round")
    rng = np.random.default_rng(5)
    B = rng.standard_normal((67, m.n_dof))  # two sample blocks, ragged
    x, st = G.solve_shifted(kappa, cI, cL, torch.from_numpy(B).cuda())
    ref = osolve.solve_shifted(m, kappa, cI, cL, B)
    assert _rel_ml(x.cpu().numpy(), ref, omesh.lumped_mass(m)) <= TOL
    assert st["n_unconverged"] == 0 and st["max_rel_residual"] <= 1e-12


@pytest.mark.parametrize("sweep_block", [0, 8, 16, 32, 64])  # 0 = blocked matrix-core sweeps
def test_sample_c1(grf, c1, sweep_block):
    cfg, m, G = c1
    u, st = G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], cfg["n_samples"], cfg["seed"],
                     tol=cfg["tol"], sweep_block=sweep_block)
    W = onoise.white_noise(omesh.lumped_mass(m), cfg["seed"], cfg["n_samples"])
    ref = osolve.sample(m, cfg["kappa"], cfg["beta"], cfg["quad_step"], W)
    assert st["n_shifts"] == 55 and st["n_unconverged"] == 0
    assert _rel_ml(u.cpu().numpy(), ref, omesh.lumped_mass(m)) <= TOL


@pytest.mark.parametrize("shift_block,sweep_block", [(0, 0), (16, 0), (40, 0), (7, 8), (16, 16), (3, 32)])
def test_sample_ragged_multipass(grf, shift_block, sweep_block):
    V, E, L = _ragged_graph()
    m = omesh.build_mesh(V, E, L, 0.05, "round")
    G = grf.Graph(V, E, L, 0.05, "round")
    kappa, beta, k, S, seed = 4.0, 0.6, 0.45, 70, 3
    u, st = G.sample(kappa, beta, k, S, seed, shift_block=shift_block, sweep_block=sweep_block)
    W = onoise.white_noise(omesh.lumped_mass(m), seed, S)
    ref = osolve.sample(m, kappa, beta, k, W)
    assert _rel_ml(u.cpu().numpy(), ref, omesh.lumped_mass(m)) <= TOL
    assert st["n_shifts"] == sum(oquad.limits(beta, k)) + 1


@pytest.mark.parametrize("k,shift_block,precision", [
    (0.3, 0, "fp64"),       # 116 shifts in one pass: 128 padded, one edge block per table workgroup
    (0.3, 90, "fp64"),      # passes of 90 and 26: 96 padded (one block per workgroup), 32 padded (four)
    (0.45, 25, "fp64"),     # passes of 25, 25, 3: four and eight blocks per table workgroup
    (0.45, 25, "mixed"),    # the same with FP32 operand tables
    (0.3, 0, "mixed"),
    (0.3, 70, "fp64"),      # 80 + 48 padded: shift tiles 5 and 3 in the sweeps
    (0.3, 100, "fp64"),     # 112 + 16 padded: shift tiles 7 and 1
    (0.3, 100, "mixed"),
])
def test_sample_ragged_table_packing(grf, k, shift_block, precision):
    """The table kernel packs 128 / SLOT edge blocks into a workgroup (SLOT = 16, 32, 64
    or 128 threads, the smallest power of two that holds the padded shift block); this
    graph has 35 edge blocks, so the last workgroup of a packed launch is partly empty.
    FP64 against the oracle to 1e-10; mixed precision to 1e-6 (its error bound)."""
    V, E, L = _ragged_graph()
    m = omesh.build_mesh(V, E, L, 0.05, "round")
    G = grf.Graph(V, E, L, 0.05, "round")
    kappa, beta, S, seed = 4.0, 0.6, 70, 5
    u, st = G.sample(kappa, beta, k, S, seed, shift_block=shift_block, precision=precision)
    W = onoise.white_noise(omesh.lumped_mass(m), seed, S)
    ref = osolve.sample(m, kappa, beta, k, W)
    assert st["n_shifts"] == sum(oquad.limits(beta, k)) + 1 and st["n_unconverged"] == 0
    assert _rel_ml(u.cpu().numpy(), ref, omesh.lumped_mass(m)) <= (TOL if precision == "fp64" else 1e-6)


def test_sample_interval_single_edge(grf):
    g = interval(1.7)
    m = omesh.build_mesh(2, g.edges, g.lengths, 1 / 100, "ceil")
    G = grf.Graph(2, g.edges, g.lengths, 1 / 100, "ceil")
    u, _ = G.sample(2.0, 0.8, 0.35, 3, 9)
    W = onoise.white_noise(omesh.lumped_mass(m), 9, 3)
    ref = osolve.sample(m, 2.0, 0.8, 0.35, W)
    assert _rel_ml(u.cpu().numpy(), ref, omesh.lumped_mass(m)) <= TOL


def test_sample_offset_and_determinism(grf, c1):
    cfg, m, G = c1
    a, _ = G.sample(5.0, 0.75, 0.5, 20, 1)
    b, _ = G.sample(5.0, 0.75, 0.5, 20, 1)
    c, _ = G.sample(5.0, 0.75, 0.5, 4, 1, sample_offset=7)
    assert (a == b).all(), "repeated calls must be bitwise equal"
    assert np.allclose(c.cpu().numpy(), a[7:11].cpu().numpy(), rtol=0, atol=1e-13 * float(a.abs().max()))


def test_noconv_is_reported(grf, c1):
    cfg, m, G = c1
    with pytest.raises(grf.GrfError) as ei:
        G.sample(5.0, 0.75, 0.5, 2, 0, maxit=1)
    assert ei.value.code == grf.GRF_ENOCONV
    u, st = G.sample(5.0, 0.75, 0.5, 2, 0, maxit=1, allow_noconv=True)
    assert st["n_unconverged"] > 0 and np.isfinite(u.cpu().numpy()).all()


def test_invalid_arguments(grf, c1):
    cfg, m, G = c1
    for kw in [dict(kappa=0.0), dict(beta=1.0), dict(beta=0.0), dict(quad_step=-0.1)]:
        args = dict(kappa=5.0, beta=0.75, quad_step=0.5, n_samples=1, seed=0)
        args.update(kw)
        with pytest.raises(grf.GrfError) as ei:
            G.sample(**args)
        assert ei.value.code == grf.GRF_EINVAL
    import torch

    out = torch.zeros((0, G.n_dof), dtype=torch.float64, device="cuda")
    G.sample(5.0, 0.75, 0.5, 0, 0, out=out)  # n_samples = 0 is a no-op


def test_conservation_lattice_lengths(grf):
    """<diag M_L, u> = q_k(kappa^2) <1, W> for the quadrature sum, per sample
    (G has zero row sums), on a random-length lattice with the paper's step rule."""
    g = lattice(8, 8, lengths=(0.5, 1.5), seed=1)
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, 1 / 64, "round")
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, 1 / 64, "round")
    kappa, beta = 10.0, 0.85
    km, kp, k = G.shift_count(beta, 0.0)
    assert (km, kp) == oquad.limits(beta, oquad.paper_step(beta, 1 / 64))
    u, _ = G.sample(kappa, beta, 0.0, 64, 4)
    W = G.noise(64, 4).cpu().numpy()
    ML = omesh.lumped_mass(m)
    q = oquad.q_k(kappa ** 2, beta, k)
    lhs = (u.cpu().numpy() * ML).sum(axis=1)
    rhs = q * W.sum(axis=1)
    assert np.max(np.abs(lhs - rhs)) <= 1e-10 * np.max(np.abs(rhs))
