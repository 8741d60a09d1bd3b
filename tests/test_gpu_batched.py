"""Batched sampling over many uneven graphs (one union mesh; noise, every shift
pass and all samples captured once in a HIP graph and replayed; the sweep
form and shift block picked by the autotuner) through the C ABI.

Bars: each graph's batched result equals grf_sample of that graph alone to
1e-12 relative (the same arithmetic, up to the vertex-PCG variant the batch
selects) and the FP64 oracle to 1e-10, in the lumped-mass norm; repeated
calls (graph replays) are bitwise equal; mixed precision within 1e-6.
"""

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import noise as onoise
from oracle import solve as osolve
from workloads import interval, lattice, preferential_attachment

pytestmark = pytest.mark.gpu
H, RULE = 1.0 / 40, "round"
BETA, K, S, SEED = 0.7, 0.45, 70, 5


def _rel_ml(u, ref, ML):
    """Worst sample's relative error, the larger of the lumped-mass norm
    ||u - ref||_{M_L} / ||ref||_{M_L} and the element-wise max |u - ref| / max |ref|
    (a local error that the norm would dilute fails the second)."""
    num = np.sqrt(((u - ref) ** 2 * ML).sum(axis=-1))
    den = np.sqrt((ref ** 2 * ML).sum(axis=-1))
    el = np.abs(u - ref).max(axis=-1) / np.abs(ref).max(axis=-1)
    return float(max(np.max(num / den), np.max(el)))


def _graphs(with_hub: bool):
    gs = [lattice(3, 4, lengths=(0.1, 2.0), seed=1), preferential_attachment(30, 1, lengths=(0.1, 2.0), seed=2),
          interval(1.3), lattice(5, 5, lengths=(0.1, 2.0), seed=3)]
    rag = preferential_attachment(12, 2, lengths=(0.05, 1.7), seed=11)
    ragged = (13, np.vstack([rag.edges, [[0, 1], [5, 5], [3, 12]]]),
              np.concatenate([rag.lengths, [0.013, 0.9, 0.31]]))
    out = [(g.n_vertices, g.edges, g.lengths) for g in gs] + [ragged]
    if with_hub:  # a star-like tree: one vertex of degree 20 (the batch then uses the global-memory PCG)
        n = 21
        out.append((n, np.array([[0, i] for i in range(1, n)]), np.linspace(0.2, 1.9, n - 1)))
    return out


@pytest.mark.parametrize("with_hub", [False, True])
def test_batched_matches_single_and_oracle(grf, with_hub):
    specs = _graphs(with_hub)
    Gs = [grf.Graph(V, E, L, H, RULE) for V, E, L in specs]
    kappas = np.linspace(2.0, 20.0, len(Gs))
    outs, st = grf.sample_batched(Gs, kappas, BETA, K, S, SEED)
    assert st["n_unconverged"] == 0 and st["n_systems"] == len(Gs) * st["n_shifts"] * S
    for (V, E, L), G, kap, u in zip(specs, Gs, kappas, outs):
        m = omesh.build_mesh(V, E, L, H, RULE)
        ML = omesh.lumped_mass(m)
        single, _ = G.sample(float(kap), BETA, K, S, SEED)
        assert _rel_ml(u.cpu().numpy(), single.cpu().numpy(), ML) <= 1e-12
        W = onoise.white_noise(ML, SEED, S)
        ref = osolve.sample(m, float(kap), BETA, K, W)
        assert _rel_ml(u.cpu().numpy(), ref, ML) <= 1e-10


def test_batched_replay_and_new_parameters(grf):
    specs = _graphs(False)
    Gs = [grf.Graph(V, E, L, H, RULE) for V, E, L in specs]
    kappas = np.linspace(3.0, 9.0, len(Gs))
    a, _ = grf.sample_batched(Gs, kappas, BETA, K, S, SEED)
    b, _ = grf.sample_batched(Gs, kappas, BETA, K, S, SEED)  # replay of the captured graph
    for x, y in zip(a, b):
        assert (x == y).all()
    c, _ = grf.sample_batched(Gs, kappas[::-1].copy(), BETA, K, 9, SEED + 1)  # new parameters: recaptured
    for (V, E, L), G, kap, u in zip(specs, Gs, kappas[::-1], c):
        single, _ = G.sample(float(kap), BETA, K, 9, SEED + 1)
        ML = omesh.lumped_mass(omesh.build_mesh(V, E, L, H, RULE))
        assert _rel_ml(u.cpu().numpy(), single.cpu().numpy(), ML) <= 1e-12


@pytest.mark.parametrize("kw", [dict(sweep_block=16), dict(shift_block=16), dict(precision="mixed")])
def test_batched_fixed_options(grf, kw):
    specs = _graphs(True)
    Gs = [grf.Graph(V, E, L, H, RULE) for V, E, L in specs]
    kappas = np.linspace(2.0, 12.0, len(Gs))
    outs, st = grf.sample_batched(Gs, kappas, BETA, K, S, SEED, **kw)
    tol = 1e-6 if kw.get("precision") == "mixed" else 1e-12
    for (V, E, L), G, kap, u in zip(specs, Gs, kappas, outs):
        single, _ = G.sample(float(kap), BETA, K, S, SEED)
        ML = omesh.lumped_mass(omesh.build_mesh(V, E, L, H, RULE))
        assert _rel_ml(u.cpu().numpy(), single.cpu().numpy(), ML) <= tol


def test_batched_invalid_and_destroyed(grf):
    specs = _graphs(False)
    Gs = [grf.Graph(V, E, L, H, RULE) for V, E, L in specs]
    other = grf.Graph(*specs[0], H / 2, RULE)
    with pytest.raises(grf.GrfError) as ei:
        grf.sample_batched([Gs[0], other], [2.0, 3.0], BETA, K, 4, 0)
    assert ei.value.code == grf.GRF_EINVAL
    with pytest.raises(grf.GrfError) as ei:
        grf.sample_batched(Gs[:2], [2.0, -1.0], BETA, K, 4, 0)
    assert ei.value.code == grf.GRF_EINVAL
    grf.sample_batched(Gs, np.full(len(Gs), 4.0), BETA, K, 4, 0)
    Gs[1].close()  # drops the cached batch that holds it
    rest = [Gs[0]] + Gs[2:]
    outs, _ = grf.sample_batched(rest, np.full(len(rest), 4.0), BETA, K, 4, 0)
    single, _ = Gs[0].sample(4.0, BETA, K, 4, 0)
    assert np.allclose(outs[0].cpu().numpy(), single.cpu().numpy(), rtol=0, atol=1e-12 * float(single.abs().max()))


def test_batched_timing_run_matches_replay(grf):
    """opts.timing runs the batch's launches uncaptured, each timed: the same
    result as the captured replay, bit for bit, with every step's time, one PCG
    launch per non-empty size class and shift block, and iteration counts per
    class that add up to the total."""
    specs = _graphs(True)
    Gs = [grf.Graph(V, E, L, H, RULE) for V, E, L in specs]
    kappas = np.linspace(2.0, 12.0, len(Gs))
    a, st0 = grf.sample_batched(Gs, kappas, BETA, K, S, SEED)
    b, st = grf.sample_batched(Gs, kappas, BETA, K, S, SEED, timing=True)
    for x, y in zip(a, b):
        assert (x == y).all()
    assert st["total_iterations"] == st0["total_iterations"]
    ms = st["kernel_ms"]
    for k in ("noise", "coeff", "condense", "pcg", "scatter", "layout"):
        assert ms[k] > 0.0, k
    nblocks = st["kernel_launches"]["condense"]
    assert nblocks >= 1
    if st["sweep_block"] == 0:  # blocked sweeps: one operand-table launch per shift block
        assert ms["table"] > 0.0 and st["kernel_launches"]["table"] == nblocks
    launched = [c for c in range(7) if st["pcg_class_launches"][c] > 0]
    assert launched and all(st["pcg_class_launches"][c] == nblocks for c in launched)
    assert sum(st["pcg_class_ms"]) <= ms["pcg"] * (1 + 1e-6)
    its_v = sum(st["pcg_class_vertex_its"])
    assert its_v > 0 and all(st["pcg_class_vertex_its"][c] == 0 for c in range(7) if c not in launched)
