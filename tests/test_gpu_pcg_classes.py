"""Vertex PCG size classes: a batch whose graphs sit on both sides of every
class capacity (64, 256, 1024, 4096, 10176 and 20352 vertices; the last
graph is beyond every on-chip class and takes the global-memory kernel), so
every on-chip variant and the fallback solve systems of the same call.

Bars: each graph's batched sample equals the FP64 oracle to 1e-10 relative
in the lumped-mass norm, with the Jacobi, the Neumann-Neumann (on chip up to
10176 vertices, in the global-memory kernel beyond) and the learned
preconditioner (an untrained network: its Jacobi fallback and the true
residual still decide convergence), the last with every on-chip variant
forced in turn (operator, initial guess only, Jacobi) and as the autotuner
picks them; every system converges.
"""

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import noise as onoise
from oracle import solve as osolve
from workloads import preferential_attachment
from workloads.learned_init import init_params

pytestmark = pytest.mark.gpu
H, RULE = 0.5, "round"          # lengths U[0.5, 1.5]: 0 to 2 interior DOFs per edge
BETA, K, S, SEED = 0.7, 1.0, 3, 13
SIZES = [64, 65, 256, 257, 1024, 1025, 4096, 4097, 10176, 10177, 20352, 20353]


def _rel_ml(u, ref, ML):
    """Worst sample's relative error, the larger of the lumped-mass norm
    ||u - ref||_{M_L} / ||ref||_{M_L} and the element-wise max |u - ref| / max |ref|
    (a local error that the norm would dilute fails the second)."""
    num = np.sqrt(((u - ref) ** 2 * ML).sum(axis=-1))
    den = np.sqrt((ref ** 2 * ML).sum(axis=-1))
    el = np.abs(u - ref).max(axis=-1) / np.abs(ref).max(axis=-1)
    return float(max(np.max(num / den), np.max(el)))


@pytest.fixture(scope="module")
def batch(grf):
    trees = [preferential_attachment(n, 1, lengths=(0.5, 1.5), seed=100 + i) for i, n in enumerate(SIZES)]
    assert [t.n_vertices for t in trees] == SIZES
    Gs = [grf.Graph(t.n_vertices, t.edges, t.lengths, H, RULE) for t in trees]
    kappas = np.linspace(4.0, 12.0, len(Gs))
    refs = []
    for t, kap in zip(trees, kappas):
        m = omesh.build_mesh(t.n_vertices, t.edges, t.lengths, H, RULE)
        ML = omesh.lumped_mass(m)
        W = onoise.white_noise(ML, SEED, S)
        refs.append((ML, osolve.sample(m, float(kap), BETA, K, W)))
    return Gs, kappas, refs


CASES = [("jacobi", None), ("nn", None), ("learned", None), ("learned", ["op"] * 5 + ["guess"]),
         ("learned", ["guess"] * 6), ("learned", ["jacobi"] * 6)]


@pytest.mark.parametrize("precond,modes", CASES, ids=["jacobi", "nn", "learned-auto", "learned-op",
                                                       "learned-guess", "learned-jacobi"])
def test_every_class_matches_oracle(grf, batch, precond, modes):
    Gs, kappas, refs = batch
    net, kw, st_j = None, {}, None
    if precond != "jacobi":
        # the same handles were just run with Jacobi: this call must not replay
        # that captured graph (its iteration total differs)
        _, st_j = grf.sample_batched(Gs, kappas, BETA, K, S, SEED)
    if precond == "learned":
        net = grf.Learned(init_params(7, head_scale=0.5))
        kw = dict(learned=net, pcg_class_modes=modes)
    elif precond == "nn":
        kw = dict(precond="nn")
    try:
        outs, st = grf.sample_batched(Gs, kappas, BETA, K, S, SEED, **kw)
    finally:
        if net is not None:
            net.close()
    assert st["n_unconverged"] == 0
    if precond == "learned":
        used = grf.class_modes(st["pcg_class_modes"])
        print(f"PCG variants per size class: {used}", flush=True)
        if modes is not None:
            assert used == modes
        else:
            assert used[5] != "op"
    if st_j is not None:
        print(f"{precond}: {st['total_iterations']} iterations, Jacobi {st_j['total_iterations']}", flush=True)
        assert st["total_iterations"] != st_j["total_iterations"]
    for n, u, (ML, ref) in zip(SIZES, outs, refs):
        err = _rel_ml(u.cpu().numpy(), ref, ML)
        print(f"{precond} V={n}: rel err {err:.2e}", flush=True)
        assert err <= 1e-10, (n, err)


def test_class_modes_are_validated(grf):
    g = preferential_attachment(40, 1, lengths=(0.5, 1.5), seed=3)
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, H, RULE)
    net = grf.Learned(init_params(7, head_scale=0.5))
    try:
        with pytest.raises(grf.GrfError, match="not available in size class 5"):
            G.sample(4.0, BETA, K, 2, SEED, learned=net, pcg_class_modes=["op"] * 6)
        with pytest.raises(grf.GrfError, match="for the learned preconditioner"):
            G.sample(4.0, BETA, K, 2, SEED, pcg_class_modes=["jacobi"] * 6)
        u, st = G.sample(4.0, BETA, K, 2, SEED, learned=net, pcg_class_modes=["guess"] * 6)
        assert st["n_unconverged"] == 0
    finally:
        net.close()
        G.close()


def test_unused_network_is_skipped(grf):
    """With Jacobi in every size class and no graph beyond them, the learned call runs
    no network kernel and returns the Jacobi batch bit for bit."""
    import torch

    trees = [preferential_attachment(n, 1, lengths=(0.5, 1.5), seed=200 + n) for n in (50, 300, 2000)]
    Gs = [grf.Graph(t.n_vertices, t.edges, t.lengths, H, RULE) for t in trees]
    kap = [3.0, 6.0, 9.0]
    net = grf.Learned(init_params(7, head_scale=0.5))
    try:
        # a fixed shift block: both calls take the same plan (the autotuner would time
        # each (precision, preconditioner) separately and may pick different sweeps)
        uj, sj = grf.sample_batched(Gs, kap, BETA, K, S, SEED, shift_block=16)
        ul, sl = grf.sample_batched(Gs, kap, BETA, K, S, SEED, learned=net, pcg_class_modes=["jacobi"] * 6,
                                    shift_block=16)
        assert sl["total_iterations"] == sj["total_iterations"]
        for a, b in zip(uj, ul):
            assert torch.equal(a, b)
        # per-kernel timing (single-graph calls): no network launch when no class reads it
        _, s1 = Gs[2].sample(kap[2], BETA, K, S, SEED, learned=net, pcg_class_modes=["jacobi"] * 6, timing=True)
        assert s1["kernel_launches"]["learned"] == 0
        _, s2 = Gs[2].sample(kap[2], BETA, K, S, SEED, learned=net, timing=True)
        assert s2["kernel_launches"]["learned"] > 0
    finally:
        net.close()
        for G in Gs:
            G.close()
