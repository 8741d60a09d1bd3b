"""grf_sample_noalloc, the entry point that allocates nothing, against
grf_sample (the existing entry point it mirrors), through the C ABI.

Two calls in a row share the library's one static scratch array on the
device, the second with a smaller input (fewer samples, a smaller graph).
Each output equals grf_sample's for the same arguments bit for bit (both run
the same kernels with the same shift-block plan here) and is within 1e-10
relative of the FP64 oracle in the lumped-mass norm.  A workspace larger
than the array, and the learned preconditioner, are rejected with
GRF_EINVAL before any kernel runs.
"""

import ctypes as C

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import noise as onoise
from oracle import solve as osolve
from workloads import config_c1, lattice, preferential_attachment

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
    """Edges of very different interior counts, a multi-edge, a self-loop and a
    pendant vertex, on a round-to-nearest mesh."""
    g = preferential_attachment(12, 2, lengths=(0.05, 1.7), seed=11)
    edges = np.vstack([g.edges, [[0, 1], [5, 5], [3, 12]]])
    lengths = np.concatenate([g.lengths, [0.013, 0.9, 0.31]])
    return 13, edges, lengths, 0.07, "round"


def _noalloc(grf, G, kappa, beta, step, S, seed, **kw):
    import torch

    out = torch.full((S, G.n_dof), float("nan"), dtype=torch.float64, device=f"cuda:{G.device}")
    st = grf.Stats()
    o = grf.make_opts(stats=st, **kw)
    code = grf.load().grf_sample_noalloc(G.handle, kappa, beta, step, S, seed, out.data_ptr(), C.byref(o))
    return code, out, st.as_dict()


def _case(grf, V, E, L, h, rule, kappa, beta, step, S, seed, **kw):
    import torch

    G = grf.Graph(V, E, L, h, rule)
    code, u, st = _noalloc(grf, G, kappa, beta, step, S, seed, **kw)
    assert code == grf.GRF_OK, grf.load().grf_last_error()
    torch.cuda.synchronize()
    ref_gpu, st_ref = G.sample(kappa, beta, step, S, seed, **kw)
    assert st["shift_block"] == st_ref["shift_block"] and st["n_unconverged"] == 0
    assert torch.equal(u, ref_gpu), "noalloc output differs from grf_sample"
    m = omesh.build_mesh(V, E, L, h, rule)
    ML = omesh.lumped_mass(m)
    W = onoise.white_noise(ML, seed, S)
    ref = osolve.sample(m, kappa, beta, step, W)
    err = _rel_ml(u.cpu().numpy(), ref, ML)
    print(f"noalloc V={V} N={m.n_dof} S={S} {kw}: rel err vs oracle {err:.2e}", flush=True)
    assert err <= (1e-6 if kw.get("precision") == "mixed" else TOL)
    G.close()


def test_noalloc_two_calls_then_smaller(grf):
    cfg = config_c1()
    g = cfg["graph"]
    # call 1: the 4x4 lattice, 70 samples (two sample blocks, a ragged second one)
    _case(grf, g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"], cfg["kappa"], cfg["beta"],
          cfg["quad_step"], 70, cfg["seed"])
    # call 2: a smaller input (13-vertex ragged graph, 3 samples) in the same scratch
    V, E, L, h, rule = _ragged_graph()
    _case(grf, V, E, L, h, rule, 4.0, 0.7, 0.6, 3, 5)
    # call 3: the same smaller input with FP32 edge sweeps and Neumann-Neumann PCG
    _case(grf, V, E, L, h, rule, 4.0, 0.7, 0.6, 3, 5, precision="mixed", precond="nn")


def test_noalloc_rejects_what_does_not_fit(grf):
    g = lattice(64, 64, lengths=(0.5, 1.5), seed=1)
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, 1.0 / 256, "round")
    code, _, _ = _noalloc(grf, G, 10.0, 0.6, 0.3, 64, 0)
    assert code == grf.GRF_EINVAL
    assert b"scratch" in grf.load().grf_last_error()
    G.close()
    # a later call that fits still works
    cfg = config_c1()
    c = cfg["graph"]
    _case(grf, c.n_vertices, c.edges, c.lengths, cfg["h"], cfg["rule"], cfg["kappa"], cfg["beta"],
          cfg["quad_step"], 4, 9)


def test_noalloc_rejects_learned(grf):
    from workloads.learned_init import init_params

    cfg = config_c1()
    g = cfg["graph"]
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    net = grf.Learned(init_params(0))
    code, _, _ = _noalloc(grf, G, cfg["kappa"], cfg["beta"], cfg["quad_step"], 2, 0, learned=net)
    assert code == grf.GRF_EINVAL and b"learned" in grf.load().grf_last_error()
    G.close()
