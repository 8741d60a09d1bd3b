"""Learned vertex preconditioner through the C ABI.

* the loss and its parameter gradient (GPU: FP32 activations on the FP32
  matrix cores, bfloat16 weights) against the FP64 autograd oracle of the same
  network, loss and bfloat16-rounded weights: loss within 1e-4, gradient
  within 1e-3 relative (norm);
* the network's operators P_hat, Q_hat (grf_learned_operators) against the
  oracle's FP64 forward: FP32 activations (training's forward) within 1e-5,
  bfloat16 activations (the sampler's forward) within 2e-2 of each array's
  largest value;
* PCG with any network (here an untrained, random one) reaches the oracle's
  result to the FP64 bar (1e-10): the preconditioner is SPD by construction and
  the true residual decides convergence;
* after training on the GPU on the method's own Schur solutions of small
  random geometric graphs, a held-out graph needs fewer PCG iterations than
  with Jacobi, for the same result (the gain is printed).
"""

import numpy as np
import pytest

from oracle import learned as ol
from oracle import mesh as omesh
from oracle import noise as onoise
from oracle import solve as osolve
from workloads import config_c1, preferential_attachment, random_geometric
from workloads.learned_init import N_PARAMS, init_params

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


def test_param_count(grf):
    assert grf.Learned.param_count() == N_PARAMS == ol.N_PARAMS


@pytest.mark.parametrize("cI,cL", [(0.7, 1.9), (30.0, 0.02)])
def test_loss_and_gradient_match_oracle(grf, cI, cL):
    import torch

    V, E, L = _ragged()
    h, kappa = 0.05, 4.0
    m = omesh.build_mesh(V, E, L, h, "round")
    G = grf.Graph(V, E, L, h, "round")
    sd, so = ol.edge_schur(m, np.full(len(E), kappa), cI, cL)
    S = ol.schur_matrix(V, E, sd, so)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((3, V))
    Gm = X @ S
    theta = init_params(3, head_scale=0.3)
    net = grf.Learned(theta)
    loss, grad = net.loss_grad(G, kappa, cI, cL, torch.from_numpy(Gm).cuda(), torch.from_numpy(X).cuda())
    f, w, D = ol.features(m, E, L, sd, so, cI, cL, np.full(V, kappa))
    L_ref, g_ref = ol.loss_and_grad(ol.effective_params(theta), f, w, E, V, D, Gm, X)
    assert abs(loss - L_ref) <= 1e-4 * abs(L_ref)
    assert np.linalg.norm(grad - g_ref) <= 1e-3 * np.linalg.norm(g_ref)
    # each parameter group on its own (weights of every layer and head get a gradient)
    o = 0
    for name, shape, _ in ol.LAYOUT:
        n = int(np.prod(shape))
        gr, gg = g_ref[o:o + n], grad[o:o + n]
        assert np.linalg.norm(gg - gr) <= 1e-3 * max(np.linalg.norm(gr), 1e-6 * np.linalg.norm(g_ref)), name
        o += n


def _op_err(got, ref):
    """max |got - ref| / max |ref| (values near zero are judged on the array's scale)."""
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(got.cpu().numpy() - ref).max() / max(np.abs(ref).max(), 1e-300))


# the operators of the network against the oracle's FP64 forward (bfloat16-rounded
# weights): FP32 activations to 1e-5 of each array's largest value (measured
# <= 1.1e-6); bfloat16
# activations (unit roundoff 2^-9 = 2e-3, rounded at every layer output and
# message: at most about 6 roundings on a path through the three layers) to 2e-2
ACT_TOL = {"fp32": 1e-5, "bf16": 2e-2}


@pytest.mark.parametrize("activations", ["fp32", "bf16"])
@pytest.mark.parametrize("which", ["ragged", "tree300"])
def test_operators_match_oracle(grf, activations, which):
    if which == "ragged":
        V, E, L = _ragged()
    else:  # 301 vertices: 19 full 16-row tiles and a ragged one, hubs of high degree
        g = preferential_attachment(301, 1, lengths=(0.05, 1.7), seed=5)
        V, E, L = g.n_vertices, g.edges, g.lengths
    h, kappa = 0.05, 4.0
    m = omesh.build_mesh(V, E, L, h, "round")
    G = grf.Graph(V, E, L, h, "round")
    theta = init_params(3, head_scale=0.3)
    net = grf.Learned(theta)
    worst = 0.0
    for cI, cL in ((0.7, 1.9), (30.0, 0.02), (1e-3, 40.0)):
        pd, pe, qd, qe = net.operators(G, kappa, cI, cL, activations=activations)
        sd, so = ol.edge_schur(m, np.full(len(E), kappa), cI, cL)
        f, w, D = ol.features(m, E, L, sd, so, cI, cL, np.full(V, kappa))
        Ph, Qh, heads = ol.forward(ol.effective_params(theta), f, w, E, V)
        _, _, p_t, p_h, rho, eta = (x.detach().numpy() for x in heads)
        errs = [_op_err(pd, np.diag(Ph.numpy())), _op_err(pe, rho * np.sqrt(p_t * p_h)),
                _op_err(qd, np.diag(Qh.numpy())), _op_err(qe, eta)]
        print(f"{which} {activations} c_I={cI:g} c_L={cL:g}: P diag {errs[0]:.1e}, P edge {errs[1]:.1e}, "
              f"Q diag {errs[2]:.1e}, Q edge {errs[3]:.1e}")
        worst = max(worst, *errs)
    assert worst <= ACT_TOL[activations]


def test_learned_pcg_reaches_oracle(grf):
    import torch

    cfg = config_c1()
    g = cfg["graph"]
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    net = grf.Learned(init_params(7, head_scale=0.5))
    u, st = G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], cfg["n_samples"], cfg["seed"], tol=cfg["tol"],
                     learned=net)
    W = onoise.white_noise(omesh.lumped_mass(m), cfg["seed"], cfg["n_samples"])
    ref = osolve.sample(m, cfg["kappa"], cfg["beta"], cfg["quad_step"], W)
    assert st["n_unconverged"] == 0
    assert _rel_ml(u.cpu().numpy(), ref, omesh.lumped_mass(m)) <= 1e-10
    V, E, L = _ragged()
    m2 = omesh.build_mesh(V, E, L, 0.07, "round")
    G2 = grf.Graph(V, E, L, 0.07, "round")
    B = np.random.default_rng(5).standard_normal((67, m2.n_dof))
    x, st2 = G2.solve_shifted(3.0, 1e-3, 5e3, torch.from_numpy(B).cuda(), learned=net)
    ref2 = osolve.solve_shifted(m2, 3.0, 1e-3, 5e3, B)
    assert _rel_ml(x.cpu().numpy(), ref2, omesh.lumped_mass(m2)) <= 1e-10


def test_training_gains_iterations(grf):
    h, beta, k = 1.0 / 32, 0.75, 0.6
    train = [random_geometric(n, seed=100 + n) for n in (600, 900, 1200)]
    Gs = [grf.Graph(g.n_vertices, g.edges, g.lengths, h, "round") for g in train]
    kappas = [2.0, 6.0, 3.5]
    net = grf.Learned(init_params(0))
    losses = net.train(Gs, kappas, beta, k, n_samples=4, seed=1, n_steps=240, shifts_per_step=8, lr=2e-3)
    assert np.isfinite(losses).all()
    first, last = losses[:24].mean(), losses[-24:].mean()
    print(f"training loss {first:.4f} -> {last:.4f}")
    assert last < 0.8 * first
    held = random_geometric(1500, seed=7)
    G = grf.Graph(held.n_vertices, held.edges, held.lengths, h, "round")
    uj, sj = G.sample(2.5, beta, k, 8, 3, tol=1e-10)
    ul, sl = G.sample(2.5, beta, k, 8, 3, tol=1e-10, learned=net)
    ML = omesh.lumped_mass(omesh.build_mesh(held.n_vertices, held.edges, held.lengths, h, "round"))
    itj = sj["total_iterations"] / sj["n_systems"]
    itl = sl["total_iterations"] / sl["n_systems"]
    print(f"held-out RGG ({held.n_vertices} vertices): mean PCG iterations Jacobi {itj:.2f}, learned {itl:.2f}")
    assert _rel_ml(ul.cpu().numpy(), uj.cpu().numpy(), ML) <= 1e-8
    assert itl < 0.9 * itj
