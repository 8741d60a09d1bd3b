"""Full-size checks in the launch configuration of the throughput benchmark
(64x64 random-length lattice, h = 1/256 rounded mesh, 2,066,964 DOFs, kappa =
10, beta = 0.6, step 0.3: 116 shifts, 256 samples, blocked FP64 sweeps), and
of the 256x256 mixed-precision configuration.  At these sizes the oracle
computes single results, so the checks are sampled outputs and properties
that hold at any size:
  * noise bit-identical to the oracle for sampled samples;
  * conservation <M_L, u> = q_k(kappa^2) <1, W> for every sample;
  * single-shift solves: the residual of the assembled system below 1e-10, and
    one shift against the oracle's sparse direct solve (1e-10);
  * linearity: the multi-shift sample equals the sum of the single-shift solves
    (sampled samples, 1e-10);
  * mixed precision at 66.7M DOFs: the sample within 1e-6 of the FP64 path,
    refined single-shift solves within 1e-9 at the extreme and middle shifts.
"""

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import noise as onoise
from oracle import quadrature as oquad
from oracle import solve as osolve
from workloads import config_c2, config_c4

pytestmark = pytest.mark.gpu


def _rel_ml(u, ref, ML):
    num = np.sqrt(((u - ref) ** 2 * ML).sum(axis=-1))
    den = np.sqrt((ref ** 2 * ML).sum(axis=-1))
    return float(np.max(num / den))


@pytest.fixture(scope="module")
def c2(grf):
    cfg = config_c2(beta=0.6, n_samples=256)
    g = cfg["graph"]
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    return cfg, m, G


def test_c2_sample_noise_and_conservation(grf, c2):
    cfg, m, G = c2
    S = cfg["n_samples"]
    u, st = G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"], tol=cfg["tol"])
    assert st["n_shifts"] == 116 and st["shift_block"] == 116 and st["sweep_block"] == 0 and st["n_unconverged"] == 0
    W = G.noise(S, cfg["seed"])
    ML = omesh.lumped_mass(m)
    for s in (0, 77, 255):  # sampled noise rows against the oracle, bit for bit
        ref = onoise.white_noise(ML, cfg["seed"], 1, sample_offset=s)[0]
        assert np.array_equal(W[s].cpu().numpy().view(np.uint64), ref.view(np.uint64))
    q = oquad.q_k(cfg["kappa"] ** 2, cfg["beta"], cfg["quad_step"])
    Wn = W.cpu().numpy()
    lhs = (u.cpu().numpy() * ML).sum(axis=1)
    rhs = q * Wn.sum(axis=1)
    scale = q * (np.abs(Wn) * 1.0).sum(axis=1)
    assert np.max(np.abs(lhs - rhs) / scale) <= 1e-12


def test_c2_single_shift_solves(grf, c2):
    import torch

    cfg, m, G = c2
    ls, cI, cL = oquad.shifts(cfg["beta"], cfg["quad_step"])
    W = G.noise(4, cfg["seed"])
    Wn = W.cpu().numpy()
    for i in (0, len(ls) // 2, len(ls) - 1):
        x, st = G.solve_shifted(cfg["kappa"], float(cI[i]), float(cL[i]), W, tol=cfg["tol"])
        A = osolve.shifted_matrix(m, cfg["kappa"], float(cI[i]), float(cL[i]))
        xn = x.cpu().numpy()
        res = np.linalg.norm((A @ xn.T).T - Wn, axis=1) / np.linalg.norm(Wn, axis=1)
        assert res.max() <= 1e-10, f"shift {ls[i]}: residual {res.max():.2e}"
    i = len(ls) // 2
    x, _ = G.solve_shifted(cfg["kappa"], float(cI[i]), float(cL[i]), W[:1], tol=cfg["tol"])
    ref = osolve.solve_shifted(m, cfg["kappa"], float(cI[i]), float(cL[i]), Wn[:1])
    assert _rel_ml(x.cpu().numpy(), ref, omesh.lumped_mass(m)) <= 1e-10


def test_c2_sample_equals_sum_of_shift_solves(grf, c2):
    import torch

    cfg, m, G = c2
    S = 8
    u, _ = G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"], tol=cfg["tol"])
    W = G.noise(S, cfg["seed"])
    ls, cI, cL = oquad.shifts(cfg["beta"], cfg["quad_step"])
    acc = torch.zeros_like(W)
    for i in range(len(ls)):
        x, _ = G.solve_shifted(cfg["kappa"], float(cI[i]), float(cL[i]), W, tol=cfg["tol"])
        acc += x
    assert _rel_ml(u.cpu().numpy(), acc.cpu().numpy(), omesh.lumped_mass(m)) <= 1e-10


def test_c4_mixed_full_size(grf):
    import torch

    cfg = config_c4(n_samples=8)
    g = cfg["graph"]
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    assert G.n_dof > 66_000_000
    K = cfg["k_minus"]
    kw = dict(k_minus=K, k_plus=cfg["k_plus"], tol=cfg["tol"])
    u64, s64 = G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], 8, cfg["seed"], **kw)
    u32, s32 = G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], 8, cfg["seed"], precision="mixed", **kw)
    assert s64["n_shifts"] == 93 == s32["n_shifts"]
    ML = torch.from_numpy(omesh.lumped_mass(omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"],
                                                            cfg["rule"]))).cuda()
    d = u32 - u64
    err = torch.sqrt((d * d * ML).sum(1) / (u64 * u64 * ML).sum(1)).max().item()
    print(f"256x256 lattice ({G.n_dof} DOFs, 93 shifts): mixed vs FP64 sample error {err:.2e}")
    assert err <= 1e-6
    ls, cI, cL = oquad.shifts(cfg["beta"], cfg["quad_step"], K, cfg["k_plus"])
    W = G.noise(2, cfg["seed"])
    for i in (0, len(ls) // 2, len(ls) - 1):
        x64, _ = G.solve_shifted(cfg["kappa"], float(cI[i]), float(cL[i]), W, tol=cfg["tol"])
        x32, st = G.solve_shifted(cfg["kappa"], float(cI[i]), float(cL[i]), W, tol=cfg["tol"], precision="mixed",
                                  refine=2)
        d = x32 - x64
        e = torch.sqrt((d * d * ML).sum(1) / (x64 * x64 * ML).sum(1)).max().item()
        print(f"shift l={ls[i]:+d}: refined mixed vs FP64 {e:.2e}, residual {st['max_rel_residual']:.1e}")
        assert e <= 1e-9
