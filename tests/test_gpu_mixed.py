"""Mixed precision (FP32 operand tables and matrix-core edge sweeps; FP64 noise,
Schur complements, PCG, accumulation; FP64-residual iterative refinement for
single-shift solves) against the FP64 oracle and the FP64 GPU path.

Bars (lumped-mass norm, max over right-hand sides / samples):
  * quadrature sum (grf_sample): within 1e-6 relative, the accuracy at which
    the throughput metric counts a result;
  * one shifted system (grf_solve_shifted) after two refinement steps: within
    1e-10 relative of the oracle at every shift of a span e^{2y} in [1e-8, 1e8],
    each shift's error reported; without refinement (the edge arithmetic of the
    sampled path, per shift) within 1e-6.
"""

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import noise as onoise
from oracle import quadrature as oquad
from oracle import solve as osolve
from workloads import config_c1, lattice, preferential_attachment

pytestmark = pytest.mark.gpu
SUM_TOL = 1e-6
REFINED_TOL = 1e-10
# one shift with FP32 edge sweeps and no refinement (the per-shift arithmetic of the
# sampled mixed path): FP32 unit roundoff 6e-8 times a small factor; measured at most
# 2.1e-7 over e^{2y} in [1e-8, 1e8], on this lattice and on the full 256x256 one
UNREFINED_TOL = 1e-6


def _rel_ml(u, ref, ML):
    """Worst sample's relative error, the larger of the lumped-mass norm
    ||u - ref||_{M_L} / ||ref||_{M_L} and the element-wise max |u - ref| / max |ref|
    (a local error that the norm would dilute fails the second)."""
    num = np.sqrt(((u - ref) ** 2 * ML).sum(axis=-1))
    den = np.sqrt((ref ** 2 * ML).sum(axis=-1))
    el = np.abs(u - ref).max(axis=-1) / np.abs(ref).max(axis=-1)
    return float(max(np.max(num / den), np.max(el)))


def test_mixed_sample_c1(grf):
    cfg = config_c1()
    g = cfg["graph"]
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    u, st = G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], cfg["n_samples"], cfg["seed"], tol=cfg["tol"],
                     precision="mixed")
    W = onoise.white_noise(omesh.lumped_mass(m), cfg["seed"], cfg["n_samples"])
    ref = osolve.sample(m, cfg["kappa"], cfg["beta"], cfg["quad_step"], W)
    err = _rel_ml(u.cpu().numpy(), ref, omesh.lumped_mass(m))
    print(f"mixed C1 sample error {err:.3e}")
    assert err <= SUM_TOL and st["n_unconverged"] == 0


def test_mixed_sample_ragged_multipass(grf):
    g = preferential_attachment(12, 2, lengths=(0.05, 1.7), seed=11)
    edges = np.vstack([g.edges, [[0, 1], [5, 5], [3, 12]]])
    lengths = np.concatenate([g.lengths, [0.013, 0.9, 0.31]])
    m = omesh.build_mesh(13, edges, lengths, 0.05, "round")
    G = grf.Graph(13, edges, lengths, 0.05, "round")
    kappa, beta, k, S, seed = 4.0, 0.6, 0.45, 70, 3
    u, _ = G.sample(kappa, beta, k, S, seed, shift_block=16, precision="mixed")
    W = onoise.white_noise(omesh.lumped_mass(m), seed, S)
    ref = osolve.sample(m, kappa, beta, k, W)
    err = _rel_ml(u.cpu().numpy(), ref, omesh.lumped_mass(m))
    print(f"mixed ragged multipass sample error {err:.3e}")
    assert err <= SUM_TOL


@pytest.mark.parametrize("S,shift_block", [(9, 0), (24, 0), (24, 40), (31, 16)])
def test_mixed_sample_few_samples(grf, S, shift_block):
    """1 and 2 wavefronts of 16 samples per edge workgroup (S <= 32), where the FP32
    edge sweeps stage each block's operands through a single LDS buffer; edges of
    up to three 16-position blocks, ragged sample lanes, one and several shift passes."""
    g = preferential_attachment(12, 2, lengths=(0.05, 1.7), seed=11)
    edges = np.vstack([g.edges, [[0, 1], [5, 5], [3, 12]]])
    lengths = np.concatenate([g.lengths, [0.013, 0.9, 0.31]])
    m = omesh.build_mesh(13, edges, lengths, 0.05, "round")
    G = grf.Graph(13, edges, lengths, 0.05, "round")
    kappa, beta, k, seed = 4.0, 0.6, 0.45, 8
    u, st = G.sample(kappa, beta, k, S, seed, shift_block=shift_block, precision="mixed")
    W = onoise.white_noise(omesh.lumped_mass(m), seed, S)
    ref = osolve.sample(m, kappa, beta, k, W)
    err = _rel_ml(u.cpu().numpy(), ref, omesh.lumped_mass(m))
    print(f"mixed, {S} samples, shift block {st['shift_block']}: sample error {err:.3e}")
    assert err <= SUM_TOL


def _c4_shaped(n=12):
    """The 256x256 mixed-precision configuration's parameters on a smaller lattice."""
    g = lattice(n, n, lengths=(0.5, 1.5), seed=4)
    return g, 1.0 / 512, 20.0, 0.55, 0.2, 46


def test_mixed_solve_refined_per_shift(grf):
    import torch

    g, h, kappa, beta, k, K = _c4_shaped()
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, h, "round")
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, h, "round")
    ML = omesh.lumped_mass(m)
    ls, cI, cL = oquad.shifts(beta, k, K, K)
    B = onoise.white_noise(ML, 0, 8)
    Bd = torch.from_numpy(B).cuda()
    report = []
    for i in np.linspace(0, len(ls) - 1, 7).round().astype(int):
        ref = osolve.solve_shifted(m, kappa, float(cI[i]), float(cL[i]), B)
        x0, _ = G.solve_shifted(kappa, float(cI[i]), float(cL[i]), Bd, precision="mixed", refine=0)
        x2, st = G.solve_shifted(kappa, float(cI[i]), float(cL[i]), Bd, precision="mixed", refine=2)
        e0 = _rel_ml(x0.cpu().numpy(), ref, ML)
        e2 = _rel_ml(x2.cpu().numpy(), ref, ML)
        report.append((int(ls[i]), e0, e2, st["max_rel_residual"]))
        assert st["refine_steps"] == 2
        assert e2 <= REFINED_TOL, f"shift l={ls[i]}: refined error {e2:.3e}"
        assert e0 <= UNREFINED_TOL, f"shift l={ls[i]}: unrefined FP32-sweep error {e0:.3e}"
    for l, e0, e2, r in report:
        print(f"l={l:+d} e^2y={np.exp(2 * l * k):.1e}: FP32 sweeps {e0:.2e}, refined x2 {e2:.2e}, residual {r:.1e}")


def test_mixed_sample_matches_fp64_c4_shape(grf):
    g, h, kappa, beta, k, K = _c4_shaped(16)
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, h, "round")
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, h, "round")
    ML = omesh.lumped_mass(m)
    u64, _ = G.sample(kappa, beta, k, 16, 0, k_minus=K, k_plus=K)
    u32, st = G.sample(kappa, beta, k, 16, 0, k_minus=K, k_plus=K, precision="mixed")
    err = _rel_ml(u32.cpu().numpy(), u64.cpu().numpy(), ML)
    print(f"mixed vs FP64 sample error (C4-shaped, {st['n_shifts']} shifts) {err:.3e}")
    assert st["n_shifts"] == 2 * K + 1
    assert err <= SUM_TOL


def test_mixed_rejects_streamed_sweeps(grf):
    cfg = config_c1()
    g = cfg["graph"]
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    with pytest.raises(grf.GrfError) as ei:
        G.sample(5.0, 0.75, 0.5, 2, 0, precision="mixed", sweep_block=16)
    assert ei.value.code == grf.GRF_EINVAL
    # refinement is a property of single-shift solves; the sampling calls reject a request for it
    with pytest.raises(grf.GrfError, match="refine") as ei:
        G.sample(5.0, 0.75, 0.5, 2, 0, precision="mixed", refine=1)
    assert ei.value.code == grf.GRF_EINVAL
    with pytest.raises(grf.GrfError, match="refine"):
        grf.sample_batched([G], [5.0], 0.75, 0.5, 2, 0, precision="mixed", refine=2)
    G.sample(5.0, 0.75, 0.5, 2, 0, precision="mixed", refine=0)  # 0: accepted
