"""Failure reporting of the HIP path (through the C ABI): a NaN or Inf in a
right-hand side or in the noise reaches every vertex Schur system it touches
(an interior value flows to both ends of its edge through the Thomas sweeps
of eq. thomas_coefficients, a vertex value is one), the call returns
GRF_ENONFINITE with the output still written, the affected right-hand sides
hold NaN, and every other right-hand side is solved as if the bad ones were
absent (within the parity bar 1e-10 of the same call without them).
"""

import numpy as np
import pytest

from workloads import config_c1

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def c1(grf):
    cfg = config_c1()
    g = cfg["graph"]
    return grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _bad_rhs(G, torch, n=6):
    gen = torch.Generator().manual_seed(5)
    B = torch.randn((n, G.n_dof), dtype=torch.float64, generator=gen)
    clean = B.clone()
    ni = G.n_interior
    B[1, ni // 2] = float("nan")      # interior DOF
    B[3, ni + 2] = float("inf")       # vertex DOF
    B[4, 7] = -float("inf")           # interior DOF near an edge end
    return B.cuda(), clean.cuda(), [1, 3, 4], [0, 2, 5]


@pytest.mark.parametrize("precond", ["jacobi", "nn"])
def test_nonfinite_rhs_is_reported(grf, c1, precond):
    import torch

    G = c1
    B, clean, bad, good = _bad_rhs(G, torch)
    with pytest.raises(grf.GrfError) as ei:
        G.solve_shifted(2.0, 1.0, 0.7, B, precond=precond)
    assert ei.value.code == grf.GRF_ENONFINITE
    x, st = G.solve_shifted(2.0, 1.0, 0.7, B, precond=precond, allow_nonfinite=True)
    ref, st_ref = G.solve_shifted(2.0, 1.0, 0.7, clean, precond=precond)
    assert st["n_nonfinite"] == len(bad) and st_ref["n_nonfinite"] == 0
    x, ref = x.cpu().numpy(), ref.cpu().numpy()
    assert np.isnan(x[bad]).all(), "every DOF of a connected graph depends on its vertex values"
    assert np.isfinite(x[good]).all()
    assert _rel(x[good], ref[good]) <= TOL


def test_nonfinite_noise_is_reported(grf, c1):
    import torch

    G = c1
    W = G.noise(4, 3)
    Wb = W.clone()
    Wb[2, 11] = float("nan")
    u, st = G.sample_from_noise(5.0, 0.75, 0.5, Wb, allow_nonfinite=True)
    ref, _ = G.sample_from_noise(5.0, 0.75, 0.5, W)
    assert st["n_nonfinite"] == st["n_shifts"], "the bad sample fails at every shift"
    u, ref = u.cpu().numpy(), ref.cpu().numpy()
    assert np.isnan(u[2]).all()
    assert _rel(u[[0, 1, 3]], ref[[0, 1, 3]]) <= TOL
    with pytest.raises(grf.GrfError) as ei:
        G.sample_from_noise(5.0, 0.75, 0.5, Wb)
    assert ei.value.code == grf.GRF_ENONFINITE
    # the same graph solves clean input again afterwards
    again, st2 = G.sample_from_noise(5.0, 0.75, 0.5, W)
    assert st2["n_nonfinite"] == 0 and np.array_equal(again.cpu().numpy(), ref)


def test_fp32_range_in_mixed_precision(grf, c1):
    """FP64 scales a right-hand side of any finite size exactly (powers of two);
    the FP32 edge sweeps of mixed precision overflow past 3.4e38, and the call
    says so instead of returning a wrong solution."""
    import torch

    G = c1
    gen = torch.Generator().manual_seed(9)
    B = torch.randn((3, G.n_dof), dtype=torch.float64, generator=gen)
    B[1] *= 1e300
    Bd = B.cuda()
    x, st = G.solve_shifted(2.0, 1.0, 0.7, Bd)
    assert st["n_nonfinite"] == 0 and np.isfinite(x.cpu().numpy()).all()
    xm, stm = G.solve_shifted(2.0, 1.0, 0.7, Bd, precision="mixed", allow_nonfinite=True)
    assert stm["n_nonfinite"] >= 1
    xm = xm.cpu().numpy()
    assert np.isnan(xm[1]).all()
    x = x.cpu().numpy()
    assert _rel(xm[[0, 2]], x[[0, 2]]) <= TOL
