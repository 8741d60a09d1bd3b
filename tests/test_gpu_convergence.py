"""The sampler with caller-supplied noise, and the paper's convergence rates
(Table 1) reproduced with the GPU sampler as the engine, scaled down.

* grf_sample_from_noise on the noise grf_noise draws equals grf_sample bit for
  bit, and equals the oracle's direct solve with the same noise to 1e-10.
* Convergence on the unit interval (section "Numerical Experiments", Table 1),
  as the oracle test of the same rates does it, with every solve on the GPU:
  kappa = 1, the paper's step k = -1/(beta ln h), 100 noise realisations drawn
  on an overkill mesh of 2^11 elements and projected onto the coarse meshes
  (2^3..2^6 elements) through the hat functions, so that all levels see the
  same white noise.  The strong error is the RMS over realisations of the
  lumped L2 norm of (overkill sample - prolonged coarse sample); the
  covariance error is the lumped L2(Gamma x Gamma) norm on the 2^10 mesh of
  the difference between the method's covariance there and on the coarse
  mesh, each covariance F M_L F^T from the solution operator F that the
  sampler applies to unit loads.  Bars as in the oracle test: strong slope
  within 0.04 of 2 beta - 1/2 and of the paper's measurement, covariance
  slope within 0.1 of min(4 beta - 1/2, 2) and of the paper's measurement.
"""

import math
import os

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import noise as onoise
from oracle import solve as osolve
from workloads import config_c1

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel_ml(u, ref, ML):
    """Worst sample's relative error, the larger of the lumped-mass norm
    ||u - ref||_{M_L} / ||ref||_{M_L} and the element-wise max |u - ref| / max |ref|
    (a local error that the norm would dilute fails the second)."""
    num = np.sqrt(((u - ref) ** 2 * ML).sum(axis=-1))
    den = np.sqrt((ref ** 2 * ML).sum(axis=-1))
    el = np.abs(u - ref).max(axis=-1) / np.abs(ref).max(axis=-1)
    return float(max(np.max(num / den), np.max(el)))


def test_from_noise_matches_sample_and_oracle(grf):
    import torch

    cfg = config_c1()
    g = cfg["graph"]
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    args = (cfg["kappa"], cfg["beta"], cfg["quad_step"])
    S = cfg["n_samples"]
    W = G.noise(S, cfg["seed"])
    u0, _ = G.sample(*args, S, cfg["seed"])
    u1, st = G.sample_from_noise(*args, W)
    assert st["n_unconverged"] == 0
    assert torch.equal(u0, u1)
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    ML = omesh.lumped_mass(m)
    Wr = np.random.default_rng(3).standard_normal((5, m.n_dof)) * np.sqrt(ML)  # any load, not only Philox noise
    u2, _ = G.sample_from_noise(*args, torch.from_numpy(Wr).cuda())
    ref = osolve.sample(m, cfg["kappa"], cfg["beta"], cfg["quad_step"], Wr)
    assert _rel_ml(u2.cpu().numpy(), ref, ML) <= 1e-10
    with pytest.raises(ValueError, match="alias"):
        G.sample_from_noise(*args, W, out=W)  # the binding's check
    # the library's own check, through the C ABI
    o = grf.make_opts()
    code = grf.load().grf_sample_from_noise(G.handle, *args, S, W.data_ptr(), W.data_ptr(), grf.C.byref(o))
    assert code == grf.GRF_EINVAL and b"alias" in grf.load().grf_last_error()


# ---- convergence rates ------------------------------------------------------------

def _order(n):
    """DOF order of the interval mesh -> node index (interior 1..n-1, then x = 0, x = 1)."""
    return np.concatenate([np.arange(1, n), [0, n]])


def _prolong(nc, nf):
    """Nodal values on the fine mesh of the coarse hat functions ([nf+1, nc+1])."""
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


def _weights(n):
    w = np.full(n + 1, 1.0 / n)
    w[0] = w[-1] = 0.5 / n
    return w


class _Interval:
    """The unit interval meshed with n elements, sampled on the GPU (node order in and out)."""

    def __init__(self, grf, n):
        self.n = n
        self.o = _order(n)
        self.G = grf.Graph(2, np.array([[0, 1]]), np.array([1.0]), 1.0 / n, "ceil")
        assert self.G.n_dof == n + 1

    def sample(self, kappa, beta, W_nodes):
        import torch

        noise = torch.from_numpy(np.ascontiguousarray(W_nodes[:, self.o])).cuda()
        u, st = self.G.sample_from_noise(kappa, beta, 0.0, noise)  # 0: the paper's step for this h
        assert st["n_unconverged"] == 0
        out = np.zeros(W_nodes.shape)
        out[:, self.o] = u.cpu().numpy()
        return out

    def operator(self, kappa, beta):
        """F (node order): column j is the sample for a unit load at node j."""
        return self.sample(kappa, beta, np.eye(self.n + 1)).T

    def close(self):
        self.G.close()


def _rates_gpu(grf, beta, kappa=1.0, pf=11, pc=10, levels=(3, 4, 5, 6), R=100):
    nf = 2 ** pf
    wf = _weights(nf)
    rng = np.random.default_rng(0)
    Wn = rng.standard_normal((R, nf + 1)) * np.sqrt(wf)
    fine = _Interval(grf, nf)
    uf = fine.sample(kappa, beta, Wn)
    fine.close()
    nr = 2 ** pc  # covariance reference mesh
    wr = _weights(nr)
    mr = _Interval(grf, nr)
    Fr = mr.operator(kappa, beta)
    mr.close()
    Cr = Fr @ np.diag(wr) @ Fr.T
    strong, cov, hs = [], [], []
    for lv in levels:
        nc = 2 ** lv
        P = _prolong(nc, nf)
        coarse = _Interval(grf, nc)
        uc = coarse.sample(kappa, beta, Wn @ P)
        e = uf - uc @ P.T
        strong.append(math.sqrt(((e * e) * wf).sum(axis=1).mean()))
        Pr = _prolong(nc, nr)
        Fc = Pr @ coarse.operator(kappa, beta) @ Pr.T
        coarse.close()
        D = Cr - Fc @ np.diag(wr) @ Fc.T
        cov.append(math.sqrt((D * D * wr[:, None] * wr[None, :]).sum()))
        hs.append(1.0 / nc)
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
def test_convergence_rates_table1_gpu(grf, row):
    beta, strong_paper, cov_paper, strong_th, cov_th = _table1()[row]
    strong, cov = _rates_gpu(grf, beta)
    print(f"beta {beta}: strong slope {strong:.3f} (paper {strong_paper}, theory {strong_th}); "
          f"covariance slope {cov:.3f} (paper {cov_paper}, theory {cov_th})", flush=True)
    assert abs(strong - strong_th) <= 0.04
    assert abs(strong - strong_paper) <= 0.04
    assert abs(cov - cov_th) <= 0.1
    assert abs(cov - cov_paper) <= 0.1


def _four_edges(grf, h=1.0 / 64):
    edges = np.array([[0, 1], [1, 2], [2, 0], [2, 3]])
    lengths = np.array([2.0, 1.5, 1.0, 3.0])
    return grf.Graph(4, edges, lengths, h, "ceil"), omesh.build_mesh(4, edges, lengths, h, "ceil")


@pytest.mark.parametrize("cI,cL", [(1e3, 1e-3), (1e4, 1e-4), (1.0, 1.0), (1e-6, 1e6)])
def test_point_loads_reach_the_oracle(grf, cI, cL):
    """Unit loads at the middle of each edge, at an edge's first node and at a vertex.
    At the two mass-dominated shifts the middle loads reach the vertices as 6e-77 down
    to 6e-230 (1e3, 1e-3) and 8e-141 down to 0 (1e4, 1e-4): their squared norms leave
    the double range and the systems are rescaled exactly.  Every system converges and
    the solution matches the direct solve."""
    import torch

    G, m = _four_edges(grf)
    rows = [int(m.offsets[e] + m.m(e) // 2) for e in range(4)] + [int(m.offsets[0]), m.n_interior + 3]
    B = np.zeros((len(rows), m.n_dof))
    B[np.arange(len(rows)), rows] = 1.0
    x, st = G.solve_shifted(2.0, cI, cL, torch.from_numpy(B).cuda())
    ref = osolve.solve_shifted(m, 2.0, cI, cL, B)
    assert st["n_unconverged"] == 0
    assert _rel_ml(x.cpu().numpy(), ref, omesh.lumped_mass(m)) <= 1e-10


@pytest.mark.parametrize("k", [-500, 500])
def test_range_scaling_is_exact(grf, k):
    """Solving for 2^k B gives exactly 2^k times the solution for B, bit for bit (power-of-two
    scaling is exact); without the range scaling the stopping test of these systems under- or
    overflows."""
    import torch

    G, m = _four_edges(grf)
    B = torch.from_numpy(np.random.default_rng(9).standard_normal((5, m.n_dof))).cuda()
    x1, _ = G.solve_shifted(3.0, 0.7, 1.9, B)
    x2, st = G.solve_shifted(3.0, 0.7, 1.9, torch.ldexp(B, torch.tensor(k, device="cuda")))
    assert st["n_unconverged"] == 0
    assert torch.equal(x2, torch.ldexp(x1, torch.tensor(k, device="cuda")))
