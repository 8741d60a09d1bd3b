"""Statistical checks of the GPU sampler on a tiny graph (through the C ABI).

With white noise of covariance M (eq. wh_def), the quadrature sum
sum_l A^(l)^{-1} W is V diag(q_k(lam)) V^T W (eq. spde_approx_fem with the
generalized eigenpairs of (kappa^2 M_L + G, M_L)), so a sample's covariance
is V diag(q_k(lam)^2) V^T exactly (oracle.spectral.eig_covariance).  100,000
seeded samples of a 19-DOF star graph must match it entry by entry: the
standard error of a covariance estimate from S zero-mean Gaussian samples is
sqrt((C_ii C_jj + C_ij^2) / S), and every entry lies within 4.5 of them (the
fixed seed's largest deviation is printed).  The same bar holds for the
lumped noise against M_L and the consistent-mass noise against M_C.
"""

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import spectral

pytestmark = pytest.mark.gpu
S = 100_000
BAR = 4.5


def _star():
    edges = np.array([[0, 1], [0, 2], [0, 3]])
    lengths = np.array([0.5, 0.75, 1.0])
    return 4, edges, lengths, 1 / 8, "ceil"


def _z(samples, C):
    Cs = samples.T @ samples / samples.shape[0]
    d = np.diag(C)
    se = np.sqrt((np.outer(d, d) + C * C) / samples.shape[0])
    return np.abs(Cs - C) / se


def test_sample_covariance_is_the_method_covariance(grf):
    V, E, L, h, rule = _star()
    m = omesh.build_mesh(V, E, L, h, rule)
    G = grf.Graph(V, E, L, h, rule)
    kappa, beta, k = 2.0, 0.75, 0.5
    u, st = G.sample(kappa, beta, k, S, 17, tol=1e-12)
    assert st["n_unconverged"] == 0 and m.n_dof == G.n_dof == 19
    z = _z(u.cpu().numpy(), spectral.eig_covariance(m, kappa, beta, k))
    print(f"sample covariance: largest deviation {z.max():.2f} standard errors over {z.size} entries")
    assert z.max() <= BAR


@pytest.mark.parametrize("kind", ["lumped", "consistent"])
def test_noise_covariance_is_the_mass_matrix(grf, kind):
    V, E, L, h, rule = _star()
    m = omesh.build_mesh(V, E, L, h, rule)
    G = grf.Graph(V, E, L, h, rule, noise=kind)
    M = np.diag(omesh.lumped_mass(m)) if kind == "lumped" else omesh.consistent_mass(m).toarray()
    W = G.noise(S, 23).cpu().numpy()
    z = _z(W, M)
    print(f"{kind} noise covariance: largest deviation {z.max():.2f} standard errors")
    assert z.max() <= BAR
