"""The condensed oracle (static condensation with LAPACK tridiagonal solves,
oracle/condensed.py) against the assembled sparse LU of oracle/solve.py: the
same shifted systems reached by a different route (paper: eq.
local_reduced_schur, eq. global_schur, eq. internal_recovery).  Bar: 1e-12
relative, element by element, at shifts from mass- to stiffness-dominated, for
both mass matrices, on graphs with edges of 0, 1, 2 and many interior nodes, a
self-loop, a multi-edge and a pendant vertex."""

import numpy as np
import pytest

from oracle import condensed, mesh, noise, quadrature, solve
from workloads import config_c1, lattice, preferential_attachment


def _ragged():
    g = preferential_attachment(12, 2, lengths=(0.05, 1.7), seed=11)
    edges = np.vstack([g.edges, [[0, 1], [5, 5], [3, 12]]])
    lengths = np.concatenate([g.lengths, [0.013, 0.9, 0.31]])
    return 13, edges, lengths


@pytest.mark.parametrize("mass", ["lumped", "consistent"])
@pytest.mark.parametrize("rule,h", [("round", 0.07), ("ceil", 0.3), ("ceil", 2.0)])
@pytest.mark.parametrize("kappa,cI,cL", [(3.0, 1.0, 1.0), (3.0, 1e-9, 1e9), (3.0, 1e9, 1e-9), (0.5, 2e3, 1e-2)])
def test_condensed_equals_assembled(mass, rule, h, kappa, cI, cL):
    V, E, L = _ragged()
    m = mesh.build_mesh(V, E, L, h, rule)
    B = np.random.default_rng(5).standard_normal((3, m.n_dof))
    x = condensed.solve_shifted(m, kappa, cI, cL, B, mass=mass)
    ref = solve.solve_shifted(m, kappa, cI, cL, B, mass=mass)
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()
    # the residual of the assembled system, a check that needs no second solver
    A = solve.shifted_matrix(m, kappa, cI, cL, mass)
    assert np.abs((A @ x.T).T - B).max() <= 1e-12 * np.abs(B).max() * max(1.0, abs(A).max())


def test_condensed_sample_c1_serial_and_parallel():
    cfg = config_c1()
    g = cfg["graph"]
    m = mesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    W = noise.white_noise(mesh.lumped_mass(m), cfg["seed"], 3)
    ref = solve.sample(m, cfg["kappa"], cfg["beta"], cfg["quad_step"], W)
    u1 = condensed.sample(m, cfg["kappa"], cfg["beta"], cfg["quad_step"], W)
    u2 = condensed.sample(m, cfg["kappa"], cfg["beta"], cfg["quad_step"], W, workers=2)
    assert np.abs(u1 - u2).max() <= 1e-15 * np.abs(u1).max() * 55  # the same terms, grouped by piece
    assert np.abs(u1 - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(u2 - ref).max() <= 1e-12 * np.abs(ref).max()


def test_condensed_lattice_with_random_lengths():
    g = lattice(6, 5, lengths=(0.5, 1.5), seed=1)
    m = mesh.build_mesh(g.n_vertices, g.edges, g.lengths, 1 / 32, "round")
    W = noise.white_noise(mesh.lumped_mass(m), 2, 2)
    _, cI, cL = quadrature.shifts(0.85, 0.3)
    for i in (0, len(cI) // 2, len(cI) - 1):
        x = condensed.solve_shifted(m, 10.0, float(cI[i]), float(cL[i]), W)
        ref = solve.solve_shifted(m, 10.0, float(cI[i]), float(cL[i]), W)
        assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()
