"""Direct solves of the shifted FEM systems and the quadrature sum (oracle).

Paper passages followed:

* eq. spde_approx_fem: u ~ sum_{l=-K^-}^{K^+} (c_I M + c_L G)^{-1} W with the
  "statically generated" noise W (one W per sample, shared by all shifts).
* "Quadrature Accumulation and Global Assembly": u = sum_l u^(l), with u^(l)
  laid out as [u_I(e_1) ... u_I(e_|E|) u_Gamma].

Readings: the operator L = kappa^2 - Delta of eq. fractional_spde
discretises to kappa^2 M + G, so the shifted matrix is
A^(l) = (c_I + c_L kappa^2) M + c_L G; M is the same mass matrix as the noise
(lumped unless ``mass="consistent"``).  No blocking, condensation or
reordering happens here: the global matrix is assembled and solved.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import mesh as _mesh
from . import quadrature as _quad


def shifted_matrix(m: _mesh.Mesh, kappa: float, c_I: float, c_L: float, mass: str = "lumped") -> sp.csc_matrix:
    """A = (c_I + c_L kappa^2) M + c_L G, sparse."""
    G = _mesh.stiffness(m)
    if mass == "lumped":
        M = sp.diags(_mesh.lumped_mass(m))
    elif mass == "consistent":
        M = _mesh.consistent_mass(m)
    else:
        raise ValueError(mass)
    alpha = c_I + c_L * kappa * kappa
    return (alpha * M + c_L * G).tocsc()


def solve_shifted(m: _mesh.Mesh, kappa: float, c_I: float, c_L: float, rhs: np.ndarray,
                  method: str = "sparse", mass: str = "lumped") -> np.ndarray:
    """x[s] = A^{-1} rhs[s] for rhs of shape [S, N] (or [N])."""
    A = shifted_matrix(m, kappa, c_I, c_L, mass)
    B = np.asarray(rhs, dtype=np.float64)
    one = B.ndim == 1
    B2 = B.reshape(1, -1) if one else B
    if method == "dense":
        X = sla.solve(A.toarray(), B2.T, assume_a="pos").T
    elif method == "sparse":
        X = spla.splu(A).solve(np.ascontiguousarray(B2.T)).T
    else:
        raise ValueError(method)
    return X[0] if one else X


def sample(m: _mesh.Mesh, kappa: float, beta: float, k: float, W: np.ndarray,
           k_minus: int | None = None, k_plus: int | None = None,
           method: str = "sparse", mass: str = "lumped", per_shift: bool = False):
    """u[s] = sum_l A^(l)^{-1} W[s], l increasing.  With ``per_shift`` also
    return the list of per-shift solutions u^(l)."""
    _, c_I, c_L = _quad.shifts(beta, k, k_minus, k_plus)
    W = np.asarray(W, dtype=np.float64)
    u = np.zeros_like(W)
    parts = []
    for ci, cl in zip(c_I, c_L):
        ul = solve_shifted(m, kappa, float(ci), float(cl), W, method, mass)
        u = u + ul
        if per_shift:
            parts.append(ul)
    return (u, parts) if per_shift else u
