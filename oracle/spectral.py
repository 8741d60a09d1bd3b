"""Spectral routes used to pin the direct solves (oracle, FP64).

* ``eig_sample``: with K = kappa^2 M_L + G and the generalised eigenpairs
  K V = M_L V diag(lam), V^T M_L V = I, every shifted matrix is
  A^(l) = c_I M_L + c_L K = M_L V diag(c_I + c_L lam) V^T M_L, hence
  sum_l A^(l)^{-1} W = V diag(q_k(lam)) V^T W with the scalar quadrature q_k.
  Its covariance is V diag(q_k(lam)^2) V^T (white noise has Cov W = M_L).
* ``interval_sample``: on a single edge with a uniform mesh of n elements
  and lumped mass, the generalised eigenvectors are the Neumann cosines
  v_n(x_j) = cos(n pi j / n), with eigenvalues kappa^2 + (4/h^2) sin^2(n pi/(2n))
  (the discrete Neumann Laplacian with trapezoid weights), n = 0..n.
  This closed form is textbook (DCT-I), not from the paper.
  With the consistent mass in the shifted matrix (``mass="consistent"``) the
  same cosines diagonalise it: the element matrices (h/6)[[2,1],[1,2]] give
  M_C v_n = c_n M_L v_n with c_n = (2 + cos(n pi / n_el)) / 3, so
  A^(l) v_n = ((c_I + c_L kappa^2) c_n + c_L mu_n) M_L v_n (mu_n the Laplacian
  eigenvalue) and sum_l 1/(...) = q_k(kappa^2 + mu_n / c_n) / c_n.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import mesh as _mesh
from . import quadrature as _quad


def generalized_eig(m: _mesh.Mesh, kappa: float):
    ML = _mesh.lumped_mass(m)
    G = _mesh.stiffness(m).toarray()
    K = kappa * kappa * np.diag(ML) + G
    lam, V = sla.eigh(K, np.diag(ML))
    return lam, V


def eig_sample(m: _mesh.Mesh, kappa: float, beta: float, k: float, W: np.ndarray,
               k_minus=None, k_plus=None) -> np.ndarray:
    lam, V = generalized_eig(m, kappa)
    q = _quad.q_k(lam, beta, k, k_minus, k_plus)
    W = np.atleast_2d(W)
    return ((V * q) @ (V.T @ W.T)).T


def eig_covariance(m: _mesh.Mesh, kappa: float, beta: float, k: float, k_minus=None, k_plus=None) -> np.ndarray:
    lam, V = generalized_eig(m, kappa)
    q = _quad.q_k(lam, beta, k, k_minus, k_plus)
    return (V * (q * q)) @ V.T


def interval_sample(length: float, n_el: int, kappa: float, beta: float, k: float, W: np.ndarray,
                    k_minus=None, k_plus=None, mass: str = "lumped") -> np.ndarray:
    """Closed-form sample on the graph interval(length) meshed with n_el
    elements, returned in the sampler's DOF order (interior nodes 1..n-1,
    then vertex 0 at x = 0, then vertex 1 at x = length).  ``mass`` is the
    mass matrix of the shifted systems (the load W is given either way)."""
    n = int(n_el)
    h = length / n
    j = np.arange(n + 1, dtype=np.float64)
    modes = np.arange(n + 1, dtype=np.float64)
    C = np.cos(np.pi * np.outer(j, modes) / n)  # C[j, mode]
    mu = (4.0 / (h * h)) * np.sin(np.pi * modes / (2.0 * n)) ** 2
    w = np.full(n + 1, h)
    w[0] = w[-1] = 0.5 * h  # lumped masses along the interval
    norm2 = (C * C * w[:, None]).sum(axis=0)
    if mass == "lumped":
        q = _quad.q_k(kappa * kappa + mu, beta, k, k_minus, k_plus)
    elif mass == "consistent":
        c = (2.0 + np.cos(np.pi * modes / n)) / 3.0
        q = _quad.q_k(kappa * kappa + mu / c, beta, k, k_minus, k_plus) / c
    else:
        raise ValueError(mass)
    order = np.concatenate([np.arange(1, n), [0, n]])  # DOF order -> node index j
    W = np.atleast_2d(W)
    Wn = np.zeros((W.shape[0], n + 1))
    Wn[:, order] = W
    coef = (Wn @ C) / norm2 * q
    un = coef @ C.T
    return un[:, order]
