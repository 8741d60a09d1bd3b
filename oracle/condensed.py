"""Static condensation of the shifted systems with LAPACK tridiagonal solves
(oracle, FP64).  TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

Paper passages followed, in their order:

* "Phase 3" / eq. local_reduced_schur: per edge, the interior block A_II^(e)
  (tridiagonal), the edge's Schur complement
  S^(e) = A_GG^(e) - A_GI^(e) A_II^(e)^{-1} A_IG^(e) on its two end vertices
  and the condensed right-hand side g = W_G - A_GI A_II^{-1} W_I;
* eq. global_schur: S u_G = g with S the sum of the S^(e);
* eq. internal_recovery: u_I = A_II^{-1} (W_I - A_IG u_G);
* "Quadrature Accumulation and Global Assembly": u = sum_l u^(l), l increasing.

The entries are those of the assembled matrices of ``solve.shifted_matrix``
(reading A1: A^(l) = (c_I + c_L kappa^2) M + c_L G), per element:
interior diagonal alpha m_i + 2 gamma / h, interior and vertex coupling
b = alpha m_o - gamma / h, vertex share alpha m_v + gamma / h per edge end,
with (m_i, m_o, m_v) = (h, 0, h/2) lumped or (2h/3, h/6, h/3) consistent.

Instead of the Thomas algorithm the block-diagonal interior matrix of all edges
at once is factored by LAPACK's dpttrf (L D L^T of an SPD tridiagonal matrix,
zero couplings between edges) and solved by dpttrs.  The four end entries of
every edge's T^{-1} come from one solve with two right-hand sides (unit
entries at every edge's first, resp. last, interior node).  The vertex system
is assembled sparse and solved with SuperLU.  Nothing here loops over edges
in Python, so it serves at sizes where the assembled LU does not fit.  It
shares no code with the HIP library.  Pinned against ``solve`` (assembled
sparse LU) in tests/test_oracle_condensed.py.
"""

from __future__ import annotations

import concurrent.futures as cf
import multiprocessing as mp

import numpy as np
import scipy.linalg.lapack as lapack
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import mesh as _mesh
from . import quadrature as _quad


class Shifted:
    """The condensed form of A = (c_I + c_L kappa^2) M + c_L G on one mesh."""

    def __init__(self, m: _mesh.Mesh, kappa: float, c_I: float, c_L: float, mass: str = "lumped"):
        he = np.asarray(m.h_e, dtype=np.float64)
        me = (np.asarray(m.n_el) - 1).astype(np.int64)
        alpha = c_I + c_L * kappa * kappa
        gamma = c_L
        if mass == "lumped":
            mi, mo, mv = he, np.zeros_like(he), 0.5 * he
        elif mass == "consistent":
            mi, mo, mv = 2.0 * he / 3.0, he / 6.0, he / 3.0
        else:
            raise ValueError(mass)
        a_e = alpha * mi + gamma * 2.0 / he
        b_e = alpha * mo - gamma / he
        d_e = alpha * mv + gamma / he
        self.m, self.NI, self.V = m, m.n_interior, m.n_vertices
        u, v = m.edges[:, 0], m.edges[:, 1]
        has = me > 0
        first = m.offsets[:-1][has]
        last = (m.offsets[1:] - 1)[has]
        # interior tridiagonal (all edges): diagonal, and couplings inside an edge only
        self.d = np.repeat(a_e, me)
        off = np.repeat(b_e, me)
        inside = np.ones(self.NI, dtype=bool)
        inside[last] = False
        self.e = np.where(inside, off, 0.0)[:-1] if self.NI > 0 else np.zeros(0)
        if self.NI > 1:
            self.df, self.ef, info = lapack.dpttrf(self.d, self.e)
            if info != 0:
                raise np.linalg.LinAlgError(f"dpttrf info {info}")
        # A_GI (V x NI): b at (u_e, first_e) and (v_e, last_e) of every edge with interior nodes
        bh = b_e[has]
        self.AGI = sp.csr_matrix((np.concatenate([bh, bh]), (np.concatenate([u[has], v[has]]),
                                                           np.concatenate([first, last]))),
                                 shape=(self.V, self.NI))
        # end entries of T^{-1} per edge: one solve with two right-hand sides
        s00 = np.array(d_e, copy=True)
        s11 = np.array(d_e, copy=True)
        s01 = np.where(has, 0.0, b_e)  # an edge with no interior node couples its ends directly
        if self.NI > 0 and has.any():
            F = np.zeros((self.NI, 2))
            F[first, 0] = 1.0
            F[last, 1] = 1.0
            Z = self._solve_ii(F)
            b2 = bh * bh
            s00[has] -= b2 * Z[first, 0]
            s11[has] -= b2 * Z[last, 1]
            s01[has] -= b2 * Z[first, 1]  # = b^2 (T^{-1})_{m,1} by symmetry
        rows = np.concatenate([u, u, v, v])
        cols = np.concatenate([u, v, u, v])
        vals = np.concatenate([s00, s01, s01, s11])
        self.S = sp.csc_matrix((vals, (rows, cols)), shape=(self.V, self.V))
        self.lu = spla.splu(self.S)

    def _solve_ii(self, B: np.ndarray) -> np.ndarray:
        if self.NI == 1:  # a 1 x 1 block (LAPACK's wrapper wants n >= 2)
            return B / self.d[0]
        X, info = lapack.dpttrs(self.df, self.ef, B)
        if info != 0:
            raise np.linalg.LinAlgError(f"dpttrs info {info}")
        return X

    def solve(self, rhs: np.ndarray) -> np.ndarray:
        """x[s] = A^{-1} rhs[s] for rhs [S, N] (or [N])."""
        B = np.asarray(rhs, dtype=np.float64)
        one = B.ndim == 1
        B2 = B.reshape(1, -1) if one else B
        WI = np.asfortranarray(B2[:, :self.NI].T)
        WG = B2[:, self.NI:].T
        w = self._solve_ii(WI) if self.NI > 0 else WI
        g = WG - self.AGI @ w
        uG = self.lu.solve(np.ascontiguousarray(g))
        uI = self._solve_ii(np.asfortranarray(WI - self.AGI.T @ uG)) if self.NI > 0 else WI
        X = np.concatenate([uI, uG], axis=0).T
        return X[0] if one else np.ascontiguousarray(X)


def solve_shifted(m: _mesh.Mesh, kappa: float, c_I: float, c_L: float, rhs: np.ndarray,
                  mass: str = "lumped") -> np.ndarray:
    return Shifted(m, kappa, c_I, c_L, mass).solve(rhs)


def _range_task(args):
    """Sum of the solutions of a contiguous range of shifts, l increasing."""
    m, kappa, cIs, cLs, W, mass = args
    if isinstance(W, str):  # a .npy file, memory-mapped (large loads are not copied to every process)
        W = np.load(W, mmap_mode="r")
    u = np.zeros(W.shape, dtype=np.float64)
    for ci, cl in zip(cIs, cLs):
        u = u + solve_shifted(m, kappa, ci, cl, W, mass)
    return u


def sample(m: _mesh.Mesh, kappa: float, beta: float, k: float, W: np.ndarray,
           k_minus: int | None = None, k_plus: int | None = None, mass: str = "lumped",
           workers: int = 1):
    """u[s] = sum_l A^(l)^{-1} W[s], l increasing.  With workers > 1 the shift
    range is cut into that many contiguous pieces, each summed (l increasing) in
    a process of its own, and the partial sums are added in increasing order:
    the same terms in the same order, grouped by piece.  W is an array [S, N] or
    the path of a .npy file holding one."""
    _, c_I, c_L = _quad.shifts(beta, k, k_minus, k_plus)
    if not isinstance(W, str):
        W = np.asarray(W, dtype=np.float64)
    if workers <= 1:
        return _range_task((m, kappa, [float(x) for x in c_I], [float(x) for x in c_L], W, mass))
    cuts = np.linspace(0, len(c_I), min(workers, len(c_I)) + 1).round().astype(int)
    tasks = [(m, kappa, [float(x) for x in c_I[a:b]], [float(x) for x in c_L[a:b]], W, mass)
             for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    with cf.ProcessPoolExecutor(max_workers=len(tasks), mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_range_task, tasks))
    u = np.zeros(parts[0].shape, dtype=np.float64)
    for p in parts:
        u = u + p
    return u


def _shift_task(args):
    m, kappa, cI, cL, W, mass = args
    if isinstance(W, str):
        W = np.load(W, mmap_mode="r")
    return solve_shifted(m, kappa, cI, cL, np.asarray(W), mass)


def solve_shifts(m: _mesh.Mesh, kappa: float, c_I, c_L, W, mass: str = "lumped", workers: int = 1) -> list:
    """[A(c_I[i], c_L[i])^{-1} W for each i], one process per shift when workers > 1
    (W an array or the path of a .npy file)."""
    tasks = [(m, kappa, float(ci), float(cl), W, mass) for ci, cl in zip(c_I, c_L)]
    if workers <= 1 or len(tasks) <= 1:
        return [_shift_task(t) for t in tasks]
    with cf.ProcessPoolExecutor(max_workers=min(workers, len(tasks)), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_shift_task, tasks))
