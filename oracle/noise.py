"""Counter-based normals and lumped-mass white noise (oracle, FP64).

Paper passages followed:

* eq. wh_def and "Generation of the Discrete White Noise Vector": draw
  xi ~ N(0, I_N) and set W = R xi with M = R R^T.
* "Mass Lumping" and Phase 2, lumped case: R = (M^lumped)^{1/2} is the
  element-wise square root of the diagonal, so W_j = sqrt(M_jj) xi_j.

The paper does not say how xi is drawn.  The generator below is this
project's definition, built so
that the CPU and the GPU produce bit-identical values:

* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): 4x64-bit counter, 2x64-bit key, ten rounds.
  Key = (seed, global sample index), counter = (j // 4, 0, 0, 0) for DOF j.
* 53-bit uniforms u = (x >> 11) * 2^-53.
* Box-Muller on the word pairs (x0, x1) and (x2, x3) with the project's own
  log and sin/cos built from +, -, *, / and sqrt in a fixed order (IEEE
  round-to-nearest, no fused multiply-add), so that any IEEE-754 machine
  evaluates them identically.
* DOF j takes component j % 4 of [r_a cos, r_a sin, r_b cos, r_b sin].

Consistent-mass noise (Phase 2, consistent case; eq. wh_def asks for any R
with M = R R^T, and the law of W = R xi does not depend on which): the paper
factors M by Cholesky.  Here R is the assembly of per-element factors.  The
consistent mass is the sum of the element matrices M_e = (h_e/6)[[2,1],[1,2]],
and M_e = F_e F_e^T with F_e = [[a, c], [a, -c]], a = sqrt(h_e/4),
c = sqrt(h_e/12) (the eigenvectors [1,1] and [1,-1] with eigenvalues h_e/2 and
h_e/6).  With two independent normals (p, q) per element, W = sum_e F_e (p, q)
has covariance sum_e M_e = M.  R is N x 2(#elements) and needs no
factorisation.  The project's definition of the draws:

* element g (global index over the edges in order, element k of edge e being
  g = offsets[e] + e + k, between local nodes k and k+1) takes the Philox block
  with counter (g // 2, 1, 0, 0) and the same key; (p, q) is the Box-Muller
  pair (r_a cos, r_a sin) for even g and (r_b cos, r_b sin) for odd g;
* element g adds t_left = a p + c q to its left node and t_right = a p - c q
  to its right node;
* an interior node adds its left element's t_right, then its right element's
  t_left; a vertex adds, starting from 0, the t of each incident edge end in
  increasing edge order, tail end before head end (t_left of the edge's first
  element at the tail, t_right of its last element at the head).
"""

from __future__ import annotations

import math

import numpy as np

# Philox4x64 round multipliers and Weyl key increments (Random123 paper).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
_MASK64 = (1 << 64) - 1


def philox4x64_10_int(counter, key) -> list[int]:
    """Reference Philox4x64-10 on Python integers (one block)."""
    c0, c1, c2, c3 = (int(x) & _MASK64 for x in counter)
    k0, k1 = (int(x) & _MASK64 for x in key)
    for _ in range(10):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & _MASK64
        hi1, lo1 = p1 >> 64, p1 & _MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + PHILOX_W0) & _MASK64
        k1 = (k1 + PHILOX_W1) & _MASK64
    return [c0, c1, c2, c3]


_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: int):
    """Full 64x64 -> 128 product of uint64 arrays by a constant, as (hi, lo)."""
    b = np.uint64(b)
    a_lo, a_hi = a & _M32, a >> _S32
    b_lo, b_hi = b & _M32, b >> _S32
    ll = a_lo * b_lo
    hl = a_hi * b_lo
    lh = a_lo * b_hi
    hh = a_hi * b_hi
    cross = (ll >> _S32) + (hl & _M32) + lh
    hi = hh + (hl >> _S32) + (cross >> _S32)
    lo = (cross << _S32) | (ll & _M32)
    return hi, lo


def philox4x64_10(ctr0: np.ndarray, k0: int, k1: int, ctr1: int = 0):
    """Vectorised Philox4x64-10 for counters (ctr0, ctr1, 0, 0) and one key."""
    with np.errstate(over="ignore"):
        c0 = np.asarray(ctr0, dtype=np.uint64).copy()
        c1 = np.full_like(c0, np.uint64(ctr1 & _MASK64))
        c2 = np.zeros_like(c0)
        c3 = np.zeros_like(c0)
        key0, key1 = np.uint64(k0 & _MASK64), np.uint64(k1 & _MASK64)
        for _ in range(10):
            hi0, lo0 = _mulhilo(c0, PHILOX_M0)
            hi1, lo1 = _mulhilo(c2, PHILOX_M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ key0, lo1, hi0 ^ c3 ^ key1, lo0
            key0 = key0 + np.uint64(PHILOX_W0)
            key1 = key1 + np.uint64(PHILOX_W1)
    return c0, c1, c2, c3


def uniform53(x: np.ndarray) -> np.ndarray:
    """u = (x >> 11) * 2^-53, in [0, 1)."""
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ---- log on (0, 1] -------------------------------------------------------
# log x = e ln2 + 2 atanh(s), s = (m-1)/(m+1), m in [sqrt(1/2), sqrt(2)),
# atanh(s) = s + s^3/3 + s^5/5 + ... truncated after s^25.
LOG_TERMS = 12
LOG_COEF = [0.0] + [1.0 / float(2 * k + 1) for k in range(1, LOG_TERMS + 1)]  # 1/3, 1/5, ...
SQRT_HALF = float.fromhex("0x1.6a09e667f3bcdp-1")
LN2_HI = float.fromhex("0x1.62e42fee00000p-1")  # ln 2 with 21 trailing zero bits
LN2_LO = float.fromhex("0x1.a39ef35793c76p-33")  # ln 2 - LN2_HI


def log_fixed(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    small = m < SQRT_HALF
    m = np.where(small, m * 2.0, m)
    e = np.where(small, e - 1, e).astype(np.float64)
    f = m - 1.0
    s = f / (m + 1.0)
    s2 = s * s
    q = np.full_like(s, LOG_COEF[LOG_TERMS])
    for k in range(LOG_TERMS - 1, 0, -1):
        q = q * s2
        q = q + LOG_COEF[k]
    r = s2 * q
    lm = s + s * r
    t1 = 2.0 * lm
    t2 = e * LN2_LO
    t3 = t1 + t2
    t4 = e * LN2_HI
    return t4 + t3


# ---- sin / cos of 2 pi u for u in [0, 1) ---------------------------------
TRIG_TERMS = 10
PI_4 = float.fromhex("0x1.921fb54442d18p-1")  # nearest double to pi/4
SIN_COEF = [0.0] + [(-1.0) ** k / float(math.factorial(2 * k + 1)) for k in range(1, TRIG_TERMS + 1)]
COS_COEF = [0.0] + [(-1.0) ** k / float(math.factorial(2 * k)) for k in range(1, TRIG_TERMS + 1)]


def sincos_2pi_fixed(u: np.ndarray):
    """(sin 2 pi u, cos 2 pi u): octant reduction on the dyadic u, Taylor
    polynomials on [0, pi/4], octant symmetries."""
    u = np.asarray(u, dtype=np.float64)
    t = u * 8.0
    o = np.floor(t)
    f = t - o
    o = o.astype(np.int64)
    odd = (o & 1) == 1
    f = np.where(odd, 1.0 - f, f)
    a = f * PI_4
    a2 = a * a
    ps = np.full_like(a, SIN_COEF[TRIG_TERMS])
    pc = np.full_like(a, COS_COEF[TRIG_TERMS])
    for k in range(TRIG_TERMS - 1, 0, -1):
        ps = ps * a2
        ps = ps + SIN_COEF[k]
        pc = pc * a2
        pc = pc + COS_COEF[k]
    sa = a + a * (a2 * ps)
    ca = 1.0 + a2 * pc
    # (sin, cos) of o*pi/4 + theta, with a = theta (even o) or pi/4 - theta (odd o)
    sin_sel = [sa, ca, ca, sa, -sa, -ca, -ca, -sa]
    cos_sel = [ca, sa, -sa, -ca, -ca, -sa, sa, ca]
    sn = np.choose(o, sin_sel)
    cs = np.choose(o, cos_sel)
    return sn, cs


def box_muller(xa: np.ndarray, xb: np.ndarray):
    """Two normals from two 64-bit words: r = sqrt(-2 log(1-u_a)),
    (r cos 2 pi u_b, r sin 2 pi u_b)."""
    u1 = 1.0 - uniform53(xa)
    u2 = uniform53(xb)
    r = np.sqrt(-2.0 * log_fixed(u1))
    sn, cs = sincos_2pi_fixed(u2)
    return r * cs, r * sn


def normals(seed: int, sample: int, n: int) -> np.ndarray:
    """Z[j], j = 0..n-1, for one (seed, global sample index)."""
    nblk = (n + 3) // 4
    x0, x1, x2, x3 = philox4x64_10(np.arange(nblk, dtype=np.uint64), seed, sample)
    za, zb = box_muller(x0, x1)
    zc, zd = box_muller(x2, x3)
    z = np.stack([za, zb, zc, zd], axis=1).reshape(-1)
    return z[:n]


def white_noise(lumped_diag: np.ndarray, seed: int, n_samples: int, sample_offset: int = 0) -> np.ndarray:
    """W[s, j] = sqrt(M_L[j]) * Z(seed, sample_offset + s, j), shape [S, N]."""
    n = lumped_diag.shape[0]
    scale = np.sqrt(lumped_diag)
    W = np.empty((n_samples, n), dtype=np.float64)
    for s in range(n_samples):
        W[s] = scale * normals(seed, sample_offset + s, n)
    return W


# ---- consistent-mass noise (element factors) ----------------------------------


def element_factor_coefficients(h_e: np.ndarray):
    """(a, c) of F_e = [[a, c], [a, -c]] with F_e F_e^T = (h_e/6)[[2,1],[1,2]]."""
    h_e = np.asarray(h_e, dtype=np.float64)
    return np.sqrt(0.25 * h_e), np.sqrt(h_e / 12.0)


def element_normals(seed: int, sample: int, n_elements: int) -> tuple[np.ndarray, np.ndarray]:
    """(p[g], q[g]) for elements g = 0..n_elements-1 of one (seed, global sample)."""
    nblk = (n_elements + 1) // 2
    x0, x1, x2, x3 = philox4x64_10(np.arange(nblk, dtype=np.uint64), seed, sample, ctr1=1)
    pa, qa = box_muller(x0, x1)
    pb, qb = box_muller(x2, x3)
    p = np.stack([pa, pb], axis=1).reshape(-1)[:n_elements]
    q = np.stack([qa, qb], axis=1).reshape(-1)[:n_elements]
    return p, q


def consistent_noise_factor(mesh):
    """R (sparse, N x 2 n_elements) with R R^T = the consistent mass; column 2g
    carries p of element g, column 2g + 1 its q."""
    import scipy.sparse as sp

    a_node, b_node, h = mesh.element_nodes()
    a, c = element_factor_coefficients(h)
    g = np.arange(a_node.shape[0])
    rows = np.concatenate([a_node, a_node, b_node, b_node])
    cols = np.concatenate([2 * g, 2 * g + 1, 2 * g, 2 * g + 1])
    vals = np.concatenate([a, c, a, -c])
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.n_dof, 2 * a_node.shape[0]))


def consistent_white_noise(mesh, seed: int, n_samples: int, sample_offset: int = 0) -> np.ndarray:
    """W[s] = R (p, q) for the element factors R, in the fixed order of the
    definition above, shape [S, N]."""
    E, NI = mesh.n_edges, mesh.n_interior
    n_el = np.asarray(mesh.n_el, dtype=np.int64)
    first = np.asarray(mesh.offsets[:-1], dtype=np.int64) + np.arange(E, dtype=np.int64)  # g of element 0
    a_e, c_e = element_factor_coefficients(mesh.h_e)
    # interior node (e, k), k = 1..m_e: left element first + k - 1, right element first + k
    ie = np.repeat(np.arange(E), n_el - 1)
    ik = np.concatenate([np.arange(1, n) for n in n_el]) if E else np.zeros(0, dtype=np.int64)
    gl, gr = first[ie] + ik - 1, first[ie] + ik
    # vertex ends in increasing edge order, tail before head
    ends = []
    for e in range(E):
        ends.append((int(mesh.edges[e, 0]), e, 0))
        ends.append((int(mesh.edges[e, 1]), e, 1))
    W = np.empty((n_samples, mesh.n_dof), dtype=np.float64)
    n_elements = int(n_el.sum())
    a_g, c_g = a_e[np.repeat(np.arange(E), n_el)], c_e[np.repeat(np.arange(E), n_el)]  # per element
    for s in range(n_samples):
        p, q = element_normals(seed, sample_offset + s, n_elements)
        t_left = a_g * p + c_g * q
        t_right = a_g * p - c_g * q
        W[s, :NI] = t_right[gl] + t_left[gr]
        wv = np.zeros(mesh.n_vertices, dtype=np.float64)
        for v, e, side in ends:
            wv[v] = wv[v] + (t_left[first[e]] if side == 0 else t_right[first[e] + n_el[e] - 1])
        W[s, NI:] = wv
    return W
