"""Learned vertex preconditioner: the network and its training loss (oracle, FP64).

Test infrastructure only.  This is the plain definition that the GPU kernels
are checked against (forward values, loss and parameter gradients).

The paper's method solves, per shift, the vertex Schur system S u = g
(eq. global_schur) by PCG ("Phase 4").  The learned part is this project's
addition: a message-passing network predicts, for one graph and one shift, a
preconditioner and an initial guess for that system.  Everything is
scale-free: with D = diag(S), the network works on the Jacobi-scaled matrix
D^{-1/2} S D^{-1/2}, and outputs

  P_hat = diag(delta) + sum_e [[p_u^e, q_e], [q_e, p_v^e]]   (SPD by construction:
          delta > 0, p >= 0, q_e = rho_e sqrt(p_u^e p_v^e), |rho_e| < 1)
  Q_hat = diag(gamma) + sum_e [[0, eta_e], [eta_e, 0]]

applied as z = D^{-1/2} P_hat D^{-1/2} r (preconditioner) and
x0 = D^{-1/2} Q_hat D^{-1/2} g (initial guess).  P_hat = I is exactly Jacobi.

Network (vertex features f_v, 8 values):
  log(1 + deg_v), mean / min / max length of the incident edges, log(c_L / c_I) / 10,
  log(kappa) / 3, sum of the incident edge weights w_e, 1;
  w_e = |s_o(e)| / sqrt(D_u D_v)  (the Jacobi-scaled edge coupling).
Three layers  h' = relu(W_s h + W_n m + b),  m_v = sum over edge ends at v of w_e h_u
(8 -> 64 -> 64 -> 64), then the heads
  delta_v = softplus(a_d . h_v + c_d),   gamma_v = a_g . h_v + c_g,
  p_u^e = softplus(a_p1 . h_u + a_p2 . h_v + c_p),  p_v^e = softplus(a_p1 . h_v + a_p2 . h_u + c_p),
  rho_e = 0.95 tanh(a_r . (h_u + h_v) + c_r),        eta_e = a_e . (h_u + h_v) + c_e
for edge e from u (tail) to v (head); a self-loop adds p_u + p_v + 2 q to P_hat_vv
and 2 eta to Q_hat_vv.  Weights (matrices and head vectors) are used rounded to
bfloat16; biases are not.

Loss for a system with solution x* of S x* = g (g_hat = D^{-1/2} g,
x_hat = D^{1/2} x*):
  L = (||P_hat g_hat - x_hat||^2 + ||Q_hat g_hat - x_hat||^2) / ||x_hat||^2,
averaged over the right-hand sides of a batch.

Parity pins (tests/test_oracle_learned.py): the features against values worked
out by hand on a graph with a multi-edge and a self-loop; the autograd gradient
against central finite differences; P_hat SPD for random parameters; the Jacobi
limit; the edge Schur complements against the dense Schur complement of the
assembled system; the reference PCG against plain CG written out step by step
(true-residual stop, zero right-hand side, non-convergence flag) and its
fallback to Jacobi after maxit // 2 iterations.
"""

from __future__ import annotations

import numpy as np

from . import mesh as _mesh
from . import solve as _solve

F_IN = 8
HID = 64
RHO_MAX = 0.95

# parameter vector layout: (name, shape, is_weight)  -- weights are used rounded to bfloat16
LAYOUT = [
    ("W1s", (HID, F_IN), True), ("W1n", (HID, F_IN), True), ("b1", (HID,), False),
    ("W2s", (HID, HID), True), ("W2n", (HID, HID), True), ("b2", (HID,), False),
    ("W3s", (HID, HID), True), ("W3n", (HID, HID), True), ("b3", (HID,), False),
    ("a_d", (HID,), True), ("c_d", (1,), False),
    ("a_g", (HID,), True), ("c_g", (1,), False),
    ("a_p1", (HID,), True), ("a_p2", (HID,), True), ("c_p", (1,), False),
    ("a_r", (HID,), True), ("c_r", (1,), False),
    ("a_e", (HID,), True), ("c_e", (1,), False),
]
N_PARAMS = sum(int(np.prod(s)) for _, s, _ in LAYOUT)


def unpack(theta):
    """Split a flat parameter vector (numpy or torch) into named views."""
    out, o = {}, 0
    for name, shape, _ in LAYOUT:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def effective_params(theta: np.ndarray) -> np.ndarray:
    """The parameters as the network uses them: weights rounded to bfloat16."""
    theta = np.asarray(theta, dtype=np.float32).copy()
    o = 0
    for _, shape, is_w in LAYOUT:
        n = int(np.prod(shape))
        if is_w:
            theta[o:o + n] = bf16_round(theta[o:o + n])
        o += n
    return theta.astype(np.float64)


def edge_schur(m: _mesh.Mesh, kappa_e: np.ndarray, c_I: float, c_L: float):
    """Per-edge 2x2 Schur complement (s_d, s_o) of the shifted system
    ((c_I + c_L kappa_e^2) M_L + c_L G) restricted to one edge (eq. local_reduced_schur):
    s_d = delta - b^2 (T^{-1})_{00}, s_o = -b^2 (T^{-1})_{0,m-1} from the dense inverse
    of the edge's interior block T (m = 0: s_d = delta, s_o = b)."""
    E = m.n_edges
    sd, so = np.zeros(E), np.zeros(E)
    for e in range(E):
        h = m.h_e[e]
        alpha = c_I + c_L * kappa_e[e] ** 2
        a, b = alpha * h + 2.0 * c_L / h, -c_L / h
        delta = alpha * h / 2.0 + c_L / h
        k = m.m(e)
        if k == 0:
            sd[e], so[e] = delta, b
            continue
        T = np.diag(np.full(k, a)) + np.diag(np.full(k - 1, b), 1) + np.diag(np.full(k - 1, b), -1)
        Ti = np.linalg.inv(T)
        sd[e] = delta - b * b * Ti[0, 0]
        so[e] = -b * b * Ti[0, k - 1]
    return sd, so


def schur_matrix(n_vertices: int, edges: np.ndarray, sd: np.ndarray, so: np.ndarray) -> np.ndarray:
    """Dense vertex Schur complement assembled from the edge 2x2 blocks."""
    S = np.zeros((n_vertices, n_vertices))
    for e, (u, v) in enumerate(edges):
        S[u, u] += sd[e]
        S[v, v] += sd[e]
        S[u, v] += so[e]
        S[v, u] += so[e]
    return S


def dense_schur(m: _mesh.Mesh, kappa: float, c_I: float, c_L: float) -> np.ndarray:
    """S = A_VV - A_VI A_II^{-1} A_IV of the assembled lumped system (for pinning edge_schur)."""
    A = _solve.shifted_matrix(m, kappa, c_I, c_L).toarray()
    ni = m.n_interior
    Aii, Aiv, Avv = A[:ni, :ni], A[:ni, ni:], A[ni:, ni:]
    return Avv - Aiv.T @ np.linalg.solve(Aii, Aiv)


def features(m: _mesh.Mesh, edges: np.ndarray, lengths: np.ndarray, sd, so, c_I, c_L, kappa_v):
    """Vertex features (V x 8), edge weights w_e and D = diag(S)."""
    V = m.n_vertices
    S = schur_matrix(V, edges, sd, so)
    D = np.diag(S).copy()
    dh = 1.0 / np.sqrt(D)
    w = np.abs(so) * dh[edges[:, 0]] * dh[edges[:, 1]]
    f = np.zeros((V, F_IN))
    deg = np.zeros(V)
    lsum, lmin, lmax, wsum = np.zeros(V), np.full(V, np.inf), np.full(V, -np.inf), np.zeros(V)
    for e, (u, v) in enumerate(edges):
        for x in (u, v):
            deg[x] += 1
            lsum[x] += lengths[e]
            lmin[x] = min(lmin[x], lengths[e])
            lmax[x] = max(lmax[x], lengths[e])
            wsum[x] += w[e]
    f[:, 0] = np.log1p(deg)
    f[:, 1] = lsum / deg
    f[:, 2] = lmin
    f[:, 3] = lmax
    f[:, 4] = np.log(c_L / c_I) / 10.0
    f[:, 5] = np.log(kappa_v) / 3.0
    f[:, 6] = wsum
    f[:, 7] = 1.0
    return f, w, D


def forward(theta, f, w, edges, V):
    """Network forward in torch (FP64): returns (P_hat, Q_hat) as dense V x V tensors
    and the head values (delta, gamma, p_t, p_h, rho, eta)."""
    import torch

    if not isinstance(theta, torch.Tensor):
        theta = torch.as_tensor(np.asarray(theta, dtype=np.float64))
    P = unpack(theta)
    f = torch.as_tensor(f, dtype=torch.float64)
    w = torch.as_tensor(w, dtype=torch.float64)
    u = torch.as_tensor(edges[:, 0], dtype=torch.long)
    v = torch.as_tensor(edges[:, 1], dtype=torch.long)

    def aggregate(h):
        m = torch.zeros_like(h)
        m = m.index_add(0, u, w[:, None] * h[v])
        m = m.index_add(0, v, w[:, None] * h[u])
        return m

    h = f
    for k in (1, 2, 3):
        mm = aggregate(h)
        h = torch.relu(h @ P[f"W{k}s"].T + mm @ P[f"W{k}n"].T + P[f"b{k}"])
    sp = torch.nn.functional.softplus
    delta = sp(h @ P["a_d"] + P["c_d"])
    gamma = h @ P["a_g"] + P["c_g"]
    hu, hv = h[u], h[v]
    p_t = sp(hu @ P["a_p1"] + hv @ P["a_p2"] + P["c_p"])
    p_h = sp(hv @ P["a_p1"] + hu @ P["a_p2"] + P["c_p"])
    rho = RHO_MAX * torch.tanh((hu + hv) @ P["a_r"] + P["c_r"])
    eta = (hu + hv) @ P["a_e"] + P["c_e"]
    q = rho * torch.sqrt(p_t * p_h)
    Ph = torch.diag(delta)
    Ph = Ph.index_put((u, u), p_t, accumulate=True)
    Ph = Ph.index_put((v, v), p_h, accumulate=True)
    Ph = Ph.index_put((u, v), q, accumulate=True)
    Ph = Ph.index_put((v, u), q, accumulate=True)
    Qh = torch.diag(gamma)
    Qh = Qh.index_put((u, v), eta, accumulate=True)
    Qh = Qh.index_put((v, u), eta, accumulate=True)
    return Ph, Qh, (delta, gamma, p_t, p_h, rho, eta)


def loss(theta, f, w, edges, V, D, G, X):
    """Mean over right-hand sides (rows of G, solutions X of S X^T = G^T) of
    (||P_hat g_hat - x_hat||^2 + ||Q_hat g_hat - x_hat||^2) / ||x_hat||^2."""
    import torch

    Ph, Qh, _ = forward(theta, f, w, edges, V)
    Dt = torch.as_tensor(D, dtype=torch.float64)
    gh = torch.as_tensor(G, dtype=torch.float64) / torch.sqrt(Dt)
    xh = torch.as_tensor(X, dtype=torch.float64) * torch.sqrt(Dt)
    rp = gh @ Ph.T - xh
    rq = gh @ Qh.T - xh
    n2 = (xh * xh).sum(dim=1)
    return (((rp * rp).sum(dim=1) + (rq * rq).sum(dim=1)) / n2).mean()


def loss_and_grad(theta_eff: np.ndarray, f, w, edges, V, D, G, X):
    """Loss and its gradient with respect to the (effective) parameters, FP64 autograd."""
    import torch

    t = torch.tensor(theta_eff, dtype=torch.float64, requires_grad=True)
    L = loss(t, f, w, edges, V, D, G, X)
    L.backward()
    return float(L.detach()), t.grad.detach().numpy().copy()


def preconditioner(theta_eff, f, w, edges, V, D):
    """The dense preconditioner D^{-1/2} P_hat D^{-1/2} and initial-guess operator."""
    Ph, Qh, _ = forward(np.asarray(theta_eff, dtype=np.float64), f, w, edges, V)
    dh = 1.0 / np.sqrt(D)
    P = dh[:, None] * Ph.numpy() * dh[None, :]
    Q = dh[:, None] * Qh.numpy() * dh[None, :]
    return P, Q


def pcg(S, g, P, x0, tol, maxit=10000, fallback=None):
    """Reference PCG on S x = g with preconditioner matrix P from x0.

    Stopping rule (reading A8, paper "Phase 4"): the iteration ends at the
    first iterate whose residual recomputed from x, g - S x, satisfies
    ||g - S x||_2 <= tol ||g||_2; the recursively updated residual is never
    used for the decision.  g = 0 returns x = 0 after 0 iterations.
    Fallback (readings L4 and N2): when ``fallback`` (a matrix, the Jacobi
    preconditioner D^{-1}) is given, once max(1, maxit // 2) iterations have
    been taken with P the iteration restarts from the current iterate with
    the fallback (r = g - S x, z = fallback r, p = z).
    Returns (x, iterations), iterations = maxit + 1 if tol was not reached."""
    gg = float(g @ g)
    if gg == 0.0:
        return np.zeros_like(g), 0
    x = x0.copy()
    M = P
    switch_at = max(1, maxit // 2)

    def start():
        r = g - S @ x
        z = M @ r
        return r, z, z.copy(), float(r @ z)

    r, z, p, rz = start()
    it = 0
    while True:
        rt = g - S @ x
        if float(rt @ rt) <= tol * tol * gg:
            return x, it
        if it == maxit:
            return x, maxit + 1
        if fallback is not None and M is P and it == switch_at:
            M = fallback
            r, z, p, rz = start()
        it += 1
        q = S @ p
        a = rz / float(p @ q)
        x += a * p
        r -= a * q
        z = M @ r
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
