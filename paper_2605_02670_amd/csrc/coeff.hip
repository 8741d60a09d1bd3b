// Per-(shift, edge) coefficients of the condensed solve, recurrence form
// (used by the streamed sweeps).
//
// Paper: eq. local_operator / eq. spde_local_quadrature_block (the local
// operator of edge e for shift l), the tridiagonal storage of A_II and the
// Thomas factorisation eq. thomas_coefficients, and eq. local_reduced_schur
// (the edge's 2x2 Schur complement S^(l,e) and its condensed right-hand side).
//
// With alpha = c_I + c_L kappa^2, gamma = c_L and the lumped mass, the
// interior block of an edge with m interior nodes is the constant-coefficient
// tridiagonal T = tridiag(b, a, b), a = alpha h + 2 gamma / h, b = -gamma / h,
// and each edge end adds delta = alpha h / 2 + gamma / h to its vertex.
// Write tau = a / |b| = 2 + eps, eps = alpha h^2 / gamma.  The Thomas pivots
// of T / |b| are pi_p = 1 + eps_p with
//     eps_0 = 1 + eps,   eps_p = eps + eps_{p-1} / (1 + eps_{p-1}),
// a form with no cancellation however close tau is to 2.  The kernel stores,
// per interior position p = 0..m-1 (shift-fastest rows, [DOF][shift]),
// rho_p = 1 / pi_p (forward/backward multiplier) and the step rows of the two
// streamed recovery sweeps,
//   fwdt[k] = (rho_{k-1}, dg_k),  bwdt[k] = (rho_{k-1}, of_k),
// with dg_p = (T^{-1})_{pp} = 1 / (|b| (eps_p + eps_{m-1-p} - eps)) and
// of_p = (T^{-1})_{p,p+1} = dg_p rho_{m-2-p} (the inverse of a symmetric
// tridiagonal matrix is semiseparable; the diagonal follows from the twisted
// factorisation, which adds the pivots from both ends; T is persymmetric, so
// the backward pivots are the forward ones reversed).  Per edge: |b|,
// rho_{m-1}, and the Schur complement
//   s_d = delta - b^2 (T^{-1})_{11} = alpha h / 2 + |b| eps_{m-1} / (1 + eps_{m-1})
//   s_o = -b^2 (T^{-1})_{1m}        = -|b| prod_p rho_p
// (an edge with no interior node has s_d = delta, s_o = b).
//
// Consistent mass in the system (GRF_MASS_CONSISTENT_SYS; paper Phase 2,
// consistent entries): a = 2 alpha h / 3 + 2 gamma / h, b = alpha h / 6 -
// gamma / h and delta = alpha h / 3 + gamma / h, so b takes either sign across
// the shifts.  With sigma = -sign(b) and D = diag(sigma^p), T = D T' D where
// T' = |b| tridiag(-1, tau, -1) has the form above, tau - 2 = eps = (a - 2|b|)
// / |b| (alpha h / |b| when b < 0, (alpha h / 3 + 4 gamma / h) / |b| when
// b > 0, both free of cancellation).  Hence (T^{-1})_{pq} = sigma^{p+q}
// (T'^{-1})_{pq}: the multipliers rho and the off-diagonal of T^{-1} carry the
// factor sigma, the diagonal does not, the end values and the recovery use
// -b = sigma |b| where the lumped form has |b|, and
//   s_d = (delta - |b|) + |b| eps_{m-1} / (1 + eps_{m-1}),
//   s_o = -|b| sigma^{m-1} prod_p rho_p   (b for an edge with no interior node),
// with delta - |b| = alpha h / 2 (b < 0) or alpha h / 6 + 2 gamma / h (b > 0).
// b = 0 makes T = a I (no coupling to the vertices).  Lumped: sigma = 1.
#include <algorithm>

#include "work.h"

namespace grf {
namespace {

__global__ void __launch_bounds__(64) k_coeff(MeshView mv, const double *__restrict__ shift, int32_t LB, int32_t LBp,
                                              double *__restrict__ rho, double2 *__restrict__ fwdt,
                                              double2 *__restrict__ bwdt, double *__restrict__ babs,
                                              double *__restrict__ rhom, double *__restrict__ sd,
                                              double *__restrict__ so) {
    const int e = blockIdx.x;
    const int l = blockIdx.y * 64 + threadIdx.x;
    if (l >= LBp) return;
    const int m = mv.m[e];
    const int64_t off = mv.off[e];
    const int64_t E = mv.E;
    auto at = [&](int p) -> int64_t { return (off + p) * LBp + l; };
    if (l >= LB) {  // padding shifts contribute nothing
        for (int p = 0; p < m; ++p) {
            rho[at(p)] = 0.0;
            fwdt[at(p)] = make_double2(0.0, 0.0);
            bwdt[at(p)] = make_double2(0.0, 0.0);
        }
        babs[e * LBp + l] = 0.0;
        rhom[e * LBp + l] = 0.0;
        sd[(int64_t)l * E + e] = 1.0;
        so[(int64_t)l * E + e] = 0.0;
        return;
    }
    const double h = mv.he[e];
    const double alpha = shift[2 * l] + shift[2 * l + 1] * mv.kap2[e];
    const double gamma = shift[2 * l + 1];
    double bab, eps, c0, sg;  // |b|, tau - 2, delta - |b|, sigma = -sign(b)
    if (!mv.consistent) {
        bab = gamma / h;
        eps = alpha * h * h / gamma;
        c0 = alpha * h * 0.5;
        sg = 1.0;
    } else {
        const double b = alpha * h / 6.0 - gamma / h;
        if (b == 0.0) {  // T = a I: no multipliers, no coupling to the vertices
            const double dg = 1.0 / (2.0 * alpha * h / 3.0 + 2.0 * gamma / h);
            for (int p = 0; p < m; ++p) {
                rho[at(p)] = 0.0;
                fwdt[at(p)] = make_double2(0.0, dg);
                bwdt[at(p)] = make_double2(0.0, 0.0);
            }
            babs[e * LBp + l] = 0.0;
            rhom[e * LBp + l] = 0.0;
            sd[(int64_t)l * E + e] = alpha * h / 3.0 + gamma / h;
            so[(int64_t)l * E + e] = 0.0;
            return;
        }
        if (b < 0.0) {
            bab = -b;
            eps = alpha * h / bab;
            c0 = alpha * h * 0.5;
            sg = 1.0;
        } else {
            bab = b;
            eps = (alpha * h / 3.0 + 4.0 * gamma / h) / bab;
            c0 = alpha * h / 6.0 + 2.0 * gamma / h;
            sg = -1.0;
        }
    }
    // pass 1: pivots eps_p (kept in fwdt.y as scratch), multipliers sigma rho_p, prod rho_p
    double ep = 1.0 + eps, prod = 1.0, ep_last = 0.0, r_last = 0.0, r_prev = 0.0;
    for (int p = 0; p < m; ++p) {
        const double r = 1.0 / (1.0 + ep);
        rho[at(p)] = sg * r;
        fwdt[at(p)] = make_double2(sg * r_prev, ep);  // .x = sigma rho_{p-1}
        bwdt[at(p)].x = sg * r_prev;
        prod *= r;
        ep_last = ep;
        r_last = r;
        r_prev = r;
        ep = eps + ep * r;
    }
    babs[e * LBp + l] = sg * bab;
    rhom[e * LBp + l] = (m > 0) ? sg * r_last : 0.0;
    sd[(int64_t)l * E + e] = c0 + ((m > 0) ? bab * (ep_last * r_last) : bab);
    const double par = (sg < 0.0 && (m & 1) == 0) ? -1.0 : 1.0;  // sigma^{m-1}
    so[(int64_t)l * E + e] = (m > 0) ? -bab * prod * par : -sg * bab;
    // pass 2: diagonal and first off-diagonal of T^{-1}, outside-in in pairs
    // (rho holds sigma rho_p, so the off-diagonal carries its sigma)
    for (int p = 0; 2 * p < m; ++p) {
        const int q = m - 1 - p;
        const double ep_p = fwdt[at(p)].y;
        const double ep_q = fwdt[at(q)].y;
        const double d = 1.0 / (bab * (ep_p + ep_q - eps));
        fwdt[at(p)].y = d;
        fwdt[at(q)].y = d;
        if (p <= m - 2) bwdt[at(p)].y = d * rho[at(m - 2 - p)];
        if (q != p && q <= m - 2) bwdt[at(q)].y = d * rho[at(m - 2 - q)];
    }
    if (m > 0) bwdt[at(m - 1)].y = 0.0;
}

}  // namespace

void launch_coeff(const MeshView &mv, const CoeffArgs &a, hipStream_t st) {
    if (mv.E == 0) return;
    GRF_REQUIRE(a.LBp % 8 == 0 && a.LBp >= a.LB, "internal: bad padded shift count");
    GRF_REQUIRE(a.rho && a.fwdt && a.bwdt, "internal: streamed coefficient rows missing");
    hipLaunchKernelGGL(k_coeff, dim3((unsigned)mv.E, (unsigned)((a.LBp + 63) / 64)), dim3(64), 0, st, mv, a.shift,
                       a.LB, a.LBp, a.rho, a.fwdt, a.bwdt, a.babs, a.rhom, a.sd, a.so);
    GRF_LAUNCH_CHECK();
}

}  // namespace grf
