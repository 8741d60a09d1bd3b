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
    const double bab = gamma / h;
    const double eps = alpha * h * h / gamma;
    // pass 1: pivots eps_p (kept in fwdt.y as scratch), multipliers rho_p, prod rho_p
    double ep = 1.0 + eps, prod = 1.0, ep_last = 0.0, r_last = 0.0, r_prev = 0.0;
    for (int p = 0; p < m; ++p) {
        const double r = 1.0 / (1.0 + ep);
        rho[at(p)] = r;
        fwdt[at(p)] = make_double2(r_prev, ep);  // .x = rho_{p-1}
        bwdt[at(p)].x = r_prev;
        prod *= r;
        ep_last = ep;
        r_last = r;
        r_prev = r;
        ep = eps + ep * r;
    }
    babs[e * LBp + l] = bab;
    rhom[e * LBp + l] = (m > 0) ? r_last : 0.0;
    sd[(int64_t)l * E + e] = alpha * h * 0.5 + ((m > 0) ? bab * (ep_last * r_last) : bab);
    so[(int64_t)l * E + e] = (m > 0) ? -bab * prod : -bab;
    // pass 2: diagonal and first off-diagonal of T^{-1}, outside-in in pairs
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
