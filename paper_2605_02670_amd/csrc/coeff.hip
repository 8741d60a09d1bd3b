// Per-(shift, edge) coefficients of the condensed solve.
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
// per interior position p = 0..m-1 (shift-fastest rows, [DOF][shift]):
//   rho_p = 1 / pi_p                       (forward/backward multiplier)
//   dg_p  = (T^{-1})_{pp} = 1 / (|b| (eps_p + eps_{m-1-p} - eps))
//   of_p  = (T^{-1})_{p,p+1} = dg_p * rho_{m-2-p}
// as rho[p] and either the step rows of the two streamed recovery sweeps,
//   fwdt[k] = (rho_{k-1}, dg_k),  bwdt[k] = (rho_{k-1}, of_k),
// or the plain rows dg[p], of[p] and zt[p] = (T^{-1})_{p,0} = dg_p prod_{k<p} rho_k
// that blocked.hip turns into matrix-core operand tables,
// (the inverse of a symmetric tridiagonal matrix is semiseparable; the
// diagonal follows from the twisted factorisation, which adds the pivots from
// both ends; T is persymmetric, so the backward pivots are the forward ones
// reversed).  Per edge: |b|, rho_{m-1}, and the Schur complement
//   s_d = delta - b^2 (T^{-1})_{11} = alpha h / 2 + |b| eps_{m-1} / (1 + eps_{m-1})
//   s_o = -b^2 (T^{-1})_{1m}        = -|b| prod_p rho_p
// (an edge with no interior node has s_d = delta, s_o = b).
#include <algorithm>

#include "work.h"

namespace grf {
namespace {

__global__ void __launch_bounds__(64) k_coeff(MeshView mv, const double *__restrict__ shift, int32_t LB, int32_t LBp,
                                              double *__restrict__ rho, double2 *__restrict__ fwdt,
                                              double2 *__restrict__ bwdt, double *__restrict__ dgp,
                                              double *__restrict__ ofp, double *__restrict__ ztp,
                                              double *__restrict__ epsp,
                                              double *__restrict__ babs, double *__restrict__ rhom,
                                              double *__restrict__ sd, double *__restrict__ so) {
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
            if (fwdt) {
                fwdt[at(p)] = make_double2(0.0, 0.0);
                bwdt[at(p)] = make_double2(0.0, 0.0);
            }
            if (dgp) {
                dgp[at(p)] = 0.0;
                ofp[at(p)] = 0.0;
                ztp[at(p)] = 0.0;
            }
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
    // pass 1: pivots eps_p (kept in the dg row as scratch), multipliers rho_p,
    // prefix products prod_{k<p} rho_k (kept in the zt row as scratch)
    double *dgs = dgp ? dgp : nullptr;
    double ep = 1.0 + eps, prod = 1.0, ep_last = 0.0, r_last = 0.0, r_prev = 0.0;
    for (int p = 0; p < m; ++p) {
        const double r = 1.0 / (1.0 + ep);
        rho[at(p)] = r;
        if (fwdt) {
            fwdt[at(p)] = make_double2(r_prev, ep);  // .x = rho_{p-1}
            bwdt[at(p)].x = r_prev;
        }
        if (dgs) {
            epsp[at(p)] = ep;
            ztp[at(p)] = prod;
        }
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
    if (dgs) return;  // the blocked path finishes the rows in k_coeff_finish (parallel over positions)
    // pass 2: diagonal and first off-diagonal of T^{-1}, outside-in in pairs
    for (int p = 0; 2 * p < m; ++p) {
        const int q = m - 1 - p;
        const double ep_p = dgs ? dgs[at(p)] : fwdt[at(p)].y;
        const double ep_q = dgs ? dgs[at(q)] : fwdt[at(q)].y;
        const double d = 1.0 / (bab * (ep_p + ep_q - eps));
        const double ofpv = (p <= m - 2) ? d * rho[at(m - 2 - p)] : 0.0;
        const double ofqv = (q <= m - 2) ? d * rho[at(m - 2 - q)] : 0.0;
        if (fwdt) {
            fwdt[at(p)].y = d;
            fwdt[at(q)].y = d;
            if (p <= m - 2) bwdt[at(p)].y = ofpv;
            if (q != p && q <= m - 2) bwdt[at(q)].y = ofqv;
        }
        if (dgs) {
            dgs[at(p)] = d;
            dgs[at(q)] = d;
            ofp[at(p)] = ofpv;
            ofp[at(q)] = ofqv;
            ztp[at(p)] *= d;
            if (q != p) ztp[at(q)] *= d;
        }
    }
    if (m > 0) {
        if (fwdt) bwdt[at(m - 1)].y = 0.0;
        if (dgs) ofp[at(m - 1)] = 0.0;
    }
}

// Finish the plain rows, one thread per (interior DOF, shift): with eps_p in
// the eps scratch and prod_{k<p} rho_k in the prefix scratch from the
// sequential pass,
//   dg_p = 1 / (|b| (eps_p + eps_{m-1-p} - eps)),  of_p = dg_p rho_{m-2-p},
//   (T^{-1})_{p,0} = dg_p prod_{k<p} rho_k.
// eps_p >= eps, so eps_p + eps_{m-1-p} - eps >= eps_{m-1-p} > 0 (no cancellation).
__global__ void __launch_bounds__(256) k_coeff_finish(MeshView mv, const int32_t *__restrict__ dof_edge,
                                                      const double *__restrict__ shift, int32_t LB, int32_t LBp,
                                                      const double *__restrict__ rho, const double *__restrict__ eps_in,
                                                      double *__restrict__ dg, double *__restrict__ of,
                                                      const double *__restrict__ prefix,
                                                      const int32_t *__restrict__ boff, int32_t NT,
                                                      double *__restrict__ ztab) {
    const int64_t n = mv.NI * LBp;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pos = idx / LBp;
        const int l = (int)(idx - pos * LBp);
        const int e = dof_edge[pos];
        const int64_t off = mv.off[e];
        const int m = mv.m[e];
        const int p = (int)(pos - off);
        double z = 0.0;  // padding shifts: zero operands (their dg/of rows were zeroed by k_coeff)
        if (l < LB) {
            const double h = mv.he[e];
            const double alpha = shift[2 * l] + shift[2 * l + 1] * mv.kap2[e];
            const double gamma = shift[2 * l + 1];
            const double bab = gamma / h;
            const double eps = alpha * h * h / gamma;
            const double ep = eps_in[idx];
            const double eq = eps_in[(off + (m - 1 - p)) * LBp + l];
            const double d = 1.0 / (bab * (ep + eq - eps));
            of[idx] = (p <= m - 2) ? d * rho[(off + (m - 2 - p)) * LBp + l] : 0.0;
            dg[idx] = d;
            z = d * prefix[idx];
        }
        // z = (T^{-1})_{p,0} = dg_p prod_{k<p} rho_k, stored in the pass-B operand
        // layout of the block of p (row p%16, shift slot 16t + 4r + k <-> lane row + 16k),
        // and, by persymmetry, as (T^{-1})_{m-1-p, m-1} in the block of m-1-p
        const int t = l >> 4, r = (l & 15) >> 2, k = l & 3;
        const int64_t base_t = (boff[e] + (p >> 4)) * (int64_t)(512 * NT);
        ztab[base_t + ((int64_t)t * 4 + r) * 64 + (p & 15) + 16 * k] = z;
        const int ph = m - 1 - p;
        const int64_t base_h = (boff[e] + (ph >> 4)) * (int64_t)(512 * NT) + 256 * NT;
        ztab[base_h + ((int64_t)t * 4 + r) * 64 + (ph & 15) + 16 * k] = z;
    }
}

}  // namespace

void launch_coeff(const MeshView &mv, const CoeffArgs &a, hipStream_t st) {
    if (mv.E == 0) return;
    GRF_REQUIRE(a.LBp % 8 == 0 && a.LBp >= a.LB, "internal: bad padded shift count");
    hipLaunchKernelGGL(k_coeff, dim3((unsigned)mv.E, (unsigned)((a.LBp + 63) / 64)), dim3(64), 0, st, mv, a.shift,
                       a.LB, a.LBp, a.rho, a.fwdt, a.bwdt, a.dg, a.of, a.zt, a.eps, a.babs, a.rhom, a.sd, a.so);
    GRF_LAUNCH_CHECK();
    if (a.dg) {
        GRF_REQUIRE(a.eps && a.dof_edge && a.boff && a.ztab && a.LBp == 16 * a.NT,
                    "internal: blocked rows need the eps scratch, the DOF-edge map and the block layout");
        const int64_t n = mv.NI * (int64_t)a.LBp;
        const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
        if (n > 0) {
            hipLaunchKernelGGL(k_coeff_finish, dim3((unsigned)blocks), dim3(256), 0, st, mv, a.dof_edge, a.shift, a.LB,
                               a.LBp, a.rho, a.eps, a.dg, a.of, a.zt, a.boff, a.NT, a.ztab);
            GRF_LAUNCH_CHECK();
        }
    }
}

}  // namespace grf
