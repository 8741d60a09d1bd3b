// Edge-interior sweeps of the condensed solve: the condensed right-hand side
// (paper: eq. local_reduced_schur, w = A_II^{-1} W_I and its two end values)
// and the interior recovery with quadrature accumulation (paper: eq.
// internal_recovery and "Quadrature Accumulation and Global Assembly").
//
// For one edge and one shift, with the rows of coeff.hip, x = T^{-1} r splits
// into two one-directional recurrences whose results add:
//   forward   y_0 = r_0,      y_p = r_p + rho_{p-1} y_{p-1}      -> x_p += dg_p y_p
//   backward  z_{m-1} = r_{m-1}, z_q = r_q + rho_{m-2-q} z_{q+1} -> x_{q-1} += of_{q-1} z_q
// (y is the Thomas forward elimination, z the same elimination run from the
// other end; x_p = dg_p y_p + of_p z_{p+1} is the twisted-factorisation
// formula).  At loop step k both directions use rho_{k-1}, and of_{m-2-k} =
// of_k by persymmetry, so every table row is read in increasing order.
// The two end values are w_{m-1} = dg_{m-1} y_{m-1}, w_0 = dg_0 z_0, and
// |b| w = rho_{m-1} (y_{m-1} or z_0).
//
// Mapping: one wavefront = one edge x 64 samples (lanes); a block of BL
// shifts is held in registers, so W is read once per BL shifts, and the table
// rows (identical for all samples) are wave-uniform scalar loads.
#include "work.h"

namespace grf {
namespace {

constexpr int PD = 8;  // prefetch depth (steps) for the streamed W and U rows
constexpr int PF = 8;  // distance (steps) of the L2 warm-up of coefficient rows

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Coefficient rows are read with scalar loads, which cannot be issued far
// ahead (the row of one step fills the scalar registers).  A lane-distributed
// vector load of the row PF steps ahead brings it into L2 so that the scalar
// loads hit there; its value only feeds a sink that is never zero-tested away.
template <int BL>
__device__ __forceinline__ double warm_row(const double *row, int lane) {
    return row[lane < BL ? lane : BL - 1];
}

// Condensed right-hand side ends: ends[l][e][side][s] = |b| w_end.
// FWD gives the head end (side 1), !FWD the tail end (side 0).
// occupancy targets: the shift block lives in 2*BL registers per lane
template <int BL>
struct Occ {
    static constexpr int ends = BL >= 64 ? 3 : (BL >= 32 ? 4 : 6);
    static constexpr int acc = BL >= 32 ? 3 : 6;
    static constexpr int pd_acc = BL >= 64 ? 4 : 8;
};

template <int BL, bool FWD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occ<BL>::ends))) k_sweep_ends(const int64_t *__restrict__ off_, const int32_t *__restrict__ m_,
                                                    int32_t E, int64_t N, int32_t nb, int32_t Sp, int32_t LB,
                                                    int32_t LBp, const double *__restrict__ X,
                                                    const double *__restrict__ rho,
                                                    const double *__restrict__ rhom, double *__restrict__ ends) {
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + wave_id();
    if (q >= (int64_t)E * nb) return;
    const int e = (int)(q / nb);
    const int b = (int)(q - (int64_t)e * nb);
    const int l0 = blockIdx.y * BL;
    const int m = m_[e];
    const int64_t off = off_[e];
    const int64_t strideL = (int64_t)E * 2 * Sp;
    double *out = ends + ((int64_t)l0 * E + e) * 2 * Sp + (FWD ? Sp : 0) + (int64_t)b * 64 + lane;
    const int nl = min(BL, LB - l0);
    if (m == 0) {
        for (int j = 0; j < nl; ++j) out[j * strideL] = 0.0;
        return;
    }
    const double *x = X + ((int64_t)b * N + off) * 64 + lane;
    const double *rr = rho + off * LBp + l0;
    // position of loop step k, clamped so that prefetches past the end stay in bounds
    auto xat = [&](int k) -> double {
        const int kc = min(k, m - 1);
        return x[(FWD ? (int64_t)kc : (int64_t)(m - 1 - kc)) * 64];
    };
    auto rowp = [&](int k) -> const double * { return rr + (int64_t)min(k - 1, m - 2) * LBp; };
    double y[BL];
    {
        const double r = xat(0);
#pragma unroll
        for (int j = 0; j < BL; ++j) y[j] = r;
    }
    // W rows PD steps ahead; L2 warm-up of the row PF steps ahead, its value
    // consumed PD steps after issue together with the W row of the same step
    // (vector-memory waits are in order, so an early use would drain the queue)
    double bw[PD], bp[PD];
    double sink = 0.0;
#pragma unroll
    for (int i = 0; i < PD; ++i) {
        bw[i] = xat(1 + i);
        bp[i] = warm_row<BL>(rowp(1 + i + PF), lane);
    }
    // main loop: whole chunks of PD steps, no per-step branch, so the
    // rotating buffers stay in fixed registers and the waits stay in order
    int k0 = 1;
#pragma unroll 1
    for (; k0 + PD <= m; k0 += PD) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
            const int k = k0 + i;
            const double r = bw[i];
            sink += bp[i];
            bw[i] = xat(k + PD);
            bp[i] = warm_row<BL>(rowp(k + PD + PF), lane);
            const double *row = rr + (int64_t)(k - 1) * LBp;
#pragma unroll
            for (int j = 0; j < BL; ++j) y[j] = fma(row[j], y[j], r);
        }
    }
    // tail: fewer than PD steps, values already in the buffer
#pragma unroll
    for (int i = 0; i < PD; ++i) {
        const int k = k0 + i;
        if (k < m) {
            const double r = bw[i];
            const double *row = rr + (int64_t)(k - 1) * LBp;
#pragma unroll
            for (int j = 0; j < BL; ++j) y[j] = fma(row[j], y[j], r);
        }
    }
    const double *rm = rhom + (int64_t)e * LBp + l0;
#pragma unroll
    for (int j = 0; j < BL; ++j)
        if (j < nl) out[j * strideL] = rm[j] * y[j];
    if (sink != sink) out[0] = sink;  // keeps the warm-up loads alive; never true for finite rows
}

// Interior recovery and accumulation, all shift sub-blocks of the pass in
// order (one wavefront owns its edge's accumulator rows, so no atomics).
// r = W_I - b (u_tail e_0 + u_head e_{m-1}) = W_I + |b| (...).
// FWD: step k (0..m-1) reads W and updates U at position k with row
//      fwdt[k] = (rho_{k-1}, dg_k); positions 0 and m-1 carry the tail and
//      head corrections.
// BWD: step k (0..m-2) reads W at m-1-k and updates U at m-2-k with row
//      bwdt[k] = (rho_{k-1}, of_k); position m-1 (step 0) carries the head
//      correction, the tail position never enters the backward part.
template <int BL, bool FWD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occ<BL>::acc))) k_sweep_acc(
    const int64_t *__restrict__ off_, const int32_t *__restrict__ m_, const int32_t *__restrict__ eu_,
    const int32_t *__restrict__ ev_, int32_t E, int32_t V, int64_t N, int32_t nb, int32_t Sp, int32_t LB,
    int32_t LBp, const double *__restrict__ X, double *__restrict__ U, const double2 *__restrict__ tab,
    const double *__restrict__ babs, const double *__restrict__ ug) {
    constexpr int PDA = Occ<BL>::pd_acc;
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + wave_id();
    if (q >= (int64_t)E * nb) return;
    const int e = (int)(q / nb);
    const int b = (int)(q - (int64_t)e * nb);
    const int m = m_[e];
    if (m == 0 || (!FWD && m == 1)) return;
    const int64_t off = off_[e];
    const double *x = X + ((int64_t)b * N + off) * 64 + lane;
    double *u = U + ((int64_t)b * N + off) * 64 + lane;
    const int64_t sidx = (int64_t)b * 64 + lane;
    const int64_t VSp = (int64_t)V * Sp;
    const double *ug_t = ug + (int64_t)eu_[e] * Sp + sidx;  // tail vertex, shift l at + l * VSp
    const double *ug_h = ug + (int64_t)ev_[e] * Sp + sidx;  // head vertex
    const int kin = m - 1;  // streamed steps 1 .. kin-1
    auto wpos = [&](int k) -> int64_t { return FWD ? (int64_t)min(k, m - 1) : (int64_t)(m - 1 - min(k, m - 1)); };
    auto upos = [&](int k) -> int64_t { return FWD ? (int64_t)min(k, m - 1) : (int64_t)(m - 2 - min(k, m - 2)); };
    double sink = 0.0;
#pragma unroll 1
    for (int l0 = 0; l0 < LB; l0 += BL) {
        const double2 *tr = tab + off * LBp + l0;
        const double *bb = babs + (int64_t)e * LBp + l0;
        auto trow = [&](int k) -> const double2 * { return tr + (int64_t)min(k, m - 1) * LBp; };
        double y[BL];
        double bw[PDA], bu[PDA], bp[PDA];
        const double r0 = x[wpos(0) * 64];
        const double u0 = u[upos(0) * 64];
#pragma unroll
        for (int i = 0; i < PDA; ++i) {
            bw[i] = x[wpos(1 + i) * 64];
            bu[i] = u[upos(1 + i) * 64];
            const double2 w2 = trow(1 + i + PF)[lane < BL / 2 ? lane : BL / 2 - 1];
            bp[i] = w2.x + w2.y;
        }
        // step 0: first position with its end correction(s)
        {
            const double *c0 = FWD ? ug_t : ug_h;
#pragma unroll
            for (int j = 0; j < BL; ++j) y[j] = fma(bb[j], c0[(int64_t)min(l0 + j, LB - 1) * VSp], r0);
            if (FWD && m == 1) {
#pragma unroll
                for (int j = 0; j < BL; ++j) y[j] = fma(bb[j], ug_h[(int64_t)min(l0 + j, LB - 1) * VSp], y[j]);
            }
            double a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int j = 0; j < BL; ++j) {
                if (j & 1) a1 = fma(tr[j].y, y[j], a1); else a0 = fma(tr[j].y, y[j], a0);
            }
            u[upos(0) * 64] = u0 + (a0 + a1);
        }
        // streamed steps 1 .. kin-1: whole chunks of PDA steps without branches, then a tail
        auto step = [&](int k, double r, double uk) {
            const double2 *row = tr + (int64_t)k * LBp;
            double b0 = 0.0, b1 = 0.0;
#pragma unroll
            for (int j = 0; j < BL; ++j) {
                const double2 c = row[j];
                y[j] = fma(c.x, y[j], r);
                if (j & 1) b1 = fma(c.y, y[j], b1); else b0 = fma(c.y, y[j], b0);
            }
            u[upos(k) * 64] = uk + (b0 + b1);
        };
        int k0 = 1;
#pragma unroll 1
        for (; k0 + PDA <= kin; k0 += PDA) {
#pragma unroll
            for (int i = 0; i < PDA; ++i) {
                const int k = k0 + i;
                const double r = bw[i];
                const double uk = bu[i];
                sink += bp[i];
                bw[i] = x[wpos(k + PDA) * 64];
                bu[i] = u[upos(k + PDA) * 64];
                const double2 w2 = trow(k + PDA + PF)[lane < BL / 2 ? lane : BL / 2 - 1];
                bp[i] = w2.x + w2.y;
                step(k, r, uk);
            }
        }
#pragma unroll
        for (int i = 0; i < PDA; ++i)
            if (k0 + i < kin) step(k0 + i, bw[i], bu[i]);
        // FWD: last position m-1 (m >= 2) carries the head correction
        if (FWD && m >= 2) {
            const int k = m - 1;
            const double r = x[(int64_t)k * 64];
            const double uk = u[(int64_t)k * 64];
            const double2 *row = tr + (int64_t)k * LBp;
            double b0 = 0.0, b1 = 0.0;
#pragma unroll
            for (int j = 0; j < BL; ++j) {
                const double2 c = row[j];
                y[j] = fma(bb[j], ug_h[(int64_t)min(l0 + j, LB - 1) * VSp], fma(c.x, y[j], r));
                if (j & 1) b1 = fma(c.y, y[j], b1); else b0 = fma(c.y, y[j], b0);
            }
            u[(int64_t)k * 64] = uk + (b0 + b1);
        }
    }
    // keeps the L2 warm-up loads alive; sink is finite (coefficients are finite), so this never stores
    if (sink != sink) u[0] = sink;
}

template <int BL>
void ends_bl(const MeshView &mv, const SweepArgs &a, bool fwd, hipStream_t st) {
    const int64_t waves = (int64_t)mv.E * a.nb;
    dim3 grid((unsigned)((waves + 3) / 4), (unsigned)((a.LB + BL - 1) / BL));
    if (fwd)
        hipLaunchKernelGGL((k_sweep_ends<BL, true>), grid, dim3(256), 0, st, mv.off, mv.m, mv.E, mv.N, a.nb, a.Sp,
                           a.LB, a.LBp, a.X, a.rho, a.rhom, a.ends);
    else
        hipLaunchKernelGGL((k_sweep_ends<BL, false>), grid, dim3(256), 0, st, mv.off, mv.m, mv.E, mv.N, a.nb, a.Sp,
                           a.LB, a.LBp, a.X, a.rho, a.rhom, a.ends);
    GRF_LAUNCH_CHECK();
}

template <int BL>
void acc_bl(const MeshView &mv, const SweepArgs &a, bool fwd, hipStream_t st) {
    const int64_t waves = (int64_t)mv.E * a.nb;
    dim3 grid((unsigned)((waves + 3) / 4));
    if (fwd)
        hipLaunchKernelGGL((k_sweep_acc<BL, true>), grid, dim3(256), 0, st, mv.off, mv.m, mv.eu, mv.ev, mv.E, mv.V,
                           mv.N, a.nb, a.Sp, a.LB, a.LBp, a.X, a.U, a.fwdt, a.babs, a.ug);
    else
        hipLaunchKernelGGL((k_sweep_acc<BL, false>), grid, dim3(256), 0, st, mv.off, mv.m, mv.eu, mv.ev, mv.E, mv.V,
                           mv.N, a.nb, a.Sp, a.LB, a.LBp, a.X, a.U, a.bwdt, a.babs, a.ug);
    GRF_LAUNCH_CHECK();
}

}  // namespace

void launch_sweep_ends(const MeshView &mv, const SweepArgs &a, bool fwd, hipStream_t st) {
    if (mv.E == 0 || a.LB == 0) return;
    GRF_REQUIRE(a.LBp % a.bl == 0, "internal: shift padding");
    switch (a.bl) {
        case 8: ends_bl<8>(mv, a, fwd, st); break;
        case 16: ends_bl<16>(mv, a, fwd, st); break;
        case 32: ends_bl<32>(mv, a, fwd, st); break;
        case 64: ends_bl<64>(mv, a, fwd, st); break;
        default: GRF_REQUIRE(false, "sweep_block must be 8, 16, 32 or 64");
    }
}

void launch_sweep_acc(const MeshView &mv, const SweepArgs &a, bool fwd, hipStream_t st) {
    if (mv.E == 0 || a.LB == 0) return;
    GRF_REQUIRE(a.LBp % a.bl == 0, "internal: shift padding");
    switch (a.bl) {
        case 8: acc_bl<8>(mv, a, fwd, st); break;
        case 16: acc_bl<16>(mv, a, fwd, st); break;
        case 32: acc_bl<32>(mv, a, fwd, st); break;
        case 64: acc_bl<64>(mv, a, fwd, st); break;
        default: GRF_REQUIRE(false, "sweep_block must be 8, 16, 32 or 64");
    }
}

}  // namespace grf
