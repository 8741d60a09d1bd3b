// Blocked edge sweeps on the matrix cores (FP64 MFMA 16x16x4).
//
// The Thomas forward elimination of every edge (paper: eq. thomas_coefficients
// and the forward/backward substitutions of "Boundary Condition and Initial
// Offset"; the interior recovery eq. internal_recovery) is run over blocks of
// 16 interior positions.  With y_p = r_p + rho_{p-1} y_{p-1} (the elimination of
// coeff.hip), for block beta (positions 16 beta + i, i = 0..15)
//     y_{16b+i} = sum_{j<=i} Lam[i][j] r_{16b+j} + lam[i] y_{16b-1},
//     Lam[i][j] = prod_{k=16b+j}^{16b+i-1} rho_k,  lam[i] = prod_{k=16b-1}^{16b+i-1} rho_k,
// so that, for all shifts l and 16 samples at once,
//     F_blk  = Ghat R + H Y_prev          (16 positions x 16 samples)
//     Y_next = d .* Y_prev + C R          (16 NT shifts x 16 samples)
// with the sample-independent block operands
//     Ghat[i][j] = sum_l g^l_i Lam^l[i][j],   H[i][l] = g^l_i lam^l[i],
//     C[l][j] = Lam^l[i*][j],   d[l] = lam^l[i*]   (i* = last position of the block),
// g = dg for the forward part of x = T^{-1} r and g = of for the backward part,
// which is the same elimination on the reversed edge (T is persymmetric, so
// the reversed elimination uses the same multipliers).  These are dense
// contractions over positions and over shifts: the matrix cores do the
// broadcast of the shift-dependent coefficients across the sample lanes.
//
// Pass A (before the vertex solve) runs both directions on W alone; it writes
// the W part of u_I = sum_l T_l^{-1} W into the accumulator and, from the final
// carries, the two end values |b| w of every edge (the condensed right-hand
// side, eq. local_reduced_schur).  Pass B (after it) adds the end corrections
// of eq. internal_recovery by linearity:
//     u_I += sum_l |b_l| (u_tail^l (T_l^{-1})_{.,0} + u_head^l (T_l^{-1})_{.,m-1}),
// a GEMM against the first/last columns of T_l^{-1}.
//
// Operand layout of v_mfma_f64_16x16x4f64 (verified on gfx950): lane L holds
// A[L%16][L/16], B[L/16][L%16], and D[4r + L/16][L%16] in accumulator item r.
// A D-layout register r of shift tile t is used directly as a B operand with
// K-slot k <-> shift 16t + 4r + k, so the carried state never changes layout;
// the tables store H, Z in that shift order.
#include "work.h"

namespace grf {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// table section offsets (doubles) within one block's table
struct TabLayout {
    int NT;
    __host__ __device__ int64_t CT() const { return 0; }                  // [t][c][64]: C[16t + L%16][4c + L/16]
    __host__ __device__ int64_t DT() const { return 256 * NT; }           // [t][r][64]: d[16t + 4r + L/16]
    __host__ __device__ int64_t HF() const { return 512 * NT; }           // [t][r][64]: H_fwd[L%16][16t + 4r + L/16]
    __host__ __device__ int64_t HB() const { return 768 * NT; }           // [t][r][64]: H_bwd[...]
    __host__ __device__ int64_t GF() const { return 1024 * NT; }          // [c][64]: Ghat_fwd[L%16][4c + L/16]
    __host__ __device__ int64_t GB() const { return 1024 * NT + 256; }    // [c][64]: Ghat_bwd
    __host__ __device__ int64_t size() const { return 1024 * (int64_t)NT + 512; }
};

__device__ __forceinline__ int find_edge(const int32_t *boff, int E, int64_t blk) {
    int lo = 0, hi = E;  // boff[lo] <= blk < boff[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (boff[mid] <= blk) lo = mid; else hi = mid;
    }
    return lo;
}

// One workgroup per edge block: stage the block's rows in LDS, then
//   phase 1 (thread = shift): C, d, H_fwd, H_bwd,
//   phase 2 (thread = (i, j)): Ghat_fwd, Ghat_bwd, summed over shifts in order.
__global__ void __launch_bounds__(256) k_blocktab(const int64_t *__restrict__ off_, const int32_t *__restrict__ m_,
                                                  const int32_t *__restrict__ boff, int32_t E, int32_t LBp, int32_t NT,
                                                  const double *__restrict__ rho, const double *__restrict__ dg,
                                                  const double *__restrict__ of, double *__restrict__ tab) {
    extern __shared__ double sm[];
    double *srho = sm;               // [17][LBp]: rho_{16b-1 .. 16b+15}
    double *sdg = sm + 17 * LBp;     // [16][LBp]
    double *sof = sdg + 16 * LBp;    // [16][LBp]
    const int64_t blk = blockIdx.x;
    const int e = find_edge(boff, E, blk);
    const int beta = (int)(blk - boff[e]);
    const int m = m_[e];
    const int64_t off = off_[e];
    const int base = 16 * beta;
    const int istar = min(15, m - 1 - base);
    for (int idx = threadIdx.x; idx < 49 * LBp; idx += blockDim.x) {
        const int row = idx / LBp, l = idx - row * LBp;
        double v = 0.0;
        if (row < 17) {
            const int p = base - 1 + row;
            if (p >= 0 && p < m) v = rho[(off + p) * LBp + l];
        } else {
            const int rr = row < 33 ? row - 17 : row - 33;
            const int p = base + rr;
            if (p < m) v = (row < 33 ? dg : of)[(off + p) * LBp + l];
        }
        sm[idx] = v;
    }
    __syncthreads();
    const TabLayout TL{NT};
    double *T = tab + blk * TL.size();
    auto r_at = [&](int k, int l) -> double { return srho[(k - base + 1) * LBp + l]; };  // rho_k, k in [base-1, base+15]
    if ((int)threadIdx.x < LBp) {
        const int l = threadIdx.x;
        const int t = l >> 4, r = (l & 15) >> 2, kk = l & 3;
        // C[l][j] = prod_{k=base+j}^{base+istar-1} rho_k for j <= istar
        double c = 1.0;
        for (int j = 15; j >= 0; --j) {
            double v = 0.0;
            if (j <= istar) {
                if (j < istar) c *= r_at(base + j, l);
                v = c;
            }
            T[TL.CT() + ((int64_t)t * 4 + (j >> 2)) * 64 + (l & 15) + 16 * (j & 3)] = v;
        }
        // lam[i] = prod_{k=base-1}^{base+i-1} rho_k (no carry into the first block)
        double lam = beta > 0 ? r_at(base - 1, l) : 0.0;
        double dv = 0.0;
        for (int i = 0; i < 16; ++i) {
            const double li = (i <= istar) ? lam : 0.0;
            if (i == istar) dv = li;
            const int64_t o = ((int64_t)t * 4 + r) * 64 + i + 16 * kk;
            T[TL.HF() + o] = sdg[i * LBp + l] * li;
            T[TL.HB() + o] = sof[i * LBp + l] * li;
            if (i < 15) lam *= r_at(base + i, l);
        }
        for (int n = 0; n < 16; ++n) T[TL.DT() + ((int64_t)t * 4 + r) * 64 + 16 * kk + n] = dv;
        // Lam[i][j] = P_i / P_j with the in-block prefix products P_i = prod_{k<i} rho_{base+k}
        // (P_j >= rho_min^15 > 0 for the positions of the block): store g_i P_i over
        // the dg/of rows and 1/P_j over rho rows 1..16 of this shift's column
        double P[16];
        P[0] = 1.0;
        for (int i = 1; i < 16; ++i) P[i] = (i <= istar) ? P[i - 1] * r_at(base + i - 1, l) : 0.0;
        // padded shifts have rho = 0, hence P = 0: they contribute nothing
        const bool live = P[istar] > 0.0;
        const double inv_last = live ? 1.0 / P[istar] : 0.0;
        double inv = inv_last;
        double invs[16];
        for (int j = istar; j >= 0; --j) {
            invs[j] = inv;
            if (j > 0) inv *= r_at(base + j - 1, l);
        }
        for (int i = 0; i < 16; ++i) {
            const bool ok = live && i <= istar;
            sdg[i * LBp + l] = ok ? sdg[i * LBp + l] * P[i] : 0.0;
            sof[i * LBp + l] = ok ? sof[i * LBp + l] * P[i] : 0.0;
            srho[(1 + i) * LBp + l] = ok ? invs[i] : 0.0;
        }
    }
    __syncthreads();
    {
        // Ghat[i][j] = sum_l g^l_i P^l_i / P^l_j  (j <= i <= istar), shifts in increasing order
        const int i = threadIdx.x >> 4, j = threadIdx.x & 15;  // 256 threads = 16 x 16 pairs
        double gf = 0.0, gb = 0.0;
        if (j <= i && i <= istar) {
            for (int l = 0; l < LBp; ++l) {
                const double bj = srho[(1 + j) * LBp + l];
                gf = fma(sdg[i * LBp + l], bj, gf);
                gb = fma(sof[i * LBp + l], bj, gb);
            }
        }
        const int64_t o = (int64_t)(j >> 2) * 64 + i + 16 * (j & 3);
        T[TL.GF() + o] = gf;
        T[TL.GB() + o] = gb;
    }
}

// Pass A: one wavefront = one edge x 16 samples, all (padded) shifts.
template <int NT, bool FWD>
__global__ void __launch_bounds__(256) k_sweep_blocked(const int64_t *__restrict__ off_,
                                                       const int32_t *__restrict__ m_,
                                                       const int32_t *__restrict__ boff, int32_t E, int64_t N,
                                                       int32_t nb, int32_t Sp, int32_t LB, int32_t LBp,
                                                       const double *__restrict__ tab, const double *__restrict__ X,
                                                       double *__restrict__ U, const double *__restrict__ rhom,
                                                       double *__restrict__ ends) {
    const int L = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + wave_id();
    const int ng = 4 * nb;
    if (q >= (int64_t)E * ng) return;
    const int e = (int)(q / ng);
    const int g = (int)(q - (int64_t)e * ng);
    const int b = g >> 2;
    const int s0 = 16 * g;
    const int n = L & 15, kq = L >> 4;
    const int m = m_[e];
    const int side = FWD ? 1 : 0;
    double *endp = ends + ((int64_t)e * 2 + side) * Sp + s0 + n;
    const int64_t endstride = (int64_t)E * 2 * Sp;
    const TabLayout TL{NT};
    if (m == 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int sh = 16 * t + 4 * r + kq;
                if (sh < LB) endp[sh * endstride] = 0.0;
            }
        return;
    }
    const int64_t off = off_[e];
    const double *xb = X + ((int64_t)b * N + off) * 64 + 16 * (g & 3) + n;
    double *ub = U + ((int64_t)b * N + off) * 64 + 16 * (g & 3) + n;
    const int nblk = (m + 15) >> 4;
    const int64_t eb0 = boff[e];
    d4 Y[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) Y[t] = d4{0.0, 0.0, 0.0, 0.0};
    auto pos = [&](int p) -> int64_t { return FWD ? (int64_t)p : (int64_t)(m - 1 - p); };
#pragma unroll 1
    for (int beta = 0; beta < nblk; ++beta) {
        const double *T = tab + (eb0 + beta) * TL.size();
        double R[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int p = 16 * beta + 4 * c + kq;
            R[c] = (p < m) ? xb[pos(p) * 64] : 0.0;
        }
        const double *G = T + (FWD ? TL.GF() : TL.GB());
        const double *H = T + (FWD ? TL.HF() : TL.HB());
        d4 F0 = d4{0.0, 0.0, 0.0, 0.0}, F1 = d4{0.0, 0.0, 0.0, 0.0};
        F0 = mfma(G[0 * 64 + L], R[0], F0);
        F1 = mfma(G[1 * 64 + L], R[1], F1);
        F0 = mfma(G[2 * 64 + L], R[2], F0);
        F1 = mfma(G[3 * 64 + L], R[3], F1);
        if (beta > 0) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                F0 = mfma(H[(t * 4 + 0) * 64 + L], Y[t][0], F0);
                F1 = mfma(H[(t * 4 + 1) * 64 + L], Y[t][1], F1);
                F0 = mfma(H[(t * 4 + 2) * 64 + L], Y[t][2], F0);
                F1 = mfma(H[(t * 4 + 3) * 64 + L], Y[t][3], F1);
            }
        }
        // carry: Y <- d .* Y + C R
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) Y[t][r] *= T[TL.DT() + (t * 4 + r) * 64 + L];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int t = 0; t < NT; ++t) Y[t] = mfma(T[TL.CT() + (t * 4 + c) * 64 + L], R[c], Y[t]);
        // accumulate the block's output rows 4r + kq
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = 16 * beta + 4 * r + kq;
            const double f = F0[r] + F1[r];
            if (FWD) {
                if (p < m) ub[(int64_t)p * 64] += f;
            } else {
                const int op = m - 2 - p;  // output position of reversed step p
                if (p < m && op >= 0) ub[(int64_t)op * 64] += f;
            }
        }
    }
    // end values |b| w = rho_{m-1} * (carry at the last position)
    const double *rm = rhom + (int64_t)e * LBp;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int sh = 16 * t + 4 * r + kq;
            if (sh < LB) endp[sh * endstride] = rm[sh] * Y[t][r];
        }
}

// Pass B: u_I += sum_l |b_l| (u_tail^l Z_tail^l + u_head^l Z_head^l), with
// Z_tail = (T^{-1})_{.,0} and Z_head = (T^{-1})_{.,m-1} in operand layout
// (written by the coefficient kernel: [t][r][64] tail, then [t][r][64] head).
template <int NT>
__global__ void __launch_bounds__(256) k_corr_blocked(const int64_t *__restrict__ off_, const int32_t *__restrict__ m_,
                                                      const int32_t *__restrict__ eu_,
                                                      const int32_t *__restrict__ ev_,
                                                      const int32_t *__restrict__ boff, int32_t E, int32_t V,
                                                      int64_t N, int32_t nb, int32_t Sp, int32_t LB, int32_t LBp,
                                                      const double *__restrict__ ztab,
                                                      const double *__restrict__ babs,
                                                      const double *__restrict__ ug, double *__restrict__ U) {
    const int L = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + wave_id();
    const int ng = 4 * nb;
    if (q >= (int64_t)E * ng) return;
    const int e = (int)(q / ng);
    const int g = (int)(q - (int64_t)e * ng);
    const int b = g >> 2;
    const int s0 = 16 * g;
    const int n = L & 15, kq = L >> 4;
    const int m = m_[e];
    if (m == 0) return;
    const int64_t off = off_[e];
    double *ub = U + ((int64_t)b * N + off) * 64 + 16 * (g & 3) + n;
    const int vt = eu_[e], vh = ev_[e];
    double ct[NT][4], ch[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int sh = 16 * t + 4 * r + kq;
            const int shc = min(sh, LB - 1);
            const double bb = (sh < LB) ? babs[(int64_t)e * LBp + sh] : 0.0;
            ct[t][r] = bb * ug[((int64_t)shc * V + vt) * Sp + s0 + n];
            ch[t][r] = bb * ug[((int64_t)shc * V + vh) * Sp + s0 + n];
        }
    const int nblk = (m + 15) >> 4;
    const int64_t eb0 = boff[e];
#pragma unroll 1
    for (int beta = 0; beta < nblk; ++beta) {
        const double *Z = ztab + (eb0 + beta) * (int64_t)(512 * NT);
        d4 F0 = d4{0.0, 0.0, 0.0, 0.0}, F1 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                F0 = mfma(Z[(t * 4 + r) * 64 + L], ct[t][r], F0);
                F1 = mfma(Z[256 * NT + (t * 4 + r) * 64 + L], ch[t][r], F1);
            }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pp = 16 * beta + 4 * r + kq;
            if (pp < m) ub[(int64_t)pp * 64] += F0[r] + F1[r];
        }
    }
}

template <int NT>
void sweep_nt(const MeshView &mv, const BlockArgs &a, bool fwd, hipStream_t st) {
    const int64_t waves = (int64_t)mv.E * 4 * a.nb;
    dim3 grid((unsigned)((waves + 3) / 4));
    if (fwd)
        hipLaunchKernelGGL((k_sweep_blocked<NT, true>), grid, dim3(256), 0, st, mv.off, mv.m, a.boff, mv.E, mv.N,
                           a.nb, a.Sp, a.LB, a.LBp, a.tab, a.X, a.U, a.rhom, a.ends);
    else
        hipLaunchKernelGGL((k_sweep_blocked<NT, false>), grid, dim3(256), 0, st, mv.off, mv.m, a.boff, mv.E, mv.N,
                           a.nb, a.Sp, a.LB, a.LBp, a.tab, a.X, a.U, a.rhom, a.ends);
    GRF_LAUNCH_CHECK();
}

template <int NT>
void corr_nt(const MeshView &mv, const BlockArgs &a, hipStream_t st) {
    const int64_t waves = (int64_t)mv.E * 4 * a.nb;
    dim3 grid((unsigned)((waves + 3) / 4));
    hipLaunchKernelGGL((k_corr_blocked<NT>), grid, dim3(256), 0, st, mv.off, mv.m, mv.eu, mv.ev, a.boff, mv.E, mv.V,
                       mv.N, a.nb, a.Sp, a.LB, a.LBp, a.ztab, a.babs, a.ug, a.U);
    GRF_LAUNCH_CHECK();
}

}  // namespace

int64_t block_tab_doubles(int32_t NT) { return TabLayout{NT}.size(); }

void launch_blocktab(const MeshView &mv, const BlockArgs &a, hipStream_t st) {
    if (a.nblocks == 0) return;
    GRF_REQUIRE(a.LBp == 16 * a.NT && a.NT >= 1 && a.NT <= 8, "internal: blocked sweeps need 16..128 padded shifts");
    GRF_REQUIRE(a.nblocks < (int64_t(1) << 31), "too many edge blocks");
    const size_t lds = sizeof(double) * 49 * (size_t)a.LBp;
    hipLaunchKernelGGL(k_blocktab, dim3((unsigned)a.nblocks), dim3(256), lds, st, mv.off, mv.m, a.boff, mv.E, a.LBp,
                       a.NT, a.rho, a.dg, a.of, a.tab);
    GRF_LAUNCH_CHECK();
}

#define GRF_NT_SWITCH(NTV, CALL)                                   \
    switch (NTV) {                                                 \
        case 1: CALL(1); break;                                    \
        case 2: CALL(2); break;                                    \
        case 3: CALL(3); break;                                    \
        case 4: CALL(4); break;                                    \
        case 5: CALL(5); break;                                    \
        case 6: CALL(6); break;                                    \
        case 7: CALL(7); break;                                    \
        case 8: CALL(8); break;                                    \
        default: GRF_REQUIRE(false, "internal: NT out of range");  \
    }

void launch_sweep_blocked(const MeshView &mv, const BlockArgs &a, bool fwd, hipStream_t st) {
    if (mv.E == 0 || a.LB == 0) return;
#define CALL_SWEEP(K) sweep_nt<K>(mv, a, fwd, st)
    GRF_NT_SWITCH(a.NT, CALL_SWEEP)
#undef CALL_SWEEP
}

void launch_corr_blocked(const MeshView &mv, const BlockArgs &a, hipStream_t st) {
    if (mv.E == 0 || a.LB == 0) return;
#define CALL_CORR(K) corr_nt<K>(mv, a, st)
    GRF_NT_SWITCH(a.NT, CALL_CORR)
#undef CALL_CORR
}

}  // namespace grf
