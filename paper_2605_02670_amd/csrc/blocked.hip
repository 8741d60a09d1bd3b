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
#include <algorithm>

#include "work.h"

namespace grf {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// FP32 16x16x4 (mixed precision): same A/B lane layout, but accumulator item r
// of lane L holds D[4 (L/16) + r][L%16] (verified on gfx950).
__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2):
// hardware workgroup b runs on XCD b % 8.  Renumber them so that each XCD gets a
// contiguous range of logical workgroups; the workgroups of one edge (which
// read the same operand tables) then share an L2.
__device__ __forceinline__ int64_t xcd_logical_block() {
    const int64_t n = gridDim.x, b = blockIdx.x;
    const int64_t x = b & 7, i = b >> 3, q = n >> 3, r = n & 7;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Closed form of the interior block.  T / |b| = tridiag(-1, 2 cosh(theta), -1)
// with cosh(theta) = 1 + eps / 2, so with s_k = sinh(k theta) (Chebyshev
// recurrence s_{k+1} = 2 cosh(theta) s_k - s_{k-1}) the Thomas pivots are
// pi_p = s_{p+2} / s_{p+1}, the multipliers rho_p = s_{p+1} / s_{p+2}, every
// product of consecutive multipliers telescopes,
//     prod_{k=a}^{c-1} rho_k = s_{a+1} / s_{c+1},
// and the inverse is
//     (T^{-1})_{pq} = s_{min(p,q)+1} s_{m-max(p,q)} / (|b| s_1 s_{m+1}).
// Every quantity is evaluated as an expression in w = e^{-theta} and
// E(k) = 1 - e^{-2 k theta} = 2 e^{-k theta} s_k (expm1, no cancellation for
// small theta, no overflow for large theta); there is no sequential pass over
// the positions of an edge.
struct EdgeShift {
    double bab;  // |b| = gamma / h
    double th;   // theta = 2 asinh(sqrt(eps) / 2)
    double w;    // e^{-theta}
    double E1;   // E(1)
    double sh2;  // 2 sinh(theta) = 2 sqrt(eps (1 + eps / 4))
    double ah;   // alpha h / 2
};

__device__ __forceinline__ EdgeShift edge_shift(double cI, double cL, double kap2, double h) {
    EdgeShift s;
    const double alpha = cI + cL * kap2;
    s.bab = cL / h;
    const double eps = alpha * h * h / cL;
    const double se = sqrt(eps);
    s.th = 2.0 * asinh(0.5 * se);
    s.w = exp(-s.th);
    s.E1 = -expm1(-2.0 * s.th);
    s.sh2 = 2.0 * se * sqrt(1.0 + 0.25 * eps);
    s.ah = 0.5 * alpha * h;
    return s;
}

__device__ __forceinline__ double Ek(double th, int k) { return -expm1(-2.0 * th * (double)k); }

// Per-(edge, shift) quantities of eq. local_reduced_schur, closed form:
//   rho_{m-1} = w E(m) / E(m+1),
//   s_d = alpha h / 2 + |b| (1 - rho_{m-1}) = alpha h / 2 + |b| (1 - w)(1 + w^{2m+1}) / E(m+1),
//   s_o = -|b| prod_p rho_p = -|b| w^m E(1) / E(m+1)
// (m = 0 gives s_d = delta, s_o = b).  Thread = (edge, shift), shift fastest.
// With etab, also the scalars every 16-position block of the edge needs for its
// operand tables (k_blocktab), so that the transcendental functions of one
// (edge, shift) run once, not once per block: [E][kEdgeTabFields][LBp], fields
// theta, w, E(1), |b|, 2 sinh(theta) and the split factors of theta_c = min(theta, 40):
// e^{-theta_c}, e^{7.5 theta_c}, e^{-7.5 theta_c}, e^{theta_c}, e^{theta_c - theta}.
enum EdgeTabField { ET_TH, ET_W, ET_E1, ET_BAB, ET_SH2, ET_WC, ET_FA, ET_FB, ET_IWC, ET_RW };
static_assert(ET_RW + 1 == kEdgeTabFields, "etab fields");
constexpr double kThetaSplit = 40.0;      // see k_blocktab

__global__ void __launch_bounds__(256) k_edge_coeff(MeshView mv, const double *__restrict__ shift, int32_t LB,
                                                    int32_t LBp, double *__restrict__ babs,
                                                    double *__restrict__ rhom, double *__restrict__ sd,
                                                    double *__restrict__ so, double *__restrict__ etab) {
    const int64_t n = mv.E * (int64_t)LBp;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = idx / LBp;
        const int l = (int)(idx - e * LBp);
        const int64_t il = (int64_t)l * mv.E + e;
        double *et = etab ? etab + e * kEdgeTabFields * LBp + l : nullptr;
        if (l >= LB) {
            babs[idx] = 0.0;
            rhom[idx] = 0.0;
            sd[il] = 1.0;
            so[il] = 0.0;
            if (et)
                for (int f = 0; f < kEdgeTabFields; ++f) et[f * LBp] = 0.0;
            continue;
        }
        const int m = mv.m[e];
        const EdgeShift s = edge_shift(shift[2 * l], shift[2 * l + 1], mv.kap2[e], mv.he[e]);
        const double Em1 = Ek(s.th, m + 1);
        babs[idx] = s.bab;
        rhom[idx] = (m > 0) ? s.w * Ek(s.th, m) / Em1 : 0.0;
        sd[il] = s.ah + s.bab * (-expm1(-s.th)) * (1.0 + exp(-(2.0 * m + 1.0) * s.th)) / Em1;
        so[il] = -s.bab * exp(-(double)m * s.th) * s.E1 / Em1;
        if (et) {
            const double thc = fmin(s.th, kThetaSplit);
            et[ET_TH * LBp] = s.th;
            et[ET_W * LBp] = s.w;
            et[ET_E1 * LBp] = s.E1;
            et[ET_BAB * LBp] = s.bab;
            et[ET_SH2 * LBp] = s.sh2;
            et[ET_WC * LBp] = exp(-thc);
            et[ET_FA * LBp] = exp(7.5 * thc);
            et[ET_FB * LBp] = exp(-7.5 * thc);
            et[ET_IWC * LBp] = exp(thc);
            et[ET_RW * LBp] = exp(thc - s.th);
        }
    }
}

// table section offsets (doubles) within one block's pass-A table; each
// direction reads two contiguous ranges: forward [HF CT] + [GF DT],
// backward [CT HB] + [DT GB]
struct TabLayout {
    int NT;
    __host__ __device__ int64_t HF() const { return 0; }                  // [t][r][64]: H_fwd[L%16][16t + 4r + L/16]
    __host__ __device__ int64_t CT() const { return 256 * NT; }           // [t][c][64]: C[16t + L%16][4c + L/16]
    __host__ __device__ int64_t HB() const { return 512 * NT; }           // [t][r][64]: H_bwd[...]
    __host__ __device__ int64_t GF() const { return 768 * NT; }           // [c][64]: Ghat_fwd[L%16][4c + L/16]
    __host__ __device__ int64_t DT() const { return 768 * NT + 256; }     // [LBp]: d[l]
    __host__ __device__ int64_t GB() const { return 784 * NT + 256; }     // [c][64]: Ghat_bwd
    __host__ __device__ int64_t size() const { return 784 * (int64_t)NT + 512; }
};

// bmap[b] = (edge, index of the block within the edge) for every 16-position block;
// thread = edge
__global__ void k_block_map(const int32_t *__restrict__ boff, int64_t E, int2 *__restrict__ bmap) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x)
        for (int32_t b = boff[e]; b < boff[e + 1]; ++b) bmap[b] = make_int2((int)e, b - boff[e]);
}

constexpr int kTabThreads = 128;          // one thread per (padded) shift, LBp <= 128
// LDS row padding of the Ghat factors: 2 doubles keeps a 96-shift block at 26.7 KB, so
// that 6 workgroups (3 wavefronts per SIMD, the register limit) fit a compute unit;
// 4 doubles allowed 5 (64 graphs, 32 samples: 35.8 -> 35.1 ms per step, mean of two runs)
constexpr int kTabPad = 2;

// 16-byte vectors of the table element type
template <typename ET> struct V16;
template <> struct V16<double> { typedef d2 type; };
template <> struct V16<float> { typedef f4 type; };

// Writes thread (shift) l's 16 per-position values v[p] into the operand
// vectors, in one of three layouts:
//   C layout: lane n + 16 q of vector (t, c) <- shift 16t + n, position 4c + q;
//   H/Z layout, FP64 (F32L false): lane i + 16 k of vector (t, r) <- shift 16t + 4r + k, position i;
//   H/Z layout, FP32 (F32L true):  lane i + 16 k of vector (t, r) <- shift 16t + 4k + r, position i
// (the shift order of the accumulator registers used as B operands).  In the
// H/Z layouts a shift's 16 values are 16 contiguous elements (16-byte vector
// stores); in the C layout a store instruction writes 16-element runs.
template <bool CLAYOUT, bool F32L, typename OT>
__device__ __forceinline__ void put16(const double (&v)[16], OT *__restrict__ dst, int l) {
    if constexpr (CLAYOUT) {
        const int t = l >> 4, n = l & 15;
#pragma unroll
        for (int p = 0; p < 16; ++p) dst[(int64_t)(4 * t + (p >> 2)) * 64 + n + 16 * (p & 3)] = (OT)v[p];
    } else {
        const int64_t at = F32L ? (int64_t)(4 * (l >> 4) + (l & 3)) * 64 + 16 * ((l & 15) >> 2)
                                : (int64_t)(l >> 2) * 64 + 16 * (l & 3);
        typedef typename V16<OT>::type VT;
        constexpr int NV = 16 / sizeof(OT);  // elements per 16-byte vector
        VT *d = reinterpret_cast<VT *>(dst + at);
#pragma unroll
        for (int c = 0; c < 16 / NV; ++c) {
            VT x;
#pragma unroll
            for (int k = 0; k < NV; ++k) x[k] = (OT)v[NV * c + k];
            d[c] = x;
        }
    }
}

// 128 / SLOT 16-position edge blocks per workgroup, SLOT >= LBp threads per block,
// thread = shift l of its block (several blocks per workgroup when the shift block
// is short, so that the threads are not mostly idle); per block (base = 16 beta,
// i* = last position of the block, all products from the closed form above):
//   Lam[i][j] = w^{i-j} E(base+j+1) / E(base+i+1)       (j <= i)
//   lam[i]    = w^{i+1} E(base) / E(base+i+1)
//   dg_p = E(p+1) E(m-p) / (2 sinh(theta) |b| E(m+1)),  of_p = w E(p+1) E(m-p-1) / (...)
//   C[l][j] = Lam[i*][j], d[l] = lam[i*], H_fwd[i][l] = dg lam, H_bwd[i][l] = of lam,
//   Z_tail[i][l] = (T^{-1})_{p,0}   = w^{p+1} E(m-p) / (|b| E(m+1)),
//   Z_head[i][l] = (T^{-1})_{p,m-1} = w^{m-p} E(p+1) / (|b| E(m+1)),
// and Ghat_fwd[i][j] = sum_l dg Lam, Ghat_bwd[i][j] = sum_l of Lam on the
// matrix cores: w^{i-j} = w^{i-7.5} w^{7.5-j} splits Ghat into a product of
// a [16 x LBp] and an [LBp x 16] operand, exact on the diagonal.  With theta
// clamped to 40 in the split factors, |exponents| <= 300 (no overflow), and the
// off-diagonal Lam of a shift with theta > 40 (relative size below e^{-40}, far
// under the rounding of its own diagonal term) is replaced by an equally
// negligible value.
template <typename OT, bool PACK>
__global__ void __launch_bounds__(kTabThreads) k_blocktab(MeshView mv, const int2 *__restrict__ bmap,
                                                          const double *__restrict__ etab, int32_t LB, int32_t LBp,
                                                          int32_t NT, int32_t SLOT, int64_t nblocks,
                                                          OT *__restrict__ tab, OT *__restrict__ ztab) {
    constexpr bool F32L = sizeof(OT) == 4;  // FP32 operand tables for the mixed-precision sweeps
    // per block slot, Ghat split factors in rows of ld = LBp + kTabPad doubles: Af rows 0..16
    // (dg / (w^i E(base+i+1))), Bm rows 0..15 (E(base+j+1)), then w / w_split
    extern __shared__ double sfac[];
    __shared__ int sistar[kTabThreads / 16];  // i* of each block slot, for the Ghat products
    const int ld = LBp + kTabPad;
    const int NBW = PACK ? kTabThreads / SLOT : 1;  // blocks per workgroup (SLOT = 128 unless PACK)
    const int tid = threadIdx.x, wv = tid >> 6;
    const int slot = PACK ? tid / SLOT : 0;
    double *sAf = sfac + (int64_t)slot * 34 * ld, *sBm = sAf + 17 * ld, *srw = sAf + 33 * ld;
    const int64_t blk0 = (int64_t)blockIdx.x * NBW;
    const bool bvalid = blk0 + slot < nblocks;  // the last workgroup may hold fewer blocks
    const int64_t blk = bvalid ? blk0 + slot : nblocks - 1;
    const int2 eb = bmap[blk];
    const int e = eb.x, beta = eb.y;
    const int m = mv.m[e];
    const int base = 16 * beta;
    const int istar = min(15, m - 1 - base);
    const TabLayout TL{NT};
    OT *T = tab + blk * TL.size();
    OT *Z = ztab + blk * (int64_t)(512 * NT);
    const int l = tid - slot * SLOT;
    if (PACK && l == 0) sistar[slot] = istar;  // read after the barrier below
    const bool live = bvalid && l < LB;
    const bool put = bvalid && l < LBp;  // a (padded) shift of a real block: its values are stored
    // the edge's per-shift scalars (k_edge_coeff)
    const double *et = etab + (int64_t)e * kEdgeTabFields * LBp + l;
    double th = 0.0, w = 0.0, E1 = 0.0, bab = 1.0, sh2 = 1.0;
    if (live) {
        th = et[ET_TH * LBp];
        w = et[ET_W * LBp];
        E1 = et[ET_E1 * LBp];
        bab = et[ET_BAB * LBp];
        sh2 = et[ET_SH2 * LBp];
    }
    // E values from two evaluations and the addition rule E(a + b) = E(a) + (1 - E(a)) E(b)
    // (positive terms only, no cancellation): Ef[k] = E(base + k), k = 0..16
    double Ef[17];
    Ef[0] = live ? Ek(th, base) : 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) Ef[k + 1] = Ef[k] + (1.0 - Ef[k]) * E1;
    // Q[i] = E(max(m - base - i, 0)), i = 0..16, upwards from Q[16]: exactly 0 for the
    // rows past the edge (i >= nr), which zeroes those rows of every operand with a Q
    // factor (H, Z_tail, Af) without a mask; when the thread is not live, Q, w and the
    // scale factors are 0 and so is every operand value
    const int nr = m - base;  // >= 1: positions of the edge from this block on
    double Q[17];
    Q[16] = live ? Ek(th, max(nr - 16, 0)) : 0.0;
#pragma unroll
    for (int i = 15; i >= 0; --i) Q[i] = (nr - i > 0) ? Q[i + 1] + (1.0 - Q[i + 1]) * E1 : 0.0;
    // E(m + 1) = E(base) + (1 - E(base)) E(nr + 1), E(nr + 1) = Q[0] + (1 - Q[0]) E(1)
    const double En1 = Q[0] + (1.0 - Q[0]) * E1;
    const double Em1 = Ef[0] + (1.0 - Ef[0]) * En1;
    const double K = live ? 1.0 / (bab * Em1) : 0.0;
    const double ascale = live ? K / sh2 : 0.0;
    const double lam0 = Ef[0] * ascale;  // E(base) / (2 sinh(theta) |b| E(m+1))

    double v[16];
    // H_fwd[i] = dg_i lam_i = w^{i+1} E(base) E(m-base-i) / (2 sinh |b| E(m+1))
    {
        double pw = w;  // w^{i+1}
#pragma unroll
        for (int i = 0; i < 16; ++i, pw *= w) v[i] = pw * lam0 * Q[i];
    }
    if (put) put16<false, F32L>(v, T + TL.HF(), l);
    // H_bwd[i] = of_i lam_i = w^{i+2} E(base) E(m-base-i-1) / (...)
    {
        double pw = w * w;  // w^{i+2}
#pragma unroll
        for (int i = 0; i < 16; ++i, pw *= w) v[i] = pw * lam0 * Q[i + 1];
    }
    if (put) put16<false, F32L>(v, T + TL.HB(), l);
    // Z_tail[i] = w^{base+1+i} E(m-base-i) K
    {
        const double wb = live ? exp(-(double)(base + 1) * th) * K : 0.0;
        double pw = 1.0;  // w^i
#pragma unroll
        for (int i = 0; i < 16; ++i, pw *= w) v[i] = wb * pw * Q[i];
    }
    if (put) put16<false, F32L>(v, Z, l);
    // C[j] = w^{i*-j} E(base+j+1) / E(base+i*+1), d = w^{i*+1} E(base) / E(base+i*+1), and
    // Z_head[i] = w^{m-base-i} E(base+i+1) K: descending chains from i*
    double dval = 0.0;
    {  // one chain at a time (fewer live registers)
        double Eis = Ef[16];  // E(base + i* + 1), picked without a division per candidate
#pragma unroll
        for (int j = 0; j < 15; ++j) Eis = (j == istar) ? Ef[j + 1] : Eis;
        const double inv = live ? 1.0 / Eis : 0.0;
        // each chain factor is 0 above i* and starts at i* (1, resp. the scale of Z_head)
        double pw = 0.0;
#pragma unroll
        for (int j = 15; j >= 0; --j) {
            pw = (j == istar) ? 1.0 : pw;
            v[j] = pw * Ef[j + 1] * inv;
            pw *= w;
        }
        dval = pw * Ef[0] * inv;  // pw = w^{i*+1}; 0 when not live (inv = 0)
        if (put) put16<true, F32L>(v, T + TL.CT(), l);
        const double zh = live ? exp(-(double)(m - base - istar) * th) * K : 0.0;
        double zc = 0.0;
#pragma unroll
        for (int j = 15; j >= 0; --j) {
            zc = (j == istar) ? zh : zc;
            v[j] = zc * Ef[j + 1];
            zc *= w;
        }
        if (put) put16<false, F32L>(v, Z + 256 * NT, l);
    }
    if (put) T[TL.DT() + l] = (OT)dval;
    // Ghat operands (split factors); rows past i*+1 (Af) / i* (Bm) are zero
    {
        const double wc = live ? et[ET_WC * LBp] : 0.0;     // w_c = e^{-theta_c}
        double fa = live ? et[ET_FA * LBp] : 0.0;           // w_c^{i-7.5}
        double fb = live ? et[ET_FB * LBp] : 0.0;           // w_c^{7.5-j}
        const double iwc = live ? et[ET_IWC * LBp] : 0.0;
#pragma unroll
        for (int i = 0; i < 17; ++i) {
            if (l < ld) {
                sAf[i * ld + l] = Q[i] * ascale * fa;
                if (i < 16) sBm[i * ld + l] = (live && i <= istar) ? Ef[i + 1] * fb : 0.0;
            }
            fa *= wc;
            fb *= iwc;
        }
        if (l < ld) srw[l] = live ? et[ET_RW * LBp] : 0.0;  // w / w_c
    }
    __syncthreads();
    // Ghat^T = B^T A^T (D layout of the transpose = the A-operand table layout) for every
    // block of the workgroup: wave 0 the forward operands (A = Af rows i), wave 1 the
    // backward ones (A = Af rows i+1 times w/w_c); waves 2, 3 (if any) have none
    if (wv < 2) {
        const int lane = tid & 63;
        const int n = lane & 15, q = lane >> 4;
        for (int sb = 0; sb < NBW; ++sb) {
            const int64_t bk = blk0 + sb;
            if (bk >= nblocks) break;  // uniform over the wavefront
            const double *bAf = sfac + (int64_t)sb * 34 * ld, *bBm = bAf + 17 * ld, *brw = bAf + 33 * ld;
            const int bistar = PACK ? sistar[sb] : istar;
            d4 acc = d4{0.0, 0.0, 0.0, 0.0};
            for (int c = 0; c < LBp / 4; ++c) {
                const int ll = 4 * c + q;
                const double a = bBm[n * ld + ll];
                const double b = (wv == 0) ? bAf[n * ld + ll] : bAf[(n + 1) * ld + ll] * brw[ll];
                acc = mfma(a, b, acc);
            }
            OT *G = tab + bk * TL.size() + (wv == 0 ? TL.GF() : TL.GB());
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int jj = 4 * r + q;  // D row of the transpose = column j of Ghat; lane row n = i
                G[r * 64 + lane] = (OT)((jj <= n && n <= bistar) ? acc[r] : 0.0);
            }
        }
    }
}

// Staging of one block's operands in LDS, shared by the four wavefronts of a
// workgroup (one edge, 64 samples), double-buffered: while the current block is
// computed, the loads of the next block's operands write the other LDS buffer
// themselves (global_load_lds_dwordx4: lane j of a wavefront's load lands 16 j
// bytes past the wavefront-uniform LDS address), so no registers carry them.
// The table is copied as contiguous 16-byte vectors, vector i by thread i mod 256;
// the caller waits with stage_wait before the barrier that publishes the buffer.
// bytes [src1, src1 + n1b) ++ [src2, ...), nbytes in all (multiples of 16, sources 16-byte aligned)
__device__ __forceinline__ void stage_direct_bytes(const char *src1, int n1b, const char *src2, char *dst, int nbytes) {
    const int nv = nbytes / 16;
    const int w = wave_id(), lane = (int)threadIdx.x & 63;
    const int T = (int)blockDim.x;  // 64, 128 or 256 threads
    for (int k = 0; k < (nv + T - 1) / T; ++k) {
        const int v0 = T * k + 64 * w;  // first vector of this wavefront's load
        const int i = v0 + lane;
        if (i < nv) {  // lanes past the table write nothing
            const int d = 16 * i;
            const char *p = d < n1b ? src1 + d : src2 + (d - n1b);
            __builtin_amdgcn_global_load_lds(p, (__attribute__((address_space(3))) void *)(dst + 16 * v0), 16, 0, 0);
        }
    }
}
// ne elements: [src1, src1 + n1) ++ [src2, ...) into dst
__device__ __forceinline__ void stage_direct(const double *src1, int n1, const double *src2, double *dst, int ne) {
    stage_direct_bytes((const char *)src1, 8 * n1, (const char *)src2, (char *)dst, 8 * ne);
}
__device__ __forceinline__ void stage_direct(const float *src1, int n1, const float *src2, float *dst, int ne) {
    stage_direct_bytes((const char *)src1, 4 * n1, (const char *)src2, (char *)dst, 4 * ne);
}

// the direct-staging loads of this wavefront have written LDS: s_waitcnt vmcnt(0)
// (expcnt and lgkmcnt at their maxima), as a builtin so that the compiler's own
// wait placement counts it
__device__ __forceinline__ void stage_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Pass A: workgroup = (edge, 64 samples), wavefront = 16 samples, all
// (padded) shifts.  LDS per buffer (doubles), forward: H 0, C 256NT, G 512NT,
// d 512NT+256; backward: C 0, H 256NT, d 512NT, G 528NT.  With first set
// (the forward pass of the first shift block) the accumulator is written,
// not updated.
template <int NT, bool FWD>
__device__ __forceinline__ void sweep_blocked_dir(const int64_t *__restrict__ off_, const int32_t *__restrict__ m_,
                                                  const int32_t *__restrict__ boff, int32_t E, int64_t N, int32_t nb,
                                                  int32_t Sp, int32_t LB, int32_t LBp, const double *__restrict__ tab,
                                                  const double *__restrict__ X, double *__restrict__ U,
                                                  const double *__restrict__ rhom, double *__restrict__ ends,
                                                  int32_t first, int64_t S, double *__restrict__ sbuf, int64_t wg) {
    constexpr int TS = 528 * NT + 256;  // doubles per buffer
    constexpr int N1 = 512 * NT;        // first contiguous range
    const int L = threadIdx.x & 63;
    const int wv = wave_id();
    // nb: workgroups per edge; a workgroup of nw wavefronts covers 16 nw samples, wavefront
    // wv the 16 samples of group g (64-sample block b of the layout, quarter g & 3)
    const int nw = (int)(blockDim.x >> 6);
    const int e = (int)(wg / nb);
    const int g = nw * (int)(wg - (int64_t)e * nb) + wv;
    const int b = g >> 2;
    const int s0 = 16 * g;
    const bool live = s0 < S;  // a wavefront of padding samples only stages operands
    const int n = L & 15, kq = L >> 4;
    const int m = m_[e];
    const int side = FWD ? 1 : 0;
    double *endp = ends + ((int64_t)e * 2 + side) * Sp + s0 + n;
    const int64_t endstride = (int64_t)E * 2 * Sp;
    const TabLayout TL{NT};
    if (m == 0) {  // uniform over the workgroup
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
    const double *tab0 = tab + (int64_t)boff[e] * TL.size();
    auto src1 = [&](int beta) { return tab0 + beta * TL.size() + (FWD ? TL.HF() : TL.CT()); };
    auto src2 = [&](int beta) { return tab0 + beta * TL.size() + (FWD ? TL.GF() : TL.DT()); };
    // position read at step p, and where its output goes (backward: T^{-1}'s upper part lands one before)
    auto inpos = [&](int p) -> int64_t { return FWD ? (int64_t)p : (int64_t)(m - 1 - p); };
    auto outpos = [&](int p) -> int { return FWD ? p : m - 2 - p; };
    stage_direct(src1(0), N1, src2(0), sbuf, TS);
    double R[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int p = 4 * c + kq;
        R[c] = (live && p < m) ? xb[inpos(p) * 64] : 0.0;
    }
    stage_wait();
    __syncthreads();
    d4 Y[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) Y[t] = d4{0.0, 0.0, 0.0, 0.0};
    const bool store_only = FWD && first;
#pragma unroll 1
    for (int beta = 0; beta < nblk; ++beta) {
        const double *sb = sbuf + (beta & 1) * TS;
        const bool more = beta + 1 < nblk;
        double Rn[4] = {0.0, 0.0, 0.0, 0.0};
        if (more) {
            stage_direct(src1(beta + 1), N1, src2(beta + 1), sbuf + ((beta + 1) & 1) * TS, TS);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int p = 16 * (beta + 1) + 4 * c + kq;
                if (live && p < m) Rn[c] = xb[inpos(p) * 64];
            }
        }
        double uo[4] = {0.0, 0.0, 0.0, 0.0};
        if (!store_only && live) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = 16 * beta + 4 * r + kq;
                const int op = outpos(p);
                if (p < m && op >= 0) uo[r] = ub[(int64_t)op * 64];
            }
        }
        if (live) {
        const double *G = sb + (FWD ? 512 * NT : 528 * NT);
            const double *H = sb + (FWD ? 0 : 256 * NT);
            const double *C = sb + (FWD ? 256 * NT : 0);
            const double *D = sb + (FWD ? 512 * NT + 256 : 512 * NT);
            d4 F[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) F[c] = mfma(G[c * 64 + L], R[c], d4{0.0, 0.0, 0.0, 0.0});
            if (beta > 0) {
                double ha[NT][4];
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) ha[t][r] = H[(t * 4 + r) * 64 + L];
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) F[r] = mfma(ha[t][r], Y[t][r], F[r]);
                // order: the operand reads of the first LA tiles, then per tile its four
                // products followed by the reads of the tile LA ahead, so that the LDS
                // latency runs under the matrix-core work
                constexpr int LA = NT < 2 ? NT : 2;
                __builtin_amdgcn_sched_group_barrier(0x100, 2 * LA, 0);
#pragma unroll
                for (int t = 0; t < NT - LA; ++t) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
                    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x008, 4 * LA, 0);
            }
            // carry: Y <- d .* Y + C R
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) Y[t][r] *= D[16 * t + 4 * r + kq];
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int t = 0; t < NT; ++t) Y[t] = mfma(C[(t * 4 + c) * 64 + L], R[c], Y[t]);
            // the block's output rows 4r + kq
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = 16 * beta + 4 * r + kq;
                const int op = outpos(p);
                const double f = (F[0][r] + F[1][r]) + (F[2][r] + F[3][r]);
                if (p < m && op >= 0) ub[(int64_t)op * 64] = uo[r] + f;
            }
        }
        if (more) stage_wait();
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 4; ++c) R[c] = Rn[c];
    }
    // end values |b| w = rho_{m-1} * (carry at the last position)
    const double *rm = rhom + (int64_t)e * LBp;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int sh = 16 * t + 4 * r + kq;
            if (live && sh < LB) endp[sh * endstride] = rm[sh] * Y[t][r];
        }
}

// Pass A, both directions in one launch: a workgroup runs the forward sweep of
// its (edge, samples), then the backward one over the same edge, whose reads of
// W and of the forward part of u_I then come from the caches rather than HBM.
// The barrier between them publishes the forward part (written by other lanes
// of the same wavefronts) and frees the staging buffers.
template <int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_sweep_blocked(const int64_t *__restrict__ off_, const int32_t *__restrict__ m_, const int32_t *__restrict__ boff,
                int32_t E, int64_t N, int32_t nb, int32_t Sp, int32_t LB, int32_t LBp, const double *__restrict__ tab,
                const double *__restrict__ X, double *__restrict__ U, const double *__restrict__ rhom,
                double *__restrict__ ends, int32_t first, int64_t S) {
    __shared__ double sbuf[2 * (528 * NT + 256)];
    const int64_t wg = xcd_logical_block();
    sweep_blocked_dir<NT, true>(off_, m_, boff, E, N, nb, Sp, LB, LBp, tab, X, U, rhom, ends, first, S, sbuf, wg);
    __syncthreads();
    sweep_blocked_dir<NT, false>(off_, m_, boff, E, N, nb, Sp, LB, LBp, tab, X, U, rhom, ends, 0, S, sbuf, wg);
}

// Pass B: u_I += sum_l |b_l| (u_tail^l Z_tail^l + u_head^l Z_head^l), with
// Z_tail = (T^{-1})_{.,0} and Z_head = (T^{-1})_{.,m-1} in operand layout
// ([t][r][64] tail, then [t][r][64] head, 512 NT doubles per block), staged
// through LDS like pass A.
template <int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_corr_blocked(const int64_t *__restrict__ off_, const int32_t *__restrict__ m_,
                                                      const int32_t *__restrict__ eu_,
                                                      const int32_t *__restrict__ ev_,
                                                      const int32_t *__restrict__ boff, int32_t E, int32_t V,
                                                      int64_t N, int32_t nb, int32_t Sp, int32_t LB, int32_t LBp,
                                                      const double *__restrict__ ztab,
                                                      const double *__restrict__ babs,
                                                      const double *__restrict__ ug, double *__restrict__ U,
                                                      int64_t S) {
    constexpr int TS = 512 * NT;
    __shared__ double sbuf[2 * TS];
    const int L = threadIdx.x & 63;
    const int wv = wave_id();
    const int64_t wg = xcd_logical_block();
    // nb: workgroups per edge; a workgroup of nw wavefronts covers 16 nw samples, wavefront
    // wv the 16 samples of group g (64-sample block b of the layout, quarter g & 3)
    const int nw = (int)(blockDim.x >> 6);
    const int e = (int)(wg / nb);
    const int g = nw * (int)(wg - (int64_t)e * nb) + wv;
    const int b = g >> 2;
    const int s0 = 16 * g;
    const bool live = s0 < S;  // a wavefront of padding samples only stages operands
    const int n = L & 15, kq = L >> 4;
    const int m = m_[e];
    if (m == 0) return;  // uniform over the workgroup
    const int64_t off = off_[e];
    double *ub = U + ((int64_t)b * N + off) * 64 + 16 * (g & 3) + n;
    const int vt = eu_[e], vh = ev_[e];
    const double *z0 = ztab + (int64_t)boff[e] * TS;
    stage_direct(z0, TS, z0, sbuf, TS);
    double ct[NT][4], ch[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int sh = 16 * t + 4 * r + kq;
            const int shc = min(sh, LB - 1);
            const double bb = (live && sh < LB) ? babs[(int64_t)e * LBp + sh] : 0.0;
            ct[t][r] = live ? bb * ug[((int64_t)shc * V + vt) * Sp + s0 + n] : 0.0;
            ch[t][r] = live ? bb * ug[((int64_t)shc * V + vh) * Sp + s0 + n] : 0.0;
        }
    stage_wait();
    __syncthreads();
    const int nblk = (m + 15) >> 4;
#pragma unroll 1
    for (int beta = 0; beta < nblk; ++beta) {
        const double *Z = sbuf + (beta & 1) * TS;
        const bool more = beta + 1 < nblk;
        if (more) stage_direct(z0 + (int64_t)(beta + 1) * TS, TS, z0, sbuf + ((beta + 1) & 1) * TS, TS);
        if (live) {
        double uo[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pp = 16 * beta + 4 * r + kq;
                uo[r] = (pp < m) ? ub[(int64_t)pp * 64] : 0.0;
            }
            d4 F[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) F[c] = d4{0.0, 0.0, 0.0, 0.0};
            double zt[NT][4], zh[NT][4];
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    zt[t][r] = Z[(t * 4 + r) * 64 + L];
                    zh[t][r] = Z[256 * NT + (t * 4 + r) * 64 + L];
                }
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    F[r & 1] = mfma(zt[t][r], ct[t][r], F[r & 1]);
                    F[2 + (r & 1)] = mfma(zh[t][r], ch[t][r], F[2 + (r & 1)]);
                }
            // order: the operand reads of the first LA tiles, then per tile its eight
            // products followed by the reads of the tile LA ahead (LDS latency under
            // the matrix-core work)
            constexpr int LA = NT < 2 ? NT : 2;
            __builtin_amdgcn_sched_group_barrier(0x100, 4 * LA, 0);
#pragma unroll
            for (int t = 0; t < NT - LA; ++t) {
                __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, 8 * LA, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pp = 16 * beta + 4 * r + kq;
                if (pp < m) ub[(int64_t)pp * 64] = uo[r] + ((F[0][r] + F[1][r]) + (F[2][r] + F[3][r]));
            }
        }
        if (more) stage_wait();
        __syncthreads();
    }
}

// Mixed precision (FP32 operand tables and matrix-core products, FP64 noise,
// accumulator and end values).  The products of each tile of 16 shifts are summed in
// FP32 on the matrix cores, and the tiles are added in FP64, so the sum over the
// quadrature shifts is FP64 (the position sum of Ghat R runs over one block's 16
// positions, its shift sum is inside Ghat, formed in FP64).  Same structure as the
// FP64 kernels; the
// carried state Y[t] item r of lane L is shift 16t + 4 (L/16) + r and the
// block output item r of lane L is position 4 (L/16) + r.
template <int NT, bool FWD, bool SB>
__device__ __forceinline__ void sweep_blocked32_dir(const int64_t *__restrict__ off_, const int32_t *__restrict__ m_,
                                                    const int32_t *__restrict__ boff, int32_t E, int64_t N, int32_t nb,
                                                    int32_t Sp, int32_t LB, int32_t LBp, const float *__restrict__ tab,
                                                    const double *__restrict__ X, double *__restrict__ U,
                                                    const double *__restrict__ rhom, float *__restrict__ ends,
                                                    int32_t first, int64_t S, float *__restrict__ sbuf, int64_t wg) {
    constexpr int TS = 528 * NT + 256;  // floats per buffer
    constexpr int N1 = 512 * NT;
    const int L = threadIdx.x & 63;
    const int wv = wave_id();
    // nb: workgroups per edge; a workgroup of nw wavefronts covers 16 nw samples, wavefront
    // wv the 16 samples of group g (64-sample block b of the layout, quarter g & 3)
    const int nw = (int)(blockDim.x >> 6);
    const int e = (int)(wg / nb);
    const int g = nw * (int)(wg - (int64_t)e * nb) + wv;
    const int b = g >> 2;
    const int s0 = 16 * g;
    const bool live = s0 < S;  // a wavefront of padding samples only stages operands
    const int n = L & 15, kq = L >> 4;
    const int m = m_[e];
    const int side = FWD ? 1 : 0;
    float *endp = ends + ((int64_t)e * 2 + side) * Sp + s0 + n;
    const int64_t endstride = (int64_t)E * 2 * Sp;
    const TabLayout TL{NT};
    if (m == 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int sh = 16 * t + 4 * kq + r;
                if (sh < LB) endp[sh * endstride] = 0.0f;
            }
        return;
    }
    const int64_t off = off_[e];
    const double *xb = X + ((int64_t)b * N + off) * 64 + 16 * (g & 3) + n;
    double *ub = U + ((int64_t)b * N + off) * 64 + 16 * (g & 3) + n;
    const int nblk = (m + 15) >> 4;
    const float *tab0 = tab + (int64_t)boff[e] * TL.size();
    auto src1 = [&](int beta) { return tab0 + beta * TL.size() + (FWD ? TL.HF() : TL.CT()); };
    auto src2 = [&](int beta) { return tab0 + beta * TL.size() + (FWD ? TL.GF() : TL.DT()); };
    auto inpos = [&](int p) -> int64_t { return FWD ? (int64_t)p : (int64_t)(m - 1 - p); };
    auto outpos = [&](int p) -> int { return FWD ? p : m - 2 - p; };
    stage_direct(src1(0), N1, src2(0), sbuf, TS);
    float R[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int p = 4 * c + kq;
        R[c] = (live && p < m) ? (float)xb[inpos(p) * 64] : 0.0f;
    }
    stage_wait();
    __syncthreads();
    f4 Y[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) Y[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const bool store_only = FWD && first;
#pragma unroll 1
    for (int beta = 0; beta < nblk; ++beta) {
        if (SB && beta > 0) {  // single buffer: the block's operands after the last block's barrier
            stage_direct(src1(beta), N1, src2(beta), sbuf, TS);
            stage_wait();
            __syncthreads();
        }
        const float *sb = SB ? sbuf : sbuf + (beta & 1) * TS;
        const bool more = beta + 1 < nblk;
        float Rn[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (more) {
            if (!SB) stage_direct(src1(beta + 1), N1, src2(beta + 1), sbuf + ((beta + 1) & 1) * TS, TS);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int p = 16 * (beta + 1) + 4 * c + kq;
                if (live && p < m) Rn[c] = (float)xb[inpos(p) * 64];
            }
        }
        double uo[4] = {0.0, 0.0, 0.0, 0.0};
        if (!store_only && live) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = 16 * beta + 4 * kq + r;
                const int op = outpos(p);
                if (p < m && op >= 0) uo[r] = ub[(int64_t)op * 64];
            }
        }
        if (live) {
        const float *G = sb + (FWD ? 512 * NT : 528 * NT);
            const float *H = sb + (FWD ? 0 : 256 * NT);
            const float *C = sb + (FWD ? 256 * NT : 0);
            const float *D = sb + (FWD ? 512 * NT + 256 : 512 * NT);
            f4 F[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) F[c] = mfma32(G[c * 64 + L], R[c], f4{0.0f, 0.0f, 0.0f, 0.0f});
            double A64[4] = {0.0, 0.0, 0.0, 0.0};
            if (beta > 0) {
                float ha[NT][4];
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) ha[t][r] = H[(t * 4 + r) * 64 + L];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    f4 P = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int r = 0; r < 4; ++r) P = mfma32(ha[t][r], Y[t][r], P);
#pragma unroll
                    for (int i = 0; i < 4; ++i) A64[i] += (double)P[i];
                }
                // reads LA tiles ahead of the products, as in the FP64 kernel
                constexpr int LA = NT < 2 ? NT : 2;
                __builtin_amdgcn_sched_group_barrier(0x100, 2 * LA, 0);
#pragma unroll
                for (int t = 0; t < NT - LA; ++t) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
                    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x008, 4 * LA, 0);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) Y[t][r] *= D[16 * t + 4 * kq + r];
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int t = 0; t < NT; ++t) Y[t] = mfma32(C[(t * 4 + c) * 64 + L], R[c], Y[t]);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = 16 * beta + 4 * kq + r;
                const int op = outpos(p);
                const float f = (F[0][r] + F[1][r]) + (F[2][r] + F[3][r]);
                if (p < m && op >= 0) ub[(int64_t)op * 64] = uo[r] + ((double)f + A64[r]);
            }
        }
        if (!SB && more) stage_wait();
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 4; ++c) R[c] = Rn[c];
    }
    const double *rm = rhom + (int64_t)e * LBp;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int sh = 16 * t + 4 * kq + r;
            if (live && sh < LB) endp[sh * endstride] = (float)(rm[sh] * (double)Y[t][r]);
        }
}

// Pass A with FP32 operands, both directions in one launch (as k_sweep_blocked).
// SB: one staging buffer instead of two (the block's operands load after the barrier
// that ends the previous block), for workgroups of 1 or 2 wavefronts, where two
// buffers would leave the LDS room for too few workgroups (64 graphs, 32 samples:
// 10 -> 16 wavefronts per compute unit, pass A 42.5 -> 34.4 ms).  With 4 wavefronts
// the registers already cap a compute unit at 16, and the FP64 kernels and pass B
// measured slower single-buffered.
template <int NT, bool SB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 4)))
k_sweep_blocked32(const int64_t *__restrict__ off_, const int32_t *__restrict__ m_, const int32_t *__restrict__ boff,
                  int32_t E, int64_t N, int32_t nb, int32_t Sp, int32_t LB, int32_t LBp,
                  const float *__restrict__ tab, const double *__restrict__ X, double *__restrict__ U,
                  const double *__restrict__ rhom, float *__restrict__ ends, int32_t first, int64_t S) {
    __shared__ float sbuf[(SB ? 1 : 2) * (528 * NT + 256)];
    const int64_t wg = xcd_logical_block();
    sweep_blocked32_dir<NT, true, SB>(off_, m_, boff, E, N, nb, Sp, LB, LBp, tab, X, U, rhom, ends, first, S, sbuf, wg);
    __syncthreads();
    sweep_blocked32_dir<NT, false, SB>(off_, m_, boff, E, N, nb, Sp, LB, LBp, tab, X, U, rhom, ends, 0, S, sbuf, wg);
}

template <int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 4)))
k_corr_blocked32(const int64_t *__restrict__ off_, const int32_t *__restrict__ m_, const int32_t *__restrict__ eu_,
                 const int32_t *__restrict__ ev_, const int32_t *__restrict__ boff, int32_t E, int32_t V, int64_t N,
                 int32_t nb, int32_t Sp, int32_t LB, int32_t LBp, const float *__restrict__ ztab,
                 const double *__restrict__ babs, const float *__restrict__ ug, double *__restrict__ U,
                 int64_t S) {
    constexpr int TS = 512 * NT;
    __shared__ float sbuf[2 * TS];
    const int L = threadIdx.x & 63;
    const int wv = wave_id();
    const int64_t wg = xcd_logical_block();
    // nb: workgroups per edge; a workgroup of nw wavefronts covers 16 nw samples, wavefront
    // wv the 16 samples of group g (64-sample block b of the layout, quarter g & 3)
    const int nw = (int)(blockDim.x >> 6);
    const int e = (int)(wg / nb);
    const int g = nw * (int)(wg - (int64_t)e * nb) + wv;
    const int b = g >> 2;
    const int s0 = 16 * g;
    const bool live = s0 < S;  // a wavefront of padding samples only stages operands
    const int n = L & 15, kq = L >> 4;
    const int m = m_[e];
    if (m == 0) return;
    const int64_t off = off_[e];
    double *ub = U + ((int64_t)b * N + off) * 64 + 16 * (g & 3) + n;
    const int vt = eu_[e], vh = ev_[e];
    const float *z0 = ztab + (int64_t)boff[e] * TS;
    stage_direct(z0, TS, z0, sbuf, TS);
    float ct[NT][4], ch[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int sh = 16 * t + 4 * kq + r;
            const int shc = min(sh, LB - 1);
            const double bb = (live && sh < LB) ? babs[(int64_t)e * LBp + sh] : 0.0;
            ct[t][r] = live ? (float)(bb * (double)ug[((int64_t)shc * V + vt) * Sp + s0 + n]) : 0.0f;
            ch[t][r] = live ? (float)(bb * (double)ug[((int64_t)shc * V + vh) * Sp + s0 + n]) : 0.0f;
        }
    stage_wait();
    __syncthreads();
    const int nblk = (m + 15) >> 4;
#pragma unroll 1
    for (int beta = 0; beta < nblk; ++beta) {
        const float *Z = sbuf + (beta & 1) * TS;
        const bool more = beta + 1 < nblk;
        if (more) stage_direct(z0 + (int64_t)(beta + 1) * TS, TS, z0, sbuf + ((beta + 1) & 1) * TS, TS);
        if (live) {
        double uo[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pp = 16 * beta + 4 * kq + r;
                uo[r] = (pp < m) ? ub[(int64_t)pp * 64] : 0.0;
            }
            f4 F[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) F[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            float zt[NT][4], zh[NT][4];
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    zt[t][r] = Z[(t * 4 + r) * 64 + L];
                    zh[t][r] = Z[256 * NT + (t * 4 + r) * 64 + L];
                }
            double A64[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                f4 P0 = f4{0.0f, 0.0f, 0.0f, 0.0f}, P1 = P0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    P0 = mfma32(zt[t][r], ct[t][r], P0);
                    P1 = mfma32(zh[t][r], ch[t][r], P1);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) A64[i] += (double)(P0[i] + P1[i]);
            }
            // reads LA tiles ahead of the products, as in the FP64 kernel
            constexpr int LA = NT < 2 ? NT : 2;
            __builtin_amdgcn_sched_group_barrier(0x100, 4 * LA, 0);
#pragma unroll
            for (int t = 0; t < NT - LA; ++t) {
                __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, 8 * LA, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pp = 16 * beta + 4 * kq + r;
                if (pp < m) ub[(int64_t)pp * 64] = uo[r] + A64[r];
            }
        }
        if (more) stage_wait();
        __syncthreads();
    }
}

// Wavefronts per workgroup of the sweeps: 16 samples each, so that a call with
// few samples has no wavefronts that only stage operands (32 samples: two per
// workgroup, and more workgroups per compute unit); nb of the kernels is then the
// number of workgroups per edge.
static int sweep_waves(int64_t S) { return S > 32 ? 4 : (S > 16 ? 2 : 1); }
static int32_t sweep_groups(int64_t S) {
    const int nw = sweep_waves(S);
    return (int32_t)((S + 16 * nw - 1) / (16 * nw));
}

template <int NT>
void sweep_nt(const MeshView &mv, const BlockArgs &a, hipStream_t st) {
    const int32_t wpe = sweep_groups(a.S);
    const dim3 grid((unsigned)(mv.E * (int64_t)wpe)), block((unsigned)(64 * sweep_waves(a.S)));
    if (a.mixed && sweep_waves(a.S) < 4)
        hipLaunchKernelGGL((k_sweep_blocked32<NT, true>), grid, block, 0, st, mv.off, mv.m, a.boff, mv.E, mv.N, wpe,
                           a.Sp, a.LB, a.LBp, a.tab32, a.X, a.U, a.rhom, a.ends32, a.first, a.S);
    else if (a.mixed)
        hipLaunchKernelGGL((k_sweep_blocked32<NT, false>), grid, block, 0, st, mv.off, mv.m, a.boff, mv.E, mv.N, wpe,
                           a.Sp, a.LB, a.LBp, a.tab32, a.X, a.U, a.rhom, a.ends32, a.first, a.S);
    else
        hipLaunchKernelGGL((k_sweep_blocked<NT>), grid, block, 0, st, mv.off, mv.m, a.boff, mv.E, mv.N, wpe, a.Sp,
                           a.LB, a.LBp, a.tab, a.X, a.U, a.rhom, a.ends, a.first, a.S);
    GRF_LAUNCH_CHECK();
}

template <int NT>
void corr_nt(const MeshView &mv, const BlockArgs &a, hipStream_t st) {
    const int32_t wpe = sweep_groups(a.S);
    const dim3 grid((unsigned)(mv.E * (int64_t)wpe)), block((unsigned)(64 * sweep_waves(a.S)));
    if (a.mixed) {
        hipLaunchKernelGGL((k_corr_blocked32<NT>), grid, block, 0, st, mv.off, mv.m, mv.eu, mv.ev, a.boff, mv.E,
                           mv.V, mv.N, wpe, a.Sp, a.LB, a.LBp, a.ztab32, a.babs, a.ug32, a.U, a.S);
        GRF_LAUNCH_CHECK();
        return;
    }
    hipLaunchKernelGGL((k_corr_blocked<NT>), grid, block, 0, st, mv.off, mv.m, mv.eu, mv.ev, a.boff, mv.E, mv.V,
                       mv.N, wpe, a.Sp, a.LB, a.LBp, a.ztab, a.babs, a.ug, a.U, a.S);
    GRF_LAUNCH_CHECK();
}

}  // namespace

int64_t block_tab_doubles(int32_t NT) { return TabLayout{NT}.size(); }

void launch_edge_coeff(const MeshView &mv, const CoeffArgs &a, hipStream_t st) {
    if (mv.E == 0) return;
    GRF_REQUIRE(a.LBp >= a.LB, "internal: bad padded shift count");
    const int64_t n = mv.E * (int64_t)a.LBp;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_edge_coeff, dim3((unsigned)blocks), dim3(256), 0, st, mv, a.shift, a.LB, a.LBp, a.babs,
                       a.rhom, a.sd, a.so, a.etab);
    GRF_LAUNCH_CHECK();
}

// threads per edge block in the table kernel: the smallest of 16, 32, 64, 128 that holds LBp
static int32_t blocktab_slot(int32_t LBp) {
    int32_t s = 16;
    while (s < LBp) s *= 2;
    return s;
}
static size_t blocktab_lds(int32_t LBp) {
    return sizeof(double) * 34 * (size_t)(LBp + kTabPad) * (kTabThreads / blocktab_slot(LBp));
}

void launch_block_map(const int32_t *boff, int64_t E, int2 *bmap, hipStream_t st) {
    if (E == 0) return;
    hipLaunchKernelGGL(k_block_map, dim3((unsigned)std::min<int64_t>((E + 255) / 256, 65536)), dim3(256), 0, st, boff,
                       E, bmap);
    GRF_LAUNCH_CHECK();
}

void launch_blocktab(const MeshView &mv, const BlockArgs &a, hipStream_t st) {
    if (a.nblocks == 0) return;
    GRF_REQUIRE(a.etab != nullptr && a.bmap != nullptr, "internal: blocked tables need the per-edge scalars");
    GRF_REQUIRE(a.LBp == 16 * a.NT && a.NT >= 1 && a.NT <= 8, "internal: blocked sweeps need 16..128 padded shifts");
    GRF_REQUIRE(a.nblocks < (int64_t(1) << 31), "too many edge blocks");
    const int32_t slot = blocktab_slot(a.LBp);
    const int64_t nbw = kTabThreads / slot;
    const dim3 grid((unsigned)((a.nblocks + nbw - 1) / nbw));
    const bool pack = nbw > 1;  // one block per workgroup compiles to the plain single-block kernel
    if (a.mixed) {
        auto *kern = pack ? k_blocktab<float, true> : k_blocktab<float, false>;
        hipLaunchKernelGGL(kern, grid, dim3(kTabThreads), blocktab_lds(a.LBp), st, mv, a.bmap, a.etab, a.LB, a.LBp,
                           a.NT, slot, a.nblocks, a.tab32, a.ztab32);
    } else {
        auto *kern = pack ? k_blocktab<double, true> : k_blocktab<double, false>;
        hipLaunchKernelGGL(kern, grid, dim3(kTabThreads), blocktab_lds(a.LBp), st, mv, a.bmap, a.etab, a.LB, a.LBp,
                           a.NT, slot, a.nblocks, a.tab, a.ztab);
    }
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

void launch_sweep_blocked(const MeshView &mv, const BlockArgs &a, hipStream_t st) {
    if (mv.E == 0 || a.LB == 0) return;
    GRF_REQUIRE(mv.E * (int64_t)sweep_groups(a.S) < (int64_t(1) << 31), "too many edge x sample-block workgroups");
#define CALL_SWEEP(K) sweep_nt<K>(mv, a, st)
    GRF_NT_SWITCH(a.NT, CALL_SWEEP)
#undef CALL_SWEEP
}

void launch_corr_blocked(const MeshView &mv, const BlockArgs &a, hipStream_t st) {
    if (mv.E == 0 || a.LB == 0) return;
    GRF_REQUIRE(mv.E * (int64_t)sweep_groups(a.S) < (int64_t(1) << 31), "too many edge x sample-block workgroups");
#define CALL_CORR(K) corr_nt<K>(mv, a, st)
    GRF_NT_SWITCH(a.NT, CALL_CORR)
#undef CALL_CORR
}

}  // namespace grf
