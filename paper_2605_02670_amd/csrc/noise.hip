// Lumped white noise W = M_L^{1/2} xi (paper: eq. wh_def; "Mass Lumping":
// the Cholesky factor of the diagonal lumped mass is its element-wise square
// root, so the noise costs O(N)); with GRF_NOISE_CONSISTENT the consistent-mass
// noise of the element factors (k_noise_consistent, also O(N)).
//
// xi is this project's counter-based definition, identical bit for bit on any
// IEEE-754 machine that evaluates the same operations in the same order:
//   * Philox4x64-10 (Salmon et al., SC'11), key = (seed, global sample),
//     counter = (j / 4, 0, 0, 0) for DOF j;
//   * 53-bit uniforms u = (x >> 11) 2^-53;
//   * Box-Muller, r = sqrt(-2 log(1 - u_a)), (r cos 2 pi u_b, r sin 2 pi u_b),
//     with log and sin/cos evaluated by the fixed polynomial schemes below;
//   * DOF j takes component j % 4 of [r_a cos, r_a sin, r_b cos, r_b sin].
// This file is compiled with -ffp-contract=off: no multiply-add is fused, so
// every operation rounds exactly once, as written.
#include "work.h"

namespace grf {
namespace {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;

struct Words {
    uint64_t x[4];
};

__device__ __forceinline__ Words philox4x64_10(uint64_t ctr, uint64_t key0, uint64_t key1, uint64_t ctr1 = 0) {
    uint64_t c0 = ctr, c1 = ctr1, c2 = 0, c3 = 0;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
        uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ key0;
        uint64_t n2 = hi0 ^ c3 ^ key1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        key0 += kWeyl0;
        key1 += kWeyl1;
    }
    return Words{{c0, c1, c2, c3}};
}

__device__ __forceinline__ double unit53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// log on (0, 1]: x = m 2^e with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(s),
// s = (m - 1)/(m + 1), atanh by its odd power series through s^25.
__device__ __forceinline__ double log_fixed(double x) {
    int e;
    double m = frexp(x, &e);
    if (m < 0x1.6a09e667f3bcdp-1) {
        m = m * 2.0;
        e = e - 1;
    }
    double ed = (double)e;
    double f = m - 1.0;
    double s = f / (m + 1.0);
    double s2 = s * s;
    // q = sum_{k=1}^{12} s2^{k-1} / (2k + 1), by Horner from the top term
    double q = 1.0 / 25.0;
    q = q * s2 + 1.0 / 23.0;
    q = q * s2 + 1.0 / 21.0;
    q = q * s2 + 1.0 / 19.0;
    q = q * s2 + 1.0 / 17.0;
    q = q * s2 + 1.0 / 15.0;
    q = q * s2 + 1.0 / 13.0;
    q = q * s2 + 1.0 / 11.0;
    q = q * s2 + 1.0 / 9.0;
    q = q * s2 + 1.0 / 7.0;
    q = q * s2 + 1.0 / 5.0;
    q = q * s2 + 1.0 / 3.0;
    double r = s2 * q;
    double lm = s + s * r;
    double t1 = 2.0 * lm;
    double t2 = ed * 0x1.a39ef35793c76p-33;  // ln2 - ln2_hi
    double t3 = t1 + t2;
    double t4 = ed * 0x1.62e42fee00000p-1;   // ln2_hi (21 trailing zero bits: e * ln2_hi is exact)
    return t4 + t3;
}

// (sin 2 pi u, cos 2 pi u) for u in [0, 1) a multiple of 2^-53: octant o and
// fraction f of 8u are exact; the polynomial runs on a in [0, pi/4].
__device__ __forceinline__ void sincos_2pi_fixed(double u, double &sn, double &cs) {
    double t = u * 8.0;
    double of = floor(t);
    double f = t - of;
    int o = (int)of;
    if (o & 1) f = 1.0 - f;
    double a = f * 0x1.921fb54442d18p-1;  // nearest double to pi/4
    double a2 = a * a;
    // sin a = a + a (a2 ps), ps = sum_{k=1}^{10} (-1)^k a2^{k-1} / (2k+1)!
    double ps = 1.0 / 51090942171709440000.0;                 // +1/21!
    ps = ps * a2 + (-1.0 / 121645100408832000.0);             // -1/19!
    ps = ps * a2 + (1.0 / 355687428096000.0);                 // +1/17!
    ps = ps * a2 + (-1.0 / 1307674368000.0);                  // -1/15!
    ps = ps * a2 + (1.0 / 6227020800.0);                      // +1/13!
    ps = ps * a2 + (-1.0 / 39916800.0);                       // -1/11!
    ps = ps * a2 + (1.0 / 362880.0);                          // +1/9!
    ps = ps * a2 + (-1.0 / 5040.0);                           // -1/7!
    ps = ps * a2 + (1.0 / 120.0);                             // +1/5!
    ps = ps * a2 + (-1.0 / 6.0);                              // -1/3!
    // cos a = 1 + a2 pc, pc = sum_{k=1}^{10} (-1)^k a2^{k-1} / (2k)!
    double pc = 1.0 / 2432902008176640000.0;                  // +1/20!
    pc = pc * a2 + (-1.0 / 6402373705728000.0);               // -1/18!
    pc = pc * a2 + (1.0 / 20922789888000.0);                  // +1/16!
    pc = pc * a2 + (-1.0 / 87178291200.0);                    // -1/14!
    pc = pc * a2 + (1.0 / 479001600.0);                       // +1/12!
    pc = pc * a2 + (-1.0 / 3628800.0);                        // -1/10!
    pc = pc * a2 + (1.0 / 40320.0);                           // +1/8!
    pc = pc * a2 + (-1.0 / 720.0);                            // -1/6!
    pc = pc * a2 + (1.0 / 24.0);                              // +1/4!
    pc = pc * a2 + (-1.0 / 2.0);                              // -1/2!
    double sa = a + a * (a2 * ps);
    double ca = 1.0 + a2 * pc;
    // angle = o pi/4 + theta; a = theta for even o, pi/4 - theta for odd o
    switch (o) {
        case 0: sn = sa; cs = ca; break;
        case 1: sn = ca; cs = sa; break;
        case 2: sn = ca; cs = -sa; break;
        case 3: sn = sa; cs = -ca; break;
        case 4: sn = -sa; cs = -ca; break;
        case 5: sn = -ca; cs = -sa; break;
        case 6: sn = -ca; cs = sa; break;
        default: sn = -sa; cs = ca; break;
    }
}

__device__ __forceinline__ void box_muller(uint64_t xa, uint64_t xb, double &z_cos, double &z_sin) {
    double u1 = 1.0 - unit53(xa);
    double u2 = unit53(xb);
    double r = sqrt(-2.0 * log_fixed(u1));
    double sn, cs;
    sincos_2pi_fixed(u2, sn, cs);
    z_cos = r * cs;
    z_sin = r * sn;
}

// One wavefront = 64 samples of one block of 4 DOFs; lanes are samples, so
// the four stores of a wavefront are each one contiguous 512-byte row.
// Graph z of the batch (blockIdx.z): local DOF j (the counter index of the
// noise definition) lives at row j of its interior range or, for j >= NI_z, at
// row (j - NI_z) of its vertex range.
// lanes of one DOF group in a block of 64 samples holding Sb real ones: the
// samples round up to 16, 32 or 64 lanes, so that a wavefront takes 4, 2 or 1
// DOF groups and no wavefront computes for more than 15 padding samples
__host__ __device__ inline int noise_group_lanes(int64_t Sb) { return Sb <= 16 ? 16 : (Sb <= 32 ? 32 : 64); }

// Thread = (group of 4 DOFs, sample).  Lanes past the real samples store 0 (the
// sweeps read whole 16-sample wavefronts); with 16 or 32 lanes per group the
// lanes of the block past them are not written.
__global__ void __launch_bounds__(256) k_noise(const double *__restrict__ msqrt, const int64_t *__restrict__ segs,
                                               int64_t N, int64_t S, int64_t soff, uint64_t seed,
                                               double *__restrict__ X) {
    const int lane = threadIdx.x & 63;
    const int64_t z = blockIdx.z;
    const int64_t n = segs[4 * z], ni = segs[4 * z + 1], ri = segs[4 * z + 2], rv = segs[4 * z + 3];
    const int64_t ngrp = (n + 3) / 4;
    const int64_t b = blockIdx.y;
    const int64_t Sb = S - b * 64 < 64 ? S - b * 64 : 64;
    const int lpg = noise_group_lanes(Sb), gpw = 64 / lpg;
    const int sl = lane & (lpg - 1), gs = lane / lpg;
    const int64_t s = b * 64 + sl;
    const bool live = sl < Sb;
    double *Xb = X + b * N * 64 + sl;
    for (int64_t g0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * gpw; g0 < ngrp;
         g0 += (int64_t)gridDim.x * 4 * gpw) {
        const int64_t g = g0 + gs;
        if (g >= ngrp) continue;
        double zz[4] = {0.0, 0.0, 0.0, 0.0};
        if (live) {
            Words w = philox4x64_10((uint64_t)g, seed, (uint64_t)(soff + s));
            box_muller(w.x[0], w.x[1], zz[0], zz[1]);
            box_muller(w.x[2], w.x[3], zz[2], zz[3]);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t j = 4 * g + c;
            if (j < n) {
                const int64_t row = j < ni ? ri + j : rv + (j - ni);
                Xb[row * 64] = msqrt[row] * zz[c];
            }
        }
    }
}

// Consistent-mass noise W = R (p, q), R the assembly of the element factors
// F_e = [[a, c], [a, -c]] of M_e = (h_e/6)[[2,1],[1,2]] (a = sqrt(h_e/4),
// c = sqrt(h_e/12)), so that R R^T is the consistent mass (eq. wh_def with any R
// of M = R R^T; the paper takes a Cholesky factor, of the same law).  Element g of
// a graph (g = local first interior row of its edge + local edge index + k for the
// element k between local nodes k and k+1) draws (p, q) from the Philox block with
// counter (g / 2, 1, 0, 0): the first Box-Muller pair for even g, the second for odd.
// It adds a p + c q to its left node and a p - c q to its right one.  Each DOF sums
// its own terms in a fixed order (interior: left element, then right; vertex: its
// edge ends in CSR order, increasing edge, tail before head), so no atomics and the
// same bits on every run.  Lanes are samples (with the lane packing of k_noise); a
// wavefront takes kRowsPerItem consecutive interior rows, so that an element shared
// by two rows of one edge, and a Philox block shared by two elements, is drawn once.
constexpr int kRowsPerItem = 8;

struct ElementDraws {
    uint64_t seed, smp;
    uint64_t blk = ~0ull;  // Philox block held in w
    Words w;
    __device__ void pq(uint64_t g, double &p, double &q) {
        if ((g >> 1) != blk) {
            blk = g >> 1;
            w = philox4x64_10(blk, seed, smp, 1);
        }
        if (g & 1)
            box_muller(w.x[2], w.x[3], p, q);
        else
            box_muller(w.x[0], w.x[1], p, q);
    }
};

__global__ void __launch_bounds__(256) k_noise_consistent(MeshView mv, int64_t S, int64_t soff, uint64_t seed,
                                                          double *__restrict__ X) {
    const int lane = threadIdx.x & 63;
    const int64_t z = blockIdx.z;
    const int64_t n = mv.segs[4 * z], ni = mv.segs[4 * z + 1], ri = mv.segs[4 * z + 2], rv = mv.segs[4 * z + 3];
    const int32_t e0 = mv.ge0[z], e1 = mv.ge0[z + 1], v0 = mv.gv0[z];
    const int64_t b = blockIdx.y;
    const int64_t Sb = S - b * 64 < 64 ? S - b * 64 : 64;
    const int lpg = noise_group_lanes(Sb), gpw = 64 / lpg;
    const int sl = lane & (lpg - 1), gs = lane / lpg;
    const bool live = sl < Sb;
    double *Xb = X + b * mv.N * 64 + sl;
    ElementDraws d{seed, (uint64_t)(soff + b * 64 + sl)};
    // items: the chunks of interior rows, then the vertices
    const int64_t nch = (ni + kRowsPerItem - 1) / kRowsPerItem, nitems = nch + (n - ni);
    for (int64_t i0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * gpw; i0 < nitems;
         i0 += (int64_t)gridDim.x * 4 * gpw) {
        const int64_t it = i0 + gs;
        if (it >= nitems) continue;
        if (it < nch) {
            const int64_t r0 = ri + it * kRowsPerItem;
            const int64_t r1 = min(r0 + kRowsPerItem, ri + ni);
            // the edge holding row r0: the last e with off[e] <= r0 (an edge without
            // interior DOFs shares its offset with the next edge)
            int32_t lo = e0, hi = e1;
            while (hi - lo > 1) {
                const int32_t mid = lo + (hi - lo) / 2;
                if (mv.off[mid] <= r0) lo = mid; else hi = mid;
            }
            int32_t e = lo;
            uint64_t gprev = ~0ull;  // the last right element drawn, and its (p, q)
            double pp = 0.0, qp = 0.0;
            for (int64_t row = r0; row < r1; ++row) {
                while (mv.off[e + 1] <= row) ++e;
                double w = 0.0;
                if (live) {
                    const double he = mv.he[e];
                    const double a = sqrt(0.25 * he), c = sqrt(he / 12.0);
                    const uint64_t gl = (uint64_t)((mv.off[e] - ri) + (e - e0) + (row - mv.off[e]));  // left element
                    double pl, ql, pr, qr;
                    if (gl == gprev) {
                        pl = pp;
                        ql = qp;
                    } else {
                        d.pq(gl, pl, ql);
                    }
                    d.pq(gl + 1, pr, qr);
                    gprev = gl + 1;
                    pp = pr;
                    qp = qr;
                    const double tr = a * pl - c * ql;  // the left element's term at its right node
                    const double tl = a * pr + c * qr;  // the right element's term at its left node
                    w = tr + tl;
                }
                Xb[row * 64] = w;
            }
        } else {
            const int64_t vl = it - nch;
            double w = 0.0;
            if (live) {
                const int64_t v = v0 + vl;
                for (int64_t k = mv.vptr[v]; k < mv.vptr[v + 1]; ++k) {
                    const int32_t e = mv.adj_e[k];
                    const double he = mv.he[e];
                    const double a = sqrt(0.25 * he), c = sqrt(he / 12.0);
                    const uint64_t first = (uint64_t)((mv.off[e] - ri) + (e - e0));
                    double p, q;
                    if (mv.adj_s[k] == 0) {
                        d.pq(first, p, q);
                        const double t = a * p + c * q;
                        w = w + t;
                    } else {
                        d.pq(first + (uint64_t)mv.m[e], p, q);  // element n_e - 1 = m_e
                        const double t = a * p - c * q;
                        w = w + t;
                    }
                }
            }
            Xb[(rv + vl) * 64] = w;
        }
    }
}

}  // namespace

void launch_noise(const MeshView &mv, int64_t S, int64_t soff, uint64_t seed, double *X, hipStream_t st) {
    int64_t nb = (S + 63) / 64;
    const int64_t per = 4 * (64 / noise_group_lanes(S < 64 ? S : 64));  // DOF groups per workgroup pass
    GRF_REQUIRE(nb < 65536 && mv.ng < 65536, "too many samples or graphs in one call");
    if (mv.cnoise) {  // items of kRowsPerItem interior rows, or one vertex
        int64_t gx = (mv.maxNg / kRowsPerItem + mv.maxVg + per - 1) / per;
        gx = std::max<int64_t>(1, std::min<int64_t>(gx, 8192));
        hipLaunchKernelGGL(k_noise_consistent, dim3((unsigned)gx, (unsigned)nb, (unsigned)mv.ng), dim3(256), 0, st,
                           mv, S, soff, seed, X);
    } else {
        int64_t ngrp = (mv.maxNg + 3) / 4;
        int64_t gx = (ngrp + per - 1) / per;
        gx = std::max<int64_t>(1, std::min<int64_t>(gx, 8192));
        hipLaunchKernelGGL(k_noise, dim3((unsigned)gx, (unsigned)nb, (unsigned)mv.ng), dim3(256), 0, st, mv.msqrt,
                           mv.segs, mv.N, S, soff, seed, X);
    }
    GRF_LAUNCH_CHECK();
}

}  // namespace grf
