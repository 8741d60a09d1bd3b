// Vertex Schur-complement system of every (shift, sample) pair.
//
// Paper: eq. global_schur (S u_Gamma = g_Gamma), the condensed right-hand
// side g = W_Gamma - A_Gamma,I A_II^{-1} W_I assembled by the scatter S(.) of
// the edge contributions (eq. local_reduced_schur), and "Phase 4: The Inside
// Loop (PCG solver)": S is never assembled; its product is the sum of the
// edge 2x2 Schur blocks (eq. goal_func_1, eq. goalfunction), here with the
// blocks precomputed per (shift, edge) by coeff.hip.
//
// Readings (the paper leaves them open): x_0 = 0; Jacobi preconditioner (the
// diagonal of S); stop when ||g - S x||_2 <= tol ||g||_2 on the residual
// recomputed from x; g = 0 gives x = 0.
#include <algorithm>
#include <type_traits>

#include "work.h"

namespace grf {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum NV values over the workgroup; every thread gets the same result (the
// partial sums are combined in a fixed order, so the result is deterministic).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds, int nwaves) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        for (int i = 0; i < NV; ++i) lds[i * 16 + (threadIdx.x >> 6)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double t = 0.0;
        for (int w = 0; w < nwaves; ++w) t += lds[i * 16 + w];
        v[i] = t;
    }
}

// g[l][s][v] = W_v + sum over edge ends at v of |b| w_end; tiles of 64 vertices
// x 64 samples are transposed through LDS so both sides are contiguous.  A
// wavefront takes four vertices at a time with their first four edge ends from
// the ELL table (all loads of a step in flight together); vertices of degree
// > 4 add their remaining ends from the CSR lists.
template <typename ET>
__global__ void __launch_bounds__(256) k_condense(MeshView mv, const double *__restrict__ X,
                                                  const ET *__restrict__ ends, int32_t Sp, int64_t S,
                                                  double *__restrict__ gT) {
    __shared__ double tile[64][65];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int v0 = blockIdx.x * 64;
    const int b = blockIdx.y;
    const int l = blockIdx.z;
    // a block of at most 32 real samples takes two vertices per wavefront step (lanes 0-31
    // and 32-63), so that no half of the wavefront only waits
    const int64_t Sb = S - (int64_t)b * 64 < 64 ? S - (int64_t)b * 64 : 64;
    const int nvw = Sb <= 32 ? 2 : 1, lpv = 64 / nvw;
    const int sl = lane & (lpv - 1), hv = lane / lpv;
    const bool real = sl < Sb;  // padding samples load nothing
    const ET *el = ends + (int64_t)l * 2 * mv.E * Sp + (int64_t)b * 64 + sl;  // row 2 e + side
    // tile vertex vb + 4 nvw q (q < 4) of step k: vb = nvw wv + hv + 16 nvw k covers the 64 once
    for (int vb = nvw * wv + hv; vb < 64; vb += 16 * nvw) {
        double g[4] = {0.0, 0.0, 0.0, 0.0};
        if (real) {  // one lane mask per step; inside it no branch until the loads are issued
            int vc[4], id[4][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int v = v0 + vb + 4 * nvw * q;
                vc[q] = min(v, mv.V - 1);
                const double x = X[((int64_t)b * mv.N + mv.NI + vc[q]) * 64 + sl];
                g[q] = v < mv.V ? x : 0.0;
#pragma unroll
                for (int j = 0; j < 4; ++j) id[q][j] = v < mv.V ? mv.eend[(int64_t)j * mv.V + vc[q]] : -1;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double e = (double)el[(int64_t)max(id[q][j], 0) * Sp];  // a valid row even past the degree
                    g[q] += id[q][j] >= 0 ? e : 0.0;
                }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int v = v0 + vb + 4 * nvw * q;
                if (v < mv.V && mv.deg[vc[q]] > 4) {
                    // the loads of eight slots in flight together, added in slot order
                    int64_t k = mv.vptr[v] + 4;
                    const int64_t ke = mv.vptr[v + 1];
                    for (; k + 8 <= ke; k += 8) {
                        int id[8];
                        double ev[8];
#pragma unroll
                        for (int j = 0; j < 8; ++j) id[j] = 2 * mv.adj_e[k + j] + mv.adj_s[k + j];
#pragma unroll
                        for (int j = 0; j < 8; ++j) ev[j] = (double)el[(int64_t)id[j] * Sp];
#pragma unroll
                        for (int j = 0; j < 8; ++j) g[q] += ev[j];
                    }
                    for (; k < ke; ++k) g[q] += (double)el[(int64_t)(2 * mv.adj_e[k] + mv.adj_s[k]) * Sp];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) tile[vb + 4 * nvw * q][sl] = g[q];
    }
    __syncthreads();
    for (int si = wv; si < 64; si += 4) {
        const int64_t s = (int64_t)b * 64 + si;
        const int v = v0 + lane;
        if (s < S && v < mv.V) gT[((int64_t)l * S + s) * mv.V + v] = tile[lane][si];
    }
}

// The vertex systems are solved on their Jacobi-scaled form: with d = diag(S)
// and h = d^{-1/2}, S^ = H S H has unit diagonal, g^ = H g and x = H x^.  CG on
// S^ from x^ = 0 takes exactly the iterates of Jacobi-PCG on S, and needs no
// diagonal in the product and no preconditioner in the update.  The learned
// operators are defined on S^ already: z^ = P^ r^, x0^ = Q^ g^.
//
// Vertex operators of a shift block in ELL-4 form, per row r = prow[u] of vertex u:
// (Op y)_u = diag[l][r] y_u + sum_{j<4} coef[l][r][j] y_{ell[j][u]} + sum over the
// CSR slots k >= vptr[u] + 4 of ovf[l][k] y_{adj_o[k]}  (a self-loop's coupling is
// in the diagonal; its slots carry 0).  For S^ the diagonal is 1 (not stored) and
// dh holds h; for P^ and Q^ diag holds their diagonal.  Rows follow the vertex
// order except in the graphs beyond every on-chip class (MeshView::prow).
struct EllOp {
    double *diag, *dh, *coef, *ovf;  // [LB][V], [LB][V], [LB][V][4], [LB][2E]
};

// h = diag(S)^{-1/2} per (shift, vertex), stored at the vertex's row (prow)
__global__ void k_ell_diag(MeshView mv, const double *__restrict__ sd, const double *__restrict__ so, int32_t LB,
                           double *__restrict__ dh) {
    const int64_t n = (int64_t)LB * mv.V;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(i / mv.V), u = (int)(i - (int64_t)l * mv.V);
        const double *sdl = sd + (int64_t)l * mv.E, *sol = so + (int64_t)l * mv.E;
        double d = 0.0;
        for (int64_t k = mv.vptr[u]; k < mv.vptr[u + 1]; ++k) {
            const int e = mv.adj_e[k];
            d += sdl[e] + (mv.adj_o[k] == u ? sol[e] : 0.0);
        }
        dh[(int64_t)l * mv.V + mv.prow[u]] = 1.0 / sqrt(d);
    }
}

// ELL rows of S^ = H S H, and of the operator preconditioner of the mode:
// learned (PM_LEARNED): P^ and Q^ from the network's per-vertex and per-edge
// outputs, already on the scaled system; Neumann-Neumann (PM_NN): P^ = H^{-1}
// D^{-1} (sum_e S_e^{-1}) D^{-1} H^{-1} (Phase 4, the Neumann step, in its closed
// form), D = diag(d_u) with d_u the edge ends at u, S_e^{-1} =
// [[sd, -so], [-so, sd]] / ((sd - so)(sd + so)) for the edge's 2x2 Schur block
// (eq. local_reduced_schur); a self-loop slot adds its whole block row to the
// diagonal.  Q is not written for PM_NN (initial guess 0).
enum { PM_JACOBI = 0, PM_LEARNED = 1, PM_NN = 2 };

__global__ void k_ell_ops(MeshView mv, const double *__restrict__ sd, const double *__restrict__ so, int32_t LB,
                          EllOp S, int32_t pm, LearnedOps lo, EllOp P, EllOp Q) {
    const int64_t n = (int64_t)LB * mv.V;
    const int64_t E2 = 2 * (int64_t)mv.E;
    const bool lrn = pm == PM_LEARNED, opP = pm != PM_JACOBI;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(i / mv.V), u = (int)(i - (int64_t)l * mv.V);
        const double *sdl = sd + (int64_t)l * mv.E, *sol = so + (int64_t)l * mv.E;
        const double *hl = S.dh + (int64_t)l * mv.V;  // by row (prow)
        const int64_t ru = (int64_t)l * mv.V + mv.prow[u];
        const double hu = hl[mv.prow[u]];
        const int64_t k0 = mv.vptr[u], k1 = mv.vptr[u + 1];
        const double du = (double)(k1 - k0);
        double pdiag = 0.0;  // PM_NN: sum over the slots of (D^-1 S_e^-1 D^-1)_uu
        for (int64_t k = k0; k < k1; ++k) {
            const int e = mv.adj_e[k];
            const int o = mv.adj_o[k];
            const double c = (o == u) ? 0.0 : hu * sol[e] * hl[mv.prow[o]];
            double cp = 0.0, cq = 0.0;
            if (lrn && o != u) {
                cp = lo.Pq[(int64_t)l * mv.E + e];
                cq = lo.Qe[(int64_t)l * mv.E + e];
            } else if (pm == PM_NN) {
                const double sde = sdl[e], soe = sol[e];
                const double det = (sde - soe) * (sde + soe);
                const double isd = sde / det, iso = -soe / det;
                if (o == u) {
                    pdiag += (isd + iso) / (du * du);
                } else {
                    pdiag += isd / (du * du);
                    const double dov = (double)(mv.vptr[o + 1] - mv.vptr[o]);
                    cp = iso / (du * dov * hu * hl[mv.prow[o]]);
                }
            }
            const int j = (int)(k - k0);
            if (j < 4) {
                S.coef[ru * 4 + j] = c;
                if (opP) P.coef[ru * 4 + j] = cp;
                if (lrn) Q.coef[ru * 4 + j] = cq;
            } else {
                S.ovf[(int64_t)l * E2 + k] = c;
                if (opP) P.ovf[(int64_t)l * E2 + k] = cp;
                if (lrn) Q.ovf[(int64_t)l * E2 + k] = cq;
            }
        }
        for (int j = (int)(k1 - k0); j < 4; ++j) {
            S.coef[ru * 4 + j] = 0.0;
            if (opP) P.coef[ru * 4 + j] = 0.0;
            if (lrn) Q.coef[ru * 4 + j] = 0.0;
        }
        if (lrn) {
            P.diag[ru] = lo.Pd[i];
            Q.diag[ru] = lo.Qd[i];
        } else if (pm == PM_NN) {
            P.diag[ru] = pdiag / (hu * hu);
        }
    }
}

// Sums of NV per-system values over a workgroup whose thread t works for system
// (sample) t % SB: every thread gets the sum of its own system.  Inside a
// wavefront the lanes of one system are combined by an xor butterfly (every
// lane ends with the same value); the wavefronts' partials are added through
// LDS in a fixed order, so the result is deterministic.  Two LDS buffers taken
// in turn (a buffer is written again only two sums later, after the barrier of
// the sum in between), so one barrier per sum.
template <int TPB, int SB>
struct SampleSum {
    static constexpr int NW = TPB / 64;
    double *lds;  // [2][4][NW][SB]
    int buf;
    template <int NV>
    __device__ __forceinline__ void operator()(double (&v)[NV]) {
        static_assert(NV <= 4, "at most four values per sum");
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
            for (int o = SB; o < 64; o <<= 1) v[i] += __shfl_xor(v[i], o, 64);
        double *b = lds + buf * 4 * NW * SB;
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        if (lane < SB) {
#pragma unroll
            for (int i = 0; i < NV; ++i) b[(i * NW + w) * SB + lane] = v[i];
        }
        __syncthreads();
        const int s = threadIdx.x % SB;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double t = 0.0;
            for (int k = 0; k < NW; ++k) t += b[(i * NW + k) * SB + s];
            v[i] = t;
        }
        buf ^= 1;
    }
};

// Vertex PCG for the graphs glist[0 .. ngl-1] that no on-chip variant takes:
// one workgroup per (graph, shift, block of SB samples), the SB systems of a
// block solved side by side.  Thread t works for sample t % SB at the local
// vertices t / SB + VS i (VS = TPB / SB).  The vectors g^, x^, r^, p and q of the
// block live in global scratch as [row][SB] rows, in the graph's row order
// (prow / pvtx: Cuthill-McKee for these graphs), (5 maxVg SB doubles per
// resident workgroup), so a neighbour gather reads one contiguous row of SB
// values and each operator row is read once for SB systems.  The systems of
// (g, l, s) are the graph's vertex range of gT / xT[l][s]; statistics go to
// its / res[(g * LB + l) * S + s].
//
// Every system keeps its own scalars, stopping test and restarts, as in the
// on-chip kernel: CG on S^ from x^ = 0 (Jacobi), or with LRN the operator
// preconditioner z^ = P^ r^ and the initial guess x0^ = Q^ g^ (none when
// Qop.diag is null), with the Jacobi fallback after maxit / 2 iterations.  The
// residual g - S x recomputed from x decides convergence; the scaled
// recursive residual only triggers that test.  A converged system stops
// changing while the others go on.  Loop control: after each decision the
// first thread of each system posts in LDS whether it is still active and
// whether it asks for the true-residual step; the barrier at the top of the
// loop makes the flags visible, and every thread reads all of them, so all
// threads take the same branches.
template <int SB, bool LRN>
__global__ void __launch_bounds__(1024) k_pcg_mrhs(MeshView mv, EllOp Sop, EllOp Pop, EllOp Qop,
                                                   const int32_t *__restrict__ glist, int32_t ngl,
                                                   const double *__restrict__ gT, double *__restrict__ xT,
                                                   double *__restrict__ scr, int32_t *__restrict__ its,
                                                   double *__restrict__ res, int32_t LB, int64_t S, double tol,
                                                   int32_t maxit) {
    constexpr int TPB = 1024, VS = TPB / SB;
    static_assert(SB >= 1 && SB <= 64 && (64 % SB) == 0, "samples per block divide a wavefront");
    __shared__ double red[2 * 4 * (TPB / 64) * SB];
    __shared__ int32_t flag[2][SB];  // [0][s]: system s active; [1][s]: it asks for the true-residual step
    SampleSum<TPB, SB> ssum{red, 0};
    const int s = threadIdx.x % SB, vs = threadIdx.x / SB;
    const int64_t E2 = 2 * (int64_t)mv.E;
    const int64_t nsb = (S + SB - 1) / SB;
    const int64_t nunits = (int64_t)ngl * LB * nsb;
    const int64_t rowlen = (int64_t)mv.maxVg * SB;
    double *Gh = scr + (int64_t)blockIdx.x * 5 * rowlen;
    double *X = Gh + rowlen, *R = X + rowlen, *P = R + rowlen, *Q = P + rowlen;
    const int switch_at = max(1, maxit / 2);
    for (int64_t unit = blockIdx.x; unit < nunits; unit += gridDim.x) {
        const int64_t tl = unit / nsb;
        const int64_t smp = (unit - tl * nsb) * SB + s;
        const bool live = smp < S;
        const int l = (int)(tl % LB);
        const int gi = glist[tl / LB];
        const int u0 = mv.gv0[gi], V = mv.gv0[gi + 1] - u0;
        const double *H = Sop.dh + (int64_t)l * mv.V + u0;
        const double *Sc = Sop.coef + (int64_t)l * 4 * mv.V, *So = Sop.ovf + (int64_t)l * E2;
        const double *Pd = LRN ? Pop.diag + (int64_t)l * mv.V : nullptr;
        const double *Pc = LRN ? Pop.coef + (int64_t)l * 4 * mv.V : nullptr;
        const double *Po = LRN ? Pop.ovf + (int64_t)l * E2 : nullptr;
        // (Op y)_v of this thread's system at graph-local row v (operator rows and y
        // in the graph's row order), y in [row][SB]; UNIT: the diagonal is 1
        auto apply = [&](auto unit_diag, const double *dg, const double *cf, const double *of, const double *y,
                         int v) -> double {
            const int r = u0 + v;
            double acc = (decltype(unit_diag)::value ? 1.0 : dg[r]) * y[v * SB + s];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc += cf[4 * (int64_t)r + j] * y[mv.pell[(int64_t)j * mv.V + r] * SB + s];
            const int u = mv.pvtx[r];
            const int d = mv.deg[u];
            if (d > 4) {
                const int64_t k0 = mv.vptr[u];
                for (int64_t k = k0 + 4; k < k0 + d; ++k) acc += of[k] * y[mv.padj[k] * SB + s];
            }
            return acc;
        };
        auto applyS = [&](const double *y, int v) { return apply(std::true_type{}, nullptr, Sc, So, y, v); };
        auto applyP = [&](const double *y, int v) { return apply(std::false_type{}, Pd, Pc, Po, y, v); };

        // g^ and x^0; Jacobi also r^ = p = g^
        double t0[2] = {0.0, 0.0};
#pragma unroll 1
        for (int v = vs; v < V; v += VS) {
            const int i = v * SB + s;
            const double gv = live ? gT[((int64_t)l * S + smp) * mv.V + mv.pvtx[u0 + v]] : 0.0;
            const double gh = H[v] * gv;
            Gh[i] = gh;
            X[i] = 0.0;
            if (!LRN) {
                R[i] = gh;
                P[i] = gh;
            }
            t0[0] += gv * gv;
            t0[1] += gh * gh;
        }
        ssum(t0);
        const double gg = t0[0];
        const double tol2 = tol * tol * gg;
        double thr = tol * tol * t0[1];  // trigger on ||r^||^2, corrected at each test
        if (LRN && Qop.diag != nullptr) {
            __syncthreads();  // g^ complete: Q^ reads neighbours
            const double *Qd = Qop.diag + (int64_t)l * mv.V, *Qc = Qop.coef + (int64_t)l * 4 * mv.V,
                         *Qo = Qop.ovf + (int64_t)l * E2;
            for (int v = vs; v < V; v += VS) X[v * SB + s] = apply(std::false_type{}, Qd, Qc, Qo, Gh, v);
        }
        bool done = !(gg > 0.0 && gg <= DBL_MAX);  // a zero right-hand side (and a padding sample) keeps x = 0;
                                                   // a non-finite one is left to k_rhs_unrange
        bool fresh = LRN && !done;
        bool lz = LRN;            // the operator preconditioner is in use
        bool switched = !LRN;
        double rz = t0[1], rr = gg, rh = t0[1], rel = done ? 0.0 : 1.0;
        int it = 0, its_s = 0;
        if (vs == 0) {
            flag[0][s] = !done;
            flag[1][s] = fresh;
        }
        for (;;) {
            __syncthreads();  // p and x^ complete; the flags of the last decisions visible
            bool any_act = false, any_fresh = false;
#pragma unroll
            for (int k = 0; k < SB; ++k) {
                any_act |= flag[0][k] != 0;
                any_fresh |= flag[1][k] != 0;
            }
            if (!any_act) break;
            if (!switched && it == switch_at) {  // fallback after maxit / 2 iterations: Jacobi from the current iterate
                switched = true;
                if (!done && lz) {
                    lz = false;
                    fresh = true;
                }
                any_fresh = true;
            }
            if (any_fresh) {
                // r^ = g^ - S^ x^; the systems that asked test it and, if they go on,
                // restart from it (z^ and p from the true residual)
                double t[3] = {0.0, 0.0, 0.0};  // r^.z^, ||g - S x||^2, ||r^||^2
#pragma unroll 1
                for (int v = vs; v < V; v += VS) {
                    if (!fresh) break;
                    const int i = v * SB + s;
                    const double rv = Gh[i] - applyS(X, v);
                    const double ru = rv / H[v];
                    R[i] = rv;
                    t[1] += ru * ru;
                    t[2] += rv * rv;
                    if (!lz) {
                        P[i] = rv;
                        t[0] += rv * rv;
                    }
                }
                if (LRN) {
                    __syncthreads();  // r^ complete: the preconditioner reads neighbours
#pragma unroll 1
                    for (int v = vs; v < V; v += VS) {
                        if (!(fresh && lz)) break;
                        const int i = v * SB + s;
                        const double zv = applyP(R, v);
                        P[i] = zv;
                        t[0] += R[i] * zv;
                    }
                }
                ssum(t);
                if (fresh) {
                    fresh = false;
                    rel = sqrt(t[1] / gg);
                    if (t[1] <= tol2) {
                        done = true;
                        its_s = it;
                    } else {
                        if (t[2] > 0.0) thr = tol2 * t[2] / t[1];
                        rz = t[0];
                        rr = t[1];
                        rh = t[2];
                    }
                }
                if (vs == 0) {
                    flag[0][s] = !done;
                    flag[1][s] = 0;
                }
                continue;
            }
            if (it == maxit) break;  // the systems still active did not converge
            ++it;
            double t1[1] = {0.0};  // p.q
#pragma unroll 1
            for (int v = vs; v < V; v += VS) {
                if (done) break;
                const int i = v * SB + s;
                const double qv = applyS(P, v);
                Q[i] = qv;
                t1[0] += P[i] * qv;
            }
            ssum(t1);
            const double alpha = done ? 0.0 : rz / t1[0];
            double t2[2] = {0.0, 0.0};  // ||r^||^2, r^.z^ (x^ is updated with p below)
#pragma unroll 1
            for (int v = vs; v < V; v += VS) {
                if (done) break;
                const int i = v * SB + s;
                const double rv = R[i] - alpha * Q[i];
                R[i] = rv;
                t2[0] += rv * rv;
            }
            if (LRN) {
                __syncthreads();  // r^ complete: the preconditioner reads neighbours
#pragma unroll 1
                for (int v = vs; v < V; v += VS) {
                    if (done || !lz) break;
                    const int i = v * SB + s;
                    const double zv = applyP(R, v);
                    Q[i] = zv;  // q is free until the next product
                    t2[1] += R[i] * zv;
                }
            }
            ssum(t2);
            if (!done) {
                if (t2[0] <= thr) {
                    fresh = true;  // test with the true residual (and restart if it fails)
#pragma unroll 1
                    for (int v = vs; v < V; v += VS) {
                        const int i = v * SB + s;
                        X[i] += alpha * P[i];
                    }
                } else {
                    rel = sqrt(t2[0] * rr / (rh > 0.0 ? rh : 1.0) / gg);  // estimate
                    const double rzn = (LRN && lz) ? t2[1] : t2[0];
                    const double beta = rzn / rz;
                    rz = rzn;
#pragma unroll 1
                    for (int v = vs; v < V; v += VS) {
                        const int i = v * SB + s;
                        const double pv = P[i];
                        X[i] += alpha * pv;
                        P[i] = ((LRN && lz) ? Q[i] : R[i]) + beta * pv;
                    }
                }
            }
            if (vs == 0) {
                flag[0][s] = !done;
                flag[1][s] = fresh;
            }
        }
        // x = H x^ (each entry read by the thread that wrote it), back in vertex order
        if (live) {
            double *xo = xT + ((int64_t)l * S + smp) * mv.V;
            for (int v = vs; v < V; v += VS) xo[mv.pvtx[u0 + v]] = (gg > 0.0) ? H[v] * X[v * SB + s] : 0.0;
            if (vs == 0) {
                const int64_t sys = ((int64_t)gi * LB + l) * S + smp;
                its[sys] = done ? its_s : maxit + 1;
                res[sys] = rel;
            }
        }
    }
}

// Sum of NV <= 3 values over a workgroup of TPB threads, every thread getting
// the result (combined in a fixed order: deterministic).  Two LDS buffers taken
// in turn: a buffer is written again only two sums later, after every thread
// has passed the barrier of the sum in between, so each sum needs one barrier.
// A single wavefront sums with shuffles alone.
template <int TPB>
struct GroupSum {
    double *lds;  // [2][3][16]
    int buf;
    template <int NV>
    __device__ __forceinline__ void operator()(double (&v)[NV]) {
        static_assert(NV <= 3, "three values per sum");
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
        if constexpr (TPB > 64) {
            // every block of NW lanes takes the NW wavefront partials (lane w
            // of a block: wavefront w's), then a butterfly within the block:
            // every lane ends with the same total, two registers per value
            constexpr int NW = TPB / 64;
            double *r = lds + buf * 48;
            const int lane = threadIdx.x & 63;
            if (lane == 0)
#pragma unroll
                for (int i = 0; i < NV; ++i) r[i * 16 + (threadIdx.x >> 6)] = v[i];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                double t = r[i * 16 + (lane & (NW - 1))];
#pragma unroll
                for (int o = NW / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
                v[i] = t;
            }
            buf ^= 1;
        }
    }
};

#ifndef GRF_PCG_GROUP
#define GRF_PCG_GROUP 1
#endif
#ifndef GRF_PCG_GROUP20
#define GRF_PCG_GROUP20 GRF_PCG_GROUP
#endif
#ifndef GRF_PCG_OPAQUE_K
#define GRF_PCG_OPAQUE_K 4
#endif

// A group of G items of this thread: graph-local vertices t + TPB i (i0 <= i <
// i0 + G).  The items of a group are processed without control flow between
// them (indices past the graph are clamped to its last vertex for the loads,
// their results masked and their stores skipped), so that their loads are in
// flight together.  With K >= GRF_PCG_OPAQUE_K items per thread the index is
// made opaque, so that the compiler reads the operator rows again in every
// iteration (from L2) instead of holding K rows in registers, which would spill.
template <int TPB, int K, int G>
struct ItemGroup {
    int v[G], vc[G];
    bool ok[G];
    __device__ __forceinline__ ItemGroup(int i0, int nv) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            int t = (int)threadIdx.x + TPB * (i0 + g);
            if constexpr (K >= GRF_PCG_OPAQUE_K) {
                if (g == 0) __builtin_amdgcn_sched_barrier(0);
                asm volatile("" : "+v"(t));
            }
            v[g] = t;
            ok[g] = t < nv;
            vc[g] = min(t, nv - 1);
        }
    }
};

// Whether the wavefront owns any vertex of item group i0 (uniform over the
// wavefront: a scalar branch skips the groups past the graph).
template <int TPB>
__device__ __forceinline__ bool group_live(int i0, int nv) {
    const int w0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~63u));
    return w0 + TPB * i0 < nv;
}

// (Op y) at the G items i0 .. i0+G-1 of a group (y graph-local; 0 at masked
// items): the row is one 8-byte load of 16-bit local neighbour ids and two
// 16-byte coefficient loads (UNIT: unit diagonal, no diagonal load).  The CSR
// slots past the first four (degree > 4) are added only for the items whose
// bit is set in the wavefront's overflow mask om (a scalar test: no branch
// waits on a vector load).
template <int G, bool UNIT>
__device__ __forceinline__ void ell_group(const MeshView &mv, const double *__restrict__ dg,
                                          const double *__restrict__ cf, const double *__restrict__ of,
                                          const double *y, const int (&vc)[G], const bool (&ok)[G], int u0,
                                          uint32_t om, int i0, double (&out)[G]) {
    double acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int u = u0 + vc[g];
        const uint2 nb = mv.ell16[u];
        const double2 c01 = *reinterpret_cast<const double2 *>(cf + 4 * (int64_t)u);
        const double2 c23 = *reinterpret_cast<const double2 *>(cf + 4 * (int64_t)u + 2);
        double a = UNIT ? y[vc[g]] : dg[u] * y[vc[g]];
        a += c01.x * y[nb.x & 0xffffu];
        a += c01.y * y[nb.x >> 16];
        a += c23.x * y[nb.y & 0xffffu];
        a += c23.y * y[nb.y >> 16];
        acc[g] = a;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if ((om >> (i0 + g)) & 1u) {
            const int u = u0 + vc[g];
            const int d = mv.deg[u];
            const int64_t k0 = mv.vptr[u];
            for (int64_t k = k0 + 4; k < k0 + d; ++k) acc[g] += of[k] * y[mv.adj_o[k] - u0];
        }
        out[g] = ok[g] ? acc[g] : 0.0;
    }
}

// The slots past the first four of graph gi's vertices of degree > 4 (MeshView::ovent)
// applied to y (graph-local, in LDS) with the coefficients cf (CSR slot order), spread
// over the whole workgroup: wavefront w takes chunks w, w + NW, ... of 64 entries, lane
// j entry j.  The lanes of one piece sum their products in a fixed order (a segmented
// inclusive scan over the lanes, pieces being contiguous), and the last lane of the
// piece stores the sum in psum[piece] (LDS), so the result does not depend on timing.
// With DOT each lane also adds y[row] * cf * y[nb] to dot: the overflow part of
// y . (Op y), which then needs no second pass.  The owner of a vertex adds its pieces
// (ovf_add) once the workgroup has passed a barrier.
template <int TPB, bool DOT>
__device__ __forceinline__ void ovf_pieces(const MeshView &mv, int gi, const double *__restrict__ cf, const double *y,
                                           double *psum, double &dot) {
    constexpr int NW = TPB / 64;
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    const int e0 = mv.ovent0[gi];
    const int nch = (mv.ovent0[gi + 1] - e0) >> 6;
    for (int c = w; c < nch; c += NW) {
        const int4 en = mv.ovent[e0 + 64 * c + lane];  // (slot, piece, row, neighbour)
        double v = en.y >= 0 ? cf[en.x] * y[en.w] : 0.0;
        if (DOT) dot += y[en.z] * v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double t = __shfl_up(v, o, 64);
            const int pt = __shfl_up(en.y, o, 64);
            if (lane >= o && pt == en.y) v += t;
        }
        const int pn = __shfl_down(en.y, 1, 64);
        if (en.y >= 0 && (lane == 63 || pn != en.y)) psum[en.y] = v;
    }
}

// out[i0 + g] += the pieces of the G items of a group (a vertex of degree <= 4 has none)
template <int G, int K>
__device__ __forceinline__ void ovf_add(const MeshView &mv, const double *psum, const int (&vc)[G],
                                        const bool (&ok)[G], int u0, double (&out)[K], int i0) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int2 pc = mv.ovpc[u0 + vc[g]];
        double a = 0.0;
        for (int p = pc.x; p < pc.y; ++p) a += psum[p];
        if (ok[g]) out[i0 + g] += a;
    }
}

// The same solve with the search direction p in LDS, for the graphs glist[0 ..
// ngl-1] of at most cap <= TPB K vertices: one workgroup per (graph, shift,
// sample) system, thread t owning the graph-local vertices t + TPB i (i < K),
// whose r^ and q = S^ p (and x^ unless XG) stay in registers.  XG keeps x^ in
// its output row of xT instead (the largest class, where K doubles fewer
// registers decide whether the kernel spills), updated by FP64 atomic adds
// that return nothing, so no wavefront waits on the row (x^ has one writer per
// entry, its owner thread, so the sum is the same as in registers).  LRN: an
// operator preconditioner z^ = P^ r^ (learned or Neumann-Neumann) and the
// initial guess x^0 = Q^ g^ (learned; 0 when Qop.diag is null); P^ reads the
// neighbours' residuals, so r^ is also kept in LDS (2 cap doubles).  XP (the
// largest class, whose p fills the LDS): the learned initial guess only, with
// the Jacobi preconditioner.  The operator
// rows (EllOp) are read from global memory; the workgroups of one (graph,
// shift) are sent to one XCD (block b goes to XCD b mod 8), so its L2 serves the
// rows to all of that shift's samples.  Three barriers per Jacobi iteration
// (four with the learned preconditioner); the update reads nothing from HBM.
template <int TPB, int K, bool LRN, bool XG, bool XP>
__global__ void __launch_bounds__(TPB) k_pcg_chip(MeshView mv, EllOp Sop, EllOp Pop, EllOp Qop,
                                                  const int32_t *__restrict__ glist, int32_t ngl, int32_t cap,
                                                  int32_t ldsd, const double *__restrict__ gT,
                                                  double *__restrict__ xT,
                                                  int32_t *__restrict__ its,
                                                  double *__restrict__ res, int32_t LB, int64_t S, double tol,
                                                  int32_t maxit) {
    constexpr int G = K < GRF_PCG_OPAQUE_K ? K : (K >= 20 ? GRF_PCG_GROUP20 : GRF_PCG_GROUP);
    static_assert(K % G == 0, "items per thread: a multiple of the group size");
    static_assert(!XP || LRN, "initial guess only: a learned variant");
    constexpr bool LP = LRN && !XP;  // the operator preconditioner is applied
    using IG = ItemGroup<TPB, K, G>;
    extern __shared__ double sv[];  // p [cap], r [cap] (LP)
    __shared__ double red[96];
    __shared__ double dump;  // target of the stores of masked items (no branch per store)
    // block -> (group = (graph, shift), sample): the S blocks of a group share b mod 8
    const int64_t b = blockIdx.x;
    const int64_t grp = (b / (8 * S)) * 8 + (b & 7);
    const int64_t smp = (b % (8 * S)) >> 3;
    if (grp >= (int64_t)ngl * LB) return;  // padding group (whole workgroup)
    const int c = (int)(grp / LB), l = (int)(grp - (int64_t)c * LB);
    const int gi = glist[c];
    const int u0 = mv.gv0[gi], nv = mv.gv0[gi + 1] - u0;
    const int64_t E2 = 2 * (int64_t)mv.E;
    const double *g = gT + ((int64_t)l * S + smp) * mv.V + u0;
    double *xo = xT + ((int64_t)l * S + smp) * mv.V + u0;
    const double *Sc = Sop.coef + (int64_t)l * 4 * mv.V, *So = Sop.ovf + (int64_t)l * E2,
                 *H = Sop.dh + (int64_t)l * mv.V + u0;
    const double *Pd = LRN ? Pop.diag + (int64_t)l * mv.V : nullptr;
    const double *Pc = LRN ? Pop.coef + (int64_t)l * 4 * mv.V : nullptr;
    const double *Po = LRN ? Pop.ovf + (int64_t)l * E2 : nullptr;
    double *ps = sv, *rs = sv + cap;
    const uint32_t om_all = mv.ovfm[16 * (int64_t)gi + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6))];
    // Jacobi-preconditioned iterations spread the overflow slots of the S^ products over
    // the workgroup (ovf_pieces) when the piece sums fit in LDS past p; otherwise (and for
    // every P^ and Q^ product) the owner of a vertex adds its own overflow slots
    // (with the operator preconditioner the piece sums sit past p inside p's region, r follows
    // it; there they pay except in the 512-thread class: measured on the 64-graph batch with
    // the learned operator, class 2 13.0 against 14.9 ms, class 3 57.1 against 52.9 ms,
    // class 4 40.6 against 69.5 ms)
    const int npc = (LP && TPB == 512) ? 0 : mv.ovnp[gi];
    const bool dov = npc > 0 && nv + npc <= (LP ? cap : ldsd);
    const uint32_t om = dov ? 0u : om_all;
    double *psum = ps + nv;
    GroupSum<TPB> gsum{red, 0};
    double x[XG ? 1 : K], r[K], q[K];

    // r^ = g^ - S^ x^, z^ = M r^ (M = P^ if lz, else the identity: Jacobi on S) and
    // p = z^; returns (r^.z^, ||g - S x||^2, ||r^||^2).  Every earlier read of p and r
    // in LDS is behind the barrier of an earlier sum.
    auto restart = [&](bool lz, double &rz, double &rr, double &rh) {
#pragma unroll
        for (int i0 = 0; i0 < K; i0 += G) {
            if (!group_live<TPB>(i0, nv)) continue;
            const IG it(i0, nv);
#pragma unroll
            for (int e = 0; e < G; ++e) {
                double xv;
                if constexpr (XG)
                    xv = unsafeAtomicAdd(&xo[it.vc[e]], 0.0);  // ordered after this thread's updates
                else
                    xv = x[i0 + e];
                *(it.ok[e] ? &ps[it.v[e]] : &dump) = xv;
            }
        }
        __syncthreads();  // x^ in LDS
        double t[3] = {0.0, 0.0, 0.0};
        if (dov) {  // the overflow pieces of S^ x^, complete for every owner below
            double unused = 0.0;
            ovf_pieces<TPB, false>(mv, gi, So, ps, psum, unused);
            __syncthreads();
        }
#pragma unroll
        for (int i0 = 0; i0 < K; i0 += G) {
            if (!group_live<TPB>(i0, nv)) continue;
            const IG it(i0, nv);
            double sx[G];
            ell_group<G, true>(mv, nullptr, Sc, So, ps, it.vc, it.ok, u0, om, i0, sx);
            if (dov && ((om_all >> i0) & 1u)) ovf_add<G, G>(mv, psum, it.vc, it.ok, u0, sx, 0);
#pragma unroll
            for (int e = 0; e < G; ++e) {
                const double h = H[it.vc[e]];
                const double rv = it.ok[e] ? h * g[it.vc[e]] - sx[e] : 0.0;
                const double ru = rv / h;
                r[i0 + e] = rv;
                t[1] += ru * ru;
                t[2] += rv * rv;
                if (!lz) {
                    q[i0 + e] = rv;
                    t[0] += rv * rv;
                }
            }
        }
        if (LP && lz) {
#pragma unroll
            for (int i0 = 0; i0 < K; i0 += G) {
                if (!group_live<TPB>(i0, nv)) continue;
                const IG it(i0, nv);
#pragma unroll
                for (int e = 0; e < G; ++e) *(it.ok[e] ? &rs[it.v[e]] : &dump) = r[i0 + e];
            }
            __syncthreads();  // r^ in LDS
#pragma unroll
            for (int i0 = 0; i0 < K; i0 += G) {
                if (!group_live<TPB>(i0, nv)) continue;
                const IG it(i0, nv);
                double z[G];
                ell_group<G, false>(mv, Pd, Pc, Po, rs, it.vc, it.ok, u0, om_all, i0, z);  // owners add overflow
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    q[i0 + e] = z[e];
                    t[0] += r[i0 + e] * z[e];
                }
            }
        }
        gsum(t);  // also: every read of x^ in LDS done
#pragma unroll
        for (int i0 = 0; i0 < K; i0 += G) {
            if (!group_live<TPB>(i0, nv)) continue;
            const IG it(i0, nv);
#pragma unroll
            for (int e = 0; e < G; ++e) *(it.ok[e] ? &ps[it.v[e]] : &dump) = q[i0 + e];
        }
        rz = t[0];
        rr = t[1];
        rh = t[2];
    };

    // ||g||^2 and ||g^||^2; Jacobi: x^0 = 0, r^ = p = g^; LRN: x^0 = Q^ g^ (g^ staged in LDS) or 0
    double rz, rr, rh, gg;
    {
        double t[2] = {0.0, 0.0};
#pragma unroll
        for (int i0 = 0; i0 < K; i0 += G) {
            if (!group_live<TPB>(i0, nv)) continue;
            const IG it(i0, nv);
#pragma unroll
            for (int e = 0; e < G; ++e) {
                const int i = i0 + e;
                const double gv = it.ok[e] ? g[it.vc[e]] : 0.0;
                const double gh = H[it.vc[e]] * gv;
                t[0] += gv * gv;
                t[1] += gh * gh;
                q[i] = 0.0;
                r[i] = LRN ? 0.0 : gh;
                *(it.ok[e] ? &ps[it.v[e]] : &dump) = gh;
                if constexpr (XG) {
                    if (it.ok[e]) xo[it.v[e]] = 0.0;
                } else {
                    x[i] = 0.0;
                }
            }
        }
        if (LRN && Qop.diag != nullptr) {
            __syncthreads();  // g^ in LDS
#pragma unroll
            for (int i0 = 0; i0 < K; i0 += G) {
                if (!group_live<TPB>(i0, nv)) continue;
                const IG it(i0, nv);
                double xq[G];
                ell_group<G, false>(mv, Qop.diag + (int64_t)l * mv.V, Qop.coef + (int64_t)l * 4 * mv.V,
                                    Qop.ovf + (int64_t)l * E2, ps, it.vc, it.ok, u0, om_all, i0, xq);
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    if constexpr (XG) {
                        if (it.ok[e]) xo[it.v[e]] = xq[e];
                    } else {
                        x[i0 + e] = xq[e];
                    }
                }
            }
        }
        gsum(t);  // also: every read of g^ in LDS done
        gg = t[0];
        rr = gg;
        rh = t[1];
        rz = t[1];
    }
    const double tol2 = tol * tol * gg;
    double thr = tol * tol * rh;  // trigger on the scaled residual, corrected at each test
    int it_n = 0;
    double rel = 1.0;
    bool lz = LP;       // the operator preconditioner is in use
    bool fresh = LRN;   // r^, z^ and p are to be recomputed from x^
    const int switch_at = max(1, maxit / 2);
    if (gg > 0.0 && gg <= DBL_MAX) {  // a non-finite right-hand side is left to k_rhs_unrange
        for (;;) {
            if (fresh) {  // the only convergence test: the residual recomputed from x
                restart(lz, rz, rr, rh);
                fresh = false;
                rel = sqrt(rr / gg);
                if (rr <= tol2) break;
                if (rh > 0.0) thr = tol2 * rh / rr;
            }
            if (it_n == maxit) {  // flags non-convergence
                it_n = maxit + 1;
                break;
            }
            if (LP && lz && it_n == switch_at) {  // fallback after maxit / 2 iterations: Jacobi from the current iterate
                lz = false;
                fresh = true;
                continue;
            }
            ++it_n;
            __syncthreads();  // p complete
            double t1[1] = {0.0};
            if (dov) ovf_pieces<TPB, true>(mv, gi, So, ps, psum, t1[0]);  // before q is live
#pragma unroll
            for (int i0 = 0; i0 < K; i0 += G) {
                if (!group_live<TPB>(i0, nv)) continue;
                const IG it(i0, nv);
                double sp[G];
                ell_group<G, true>(mv, nullptr, Sc, So, ps, it.vc, it.ok, u0, om, i0, sp);
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    q[i0 + e] = sp[e];
                    t1[0] += ps[it.vc[e]] * sp[e];
                }
            }
            gsum(t1);  // also: the piece sums complete
            if (dov) {
#pragma unroll
                for (int i0 = 0; i0 < K; i0 += G) {
                    if (!group_live<TPB>(i0, nv) || !((om_all >> i0) & 1u)) continue;
                    const IG it(i0, nv);
                    ovf_add<G, K>(mv, psum, it.vc, it.ok, u0, q, i0);
                }
            }
            const double alpha = rz / t1[0];
            double t3[1] = {0.0};  // ||r^||^2 (= r^.z^ for Jacobi)
#pragma unroll
            for (int i0 = 0; i0 < K; i0 += G) {
                if (!group_live<TPB>(i0, nv)) continue;
                const IG it(i0, nv);
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    const int i = i0 + e;
                    const double pv = ps[it.vc[e]];
                    if constexpr (XG) {  // no return value: the wavefront does not wait (+0 at masked items)
                        unsafeAtomicAdd(&xo[it.vc[e]], it.ok[e] ? alpha * pv : 0.0);
                    } else {
                        x[i] += alpha * pv;
                    }
                    r[i] -= alpha * q[i];  // 0 at masked items
                    t3[0] += r[i] * r[i];
                    if (!lz) q[i] = r[i];  // z^ = r^, kept in q for the direction update
                    if (LP && lz) *(it.ok[e] ? &rs[it.v[e]] : &dump) = r[i];
                }
            }
            gsum(t3);
            if (t3[0] <= thr) {  // test with the true residual (and restart if it fails)
                fresh = true;
                continue;
            }
            rel = sqrt(t3[0] * rr / (rh > 0.0 ? rh : 1.0) / gg);  // estimate
            double rz_new = t3[0];
            if (LP && lz) {
                double t4[1] = {0.0};
                // the overflow slots of P^ r^ spread over the workgroup as for S^ p (r^ is
                // complete in LDS behind the last sum; the S^ pieces were added before it)
                if (dov) ovf_pieces<TPB, true>(mv, gi, Po, rs, psum, t4[0]);
#pragma unroll
                for (int i0 = 0; i0 < K; i0 += G) {
                    if (!group_live<TPB>(i0, nv)) continue;
                    const IG it(i0, nv);
                    double z[G];
                    ell_group<G, false>(mv, Pd, Pc, Po, rs, it.vc, it.ok, u0, om, i0, z);
#pragma unroll
                    for (int e = 0; e < G; ++e) {
                        q[i0 + e] = z[e];
                        t4[0] += r[i0 + e] * z[e];
                    }
                }
                gsum(t4);  // also: the piece sums complete
                if (dov) {
#pragma unroll
                    for (int i0 = 0; i0 < K; i0 += G) {
                        if (!group_live<TPB>(i0, nv) || !((om_all >> i0) & 1u)) continue;
                        const IG it(i0, nv);
                        ovf_add<G, K>(mv, psum, it.vc, it.ok, u0, q, i0);
                    }
                }
                rz_new = t4[0];
            }
            const double beta = rz_new / rz;
            rz = rz_new;
#pragma unroll
            for (int i0 = 0; i0 < K; i0 += G) {
                if (!group_live<TPB>(i0, nv)) continue;
                const IG it(i0, nv);
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    const double pn = q[i0 + e] + beta * ps[it.vc[e]];  // q = z^
                    *(it.ok[e] ? &ps[it.v[e]] : &dump) = pn;
                }
            }
        }
    } else {
        rel = 0.0;
    }
    // x = H x^
    if constexpr (XG) __syncthreads();  // the atomic updates of the row are complete
#pragma unroll
    for (int i0 = 0; i0 < K; i0 += G) {
        if (!group_live<TPB>(i0, nv)) continue;
        const IG it(i0, nv);
#pragma unroll
        for (int e = 0; e < G; ++e) {
            double xv;
            if constexpr (XG)
                xv = unsafeAtomicAdd(&xo[it.vc[e]], 0.0);
            else
                xv = x[i0 + e];
            const double xs = H[it.vc[e]] * xv;
            if (it.ok[e]) xo[it.v[e]] = xs;
        }
    }
    if (threadIdx.x == 0) {
        const int64_t sys = ((int64_t)gi * LB + l) * S + smp;
        its[sys] = it_n;
        res[sys] = rel;
    }
}

// ug[l][v][s] = xT[l][s][v] (padded samples 0) and U[b][NI+v][s] += sum_l xT[l][s][v],
// shifts summed in increasing order.
template <typename GT>
__global__ void __launch_bounds__(256) k_vertex_scatter(MeshView mv, const double *__restrict__ xT, int32_t LB,
                                                        int64_t S, int32_t Sp, GT *__restrict__ ug,
                                                        double *__restrict__ U) {
    __shared__ double tile[64][65];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int v0 = blockIdx.x * 64;
    const int b = blockIdx.y;
    // lanes read by the recovery sweeps: the samples rounded up to a 16-sample wavefront
    // (padding lanes among them get 0); lanes past them are not written
    const bool lw = (int64_t)b * 64 + lane < ((S + 15) / 16) * 16;
    double acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0;
    // sample rows of the tile: up to the 16-sample wavefronts of the recovery (0 past S)
    const int64_t rows = min((int64_t)64, ((S - (int64_t)b * 64 + 15) / 16) * 16);
    for (int l = 0; l < LB; ++l) {
        __syncthreads();
        for (int si = wv; si < rows; si += 4) {
            const int64_t s = (int64_t)b * 64 + si;
            const int v = v0 + lane;
            tile[si][lane] = (s < S && v < mv.V) ? xT[((int64_t)l * S + s) * mv.V + v] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int vi = wv + 4 * i;
            const int v = v0 + vi;
            const double val = tile[lane][vi];
            if (v < mv.V && lw) ug[((int64_t)l * mv.V + v) * Sp + (int64_t)b * 64 + lane] = (GT)val;
            acc[i] += val;
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int v = v0 + wv + 4 * i;
        if (v < mv.V && lw) U[((int64_t)b * mv.N + mv.NI + v) * 64 + lane] += acc[i];
    }
}

}  // namespace

// Range of a right-hand side.  The stopping test compares squared norms,
// ||g - S x||^2 <= tol^2 ||g||^2, which underflow when g is tiny.  A load far
// inside an edge reaches the vertices damped like e^{-d theta}, 1e-170 and less
// at strongly mass-dominated shifts.  Before the PCG every (graph, shift,
// sample) system whose sum of |g| lies outside [2^-300, 2^300] has its row
// scaled in place by the power of two 2^e that brings the sum into [1, 2)
// (exact: the solve is unchanged but for the scale), and e is kept.  After the
// PCG both g and x of such a system are scaled back by 2^-e.  Every other
// system keeps e = 0 and is not touched again.  A system whose sum is NaN or
// Inf gets e = kRangeNonFinite instead: the PCG leaves it alone, its x is set
// to NaN afterwards, and the host reports it.  One workgroup per system.
__global__ void __launch_bounds__(256) k_rhs_range(MeshView mv, double *__restrict__ gT, int32_t *__restrict__ gexp,
                                                   int32_t LB, int64_t S) {
    __shared__ double red[16];
    const int64_t sys = blockIdx.x;  // (g * LB + l) * S + s
    const int64_t s = sys % S, l = (sys / S) % LB, gi = sys / (S * LB);
    const int u0 = mv.gv0[gi], V = mv.gv0[gi + 1] - u0;
    double *g = gT + (l * S + s) * mv.V + u0;
    double t[1] = {0.0};
    for (int v = threadIdx.x; v < V; v += blockDim.x) t[0] += fabs(g[v]);
    block_sum<1>(t, red, blockDim.x >> 6);
    const double a = t[0];
    const bool bad = !(a <= DBL_MAX);  // NaN or Inf
    const int e = bad ? 0 : (a > 0.0 && (a < 0x1p-300 || a > 0x1p300)) ? -ilogb(a) : 0;
    if (threadIdx.x == 0) gexp[sys] = bad ? kRangeNonFinite : e;
    if (e != 0)
        for (int v = threadIdx.x; v < V; v += blockDim.x) g[v] = ldexp(g[v], e);
}

__global__ void __launch_bounds__(256) k_rhs_unrange(MeshView mv, double *__restrict__ gT, double *__restrict__ xT,
                                                     const int32_t *__restrict__ gexp, int32_t LB, int64_t S) {
    const int64_t sys = blockIdx.x;
    const int e = gexp[sys];
    if (e == 0) return;
    const int64_t s = sys % S, l = (sys / S) % LB, gi = sys / (S * LB);
    const int u0 = mv.gv0[gi], V = mv.gv0[gi + 1] - u0;
    double *g = gT + (l * S + s) * mv.V + u0, *x = xT + (l * S + s) * mv.V + u0;
    if (e == kRangeNonFinite) {
        for (int v = threadIdx.x; v < V; v += blockDim.x) x[v] = __builtin_nan("");
        return;
    }
    for (int v = threadIdx.x; v < V; v += blockDim.x) {
        g[v] = ldexp(g[v], -e);
        x[v] = ldexp(x[v], -e);
    }
}

size_t pcg_scratch_bytes(const MeshView &mv, int32_t blocks) {
    return (size_t)blocks * 5 * kMrhsSB * (size_t)mv.maxVg * sizeof(double);
}

// diag, dh, coef [4], ovf of each shift, for S^ (and P^, Q^ with the learned preconditioner)
static size_t ell_op_doubles(const MeshView &mv, int32_t LB) {
    return (size_t)LB * (6 * (size_t)mv.V + 2 * (size_t)mv.E);
}

size_t pcg_ops_bytes(const MeshView &mv, int32_t LB, int32_t precond) {
    const int n = precond == GRF_PRECOND_LEARNED ? 3 : precond == GRF_PRECOND_NN ? 2 : 1;  // S^, P^, Q^
    return n * ell_op_doubles(mv, LB) * sizeof(double) + 64;
}

void launch_condense(const MeshView &mv, const SchurArgs &a, hipStream_t st) {
    if (a.LB == 0 || a.S == 0) return;
    GRF_REQUIRE(a.LB < 65536 && a.nb < 65536, "internal: grid too large");
    const dim3 grid((unsigned)((mv.V + 63) / 64), (unsigned)a.nb, (unsigned)a.LB);
    if (a.ends32)  // FP32 end values (mixed precision), summed in FP64
        hipLaunchKernelGGL(k_condense<float>, grid, dim3(256), 0, st, mv, a.X, a.ends32, a.Sp, a.S, a.gT);
    else
        hipLaunchKernelGGL(k_condense<double>, grid, dim3(256), 0, st, mv, a.X, a.ends, a.Sp, a.S, a.gT);
    GRF_LAUNCH_CHECK();
}

// Variant of the on-chip kernel per size class (ChipMode, work.h): CM_OP applies
// the operator preconditioner P^ (and the learned initial guess, if any) with r^
// and p in LDS, which only the classes 0 .. kChipOpClasses - 1 can hold;
// CM_GUESS applies the learned initial guess with the Jacobi preconditioner
// (one vector in LDS); CM_JACOBI is plain Jacobi-PCG.
static_assert(2 * kPcgCap[kChipOpClasses - 1] * 8 <= 160 * 1024 && 2 * kPcgCap[kChipOpClasses] * 8 > 160 * 1024,
              "two FP64 vectors of the class capacity in 160 KiB of LDS");

template <int C, bool LRN, bool XP>
static void chip_launch(const MeshView &mv, const SchurArgs *a, const EllOp *ops, hipStream_t st) {
    constexpr int TPB = kChipTpb[C], K = kChipK[C];
    static_assert(TPB * K >= kPcgCap[C], "class capacity");
    constexpr bool XG = K > 10;
    // p (and r^ with the operator preconditioner); past p, the overflow piece sums of the
    // Jacobi-preconditioned variants (room for half the capacity; the largest class uses
    // what its graph leaves of p's capacity)
    constexpr bool LP = LRN && !XP;
    constexpr int32_t ldsd = kPcgCap[C] * (LP ? 2 : 1) + (LP || C == kPcgClasses - 1 ? 0 : kPcgCap[C] / 2);
    constexpr size_t lds = (size_t)ldsd * sizeof(double);
    static_assert(lds + 1024 <= 160 * 1024, "LDS of the class");
    if (!a) {  // preparation: the dynamic LDS of the variant (not a stream operation)
        GRF_HIP(hipFuncSetAttribute((const void *)k_pcg_chip<TPB, K, LRN, XG, XP>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        return;
    }
    const int32_t n = mv.cls_off[C + 1] - mv.cls_off[C];
    const int64_t groups = (int64_t)n * a->LB;
    const int64_t blocks = (groups + 7) / 8 * 8 * a->S;
    GRF_REQUIRE(blocks < ((int64_t)1 << 31), "too many systems in one shift block");
    hipLaunchKernelGGL((k_pcg_chip<TPB, K, LRN, XG, XP>), dim3((unsigned)blocks), dim3(TPB), lds, st, mv, ops[0],
                       ops[1], ops[2], mv.gord + mv.cls_off[C], n, kPcgCap[C], ldsd, a->gT, a->xT, a->its, a->res,
                       a->LB, a->S, a->tol, a->maxit);
    GRF_LAUNCH_CHECK();
}

template <int C>
static void chip_class(const MeshView &mv, const SchurArgs *a, const EllOp *ops, hipStream_t st, int mode) {
    if (mode == CM_OP) {
        if constexpr (C < kChipOpClasses)
            chip_launch<C, true, false>(mv, a, ops, st);
        else
            GRF_REQUIRE(false, "internal: operator preconditioner in a class without room for it");
    } else if (mode == CM_GUESS) {
        chip_launch<C, true, true>(mv, a, ops, st);
    } else {
        chip_launch<C, false, false>(mv, a, ops, st);
    }
}

static void chip_dispatch(int c, const MeshView &mv, const SchurArgs *a, const EllOp *ops, hipStream_t st,
                          int mode) {
    switch (c) {
    case 0: chip_class<0>(mv, a, ops, st, mode); break;
    case 1: chip_class<1>(mv, a, ops, st, mode); break;
    case 2: chip_class<2>(mv, a, ops, st, mode); break;
    case 3: chip_class<3>(mv, a, ops, st, mode); break;
    case 4: chip_class<4>(mv, a, ops, st, mode); break;
    case 5: chip_class<5>(mv, a, ops, st, mode); break;
    default: GRF_REQUIRE(false, "internal: size class %d", c);
    }
}
static_assert(kPcgClasses == 6, "chip_dispatch covers every class");

void prepare_pcg(const MeshView &mv) {
    static bool done = false;  // the attributes hold for the process (every device)
    if (done) return;
    for (int c = 0; c < kPcgClasses; ++c) {
        chip_dispatch(c, mv, nullptr, nullptr, nullptr, CM_JACOBI);
        chip_dispatch(c, mv, nullptr, nullptr, nullptr, CM_GUESS);
        if (c < kChipOpClasses) chip_dispatch(c, mv, nullptr, nullptr, nullptr, CM_OP);
    }
    done = true;
}

void default_chip_modes(int32_t precond, int8_t *mode) {
    for (int c = 0; c < kPcgClasses; ++c)
        mode[c] = precond == GRF_PRECOND_JACOBI    ? CM_JACOBI
                  : c < kChipOpClasses             ? CM_OP
                  : precond == GRF_PRECOND_NN      ? CM_GLOBAL
                                                   : CM_GUESS;
}

bool chip_mode_valid(int c, int mode) {
    return mode == CM_JACOBI || mode == CM_GUESS || (mode == CM_OP && c < kChipOpClasses);
}

static void launch_mrhs(const MeshView &mv, const SchurArgs &a, const EllOp *ops, bool lrn, int32_t ngl, int c_end,
                        hipStream_t st);

void launch_pcg(const MeshView &mv, const SchurArgs &a, hipStream_t st) {
    if (a.LB == 0 || a.S == 0) return;
    const int32_t pm = a.precond == GRF_PRECOND_LEARNED ? PM_LEARNED : a.precond == GRF_PRECOND_NN ? PM_NN : PM_JACOBI;
    GRF_REQUIRE(pm != PM_LEARNED || a.learned, "internal: learned operators missing");
    const bool lrn = pm != PM_JACOBI;  // an operator preconditioner (the LRN kernels)
    const size_t per = ell_op_doubles(mv, a.LB);
    EllOp ops[3];
    for (int i = 0; i < 3; ++i) {
        double *base = a.ops + (lrn ? i : 0) * per;
        ops[i] = EllOp{base, base + (size_t)a.LB * mv.V, base + 2 * (size_t)a.LB * mv.V,
                       base + 6 * (size_t)a.LB * mv.V};
    }
    if (pm == PM_NN) ops[2] = EllOp{nullptr, nullptr, nullptr, nullptr};  // no initial-guess operator
    const LearnedOps lo = pm == PM_LEARNED ? *a.learned : LearnedOps{};
    const int64_t n = (int64_t)a.LB * mv.V;
    const dim3 eg((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)));
    hipLaunchKernelGGL(k_ell_diag, eg, dim3(256), 0, st, mv, a.sd, a.so, a.LB, ops[0].dh);
    hipLaunchKernelGGL(k_ell_ops, eg, dim3(256), 0, st, mv, a.sd, a.so, a.LB, ops[0], pm, lo, ops[1], ops[2]);
    const int64_t nsys_all = (int64_t)mv.ng * a.LB * a.S;
    GRF_REQUIRE(nsys_all < ((int64_t)1 << 31), "too many systems in one shift block");
    hipLaunchKernelGGL(k_rhs_range, dim3((unsigned)nsys_all), dim3(256), 0, st, mv, a.gT, a.gexp, a.LB, a.S);
    GRF_LAUNCH_CHECK();
    // on-chip classes: Jacobi everywhere; Neumann-Neumann in the classes that hold both
    // vectors (the others take the global-memory kernel); learned: per class as chosen
    int8_t mode[kPcgClasses];
    default_chip_modes(a.precond, mode);
    if (pm == PM_LEARNED && a.cls_mode)
        for (int c = 0; c < kPcgClasses; ++c) mode[c] = a.cls_mode[c];
    const int c_end = pm == PM_NN ? kChipOpClasses : kPcgClasses;
    for (int c = 0; c < c_end; ++c) {
        if (mv.cls_off[c + 1] == mv.cls_off[c]) continue;
        GRF_REQUIRE(chip_mode_valid(c, mode[c]), "internal: PCG variant %d in size class %d", mode[c], c);
        if (a.ctimer) a.ctimer->begin(kClassTimerId + c);
        chip_dispatch(c, mv, &a, ops, st, mode[c]);
        if (a.ctimer) a.ctimer->end();
    }
    // graphs beyond the on-chip classes
    const int32_t ngl = mv.cls_off[kPcgClasses + 1] - mv.cls_off[c_end];
    if (ngl > 0) {
        if (a.ctimer) a.ctimer->begin(kClassTimerId + kPcgClasses);
        launch_mrhs(mv, a, ops, lrn, ngl, c_end, st);
        if (a.ctimer) a.ctimer->end();
    }
    hipLaunchKernelGGL(k_rhs_unrange, dim3((unsigned)nsys_all), dim3(256), 0, st, mv, a.gT, a.xT, a.gexp, a.LB, a.S);
    GRF_LAUNCH_CHECK();
}

static void launch_mrhs(const MeshView &mv, const SchurArgs &a, const EllOp *ops, bool lrn, int32_t ngl, int c_end,
                        hipStream_t st) {
    // four samples per block: on the 98k-vertex random geometric graph, 8 and 16 took
    // 1.6x and 2.5x longer (fewer workgroups), and 8 was slower even at equal workgroup
    // counts (a block runs until its slowest system has converged)
    const int64_t units = (int64_t)ngl * a.LB * ((a.S + kMrhsSB - 1) / kMrhsSB);
    const int64_t blocks = std::min<int64_t>(units, (int64_t)a.pcg_blocks);
    GRF_REQUIRE(blocks >= 1 && blocks < ((int64_t)1 << 31), "internal: no scratch for the multi-system PCG");
    GRF_REQUIRE((int64_t)mv.maxVg * kMrhsSB < ((int64_t)1 << 31), "a graph too large for the vertex PCG");
    const int32_t *glist = mv.gord + mv.cls_off[c_end];
    if (lrn)
        hipLaunchKernelGGL((k_pcg_mrhs<kMrhsSB, true>), dim3((unsigned)blocks), dim3(1024), 0, st, mv, ops[0], ops[1],
                           ops[2], glist, ngl, a.gT, a.xT, a.scr, a.its, a.res, a.LB, a.S, a.tol, a.maxit);
    else
        hipLaunchKernelGGL((k_pcg_mrhs<kMrhsSB, false>), dim3((unsigned)blocks), dim3(1024), 0, st, mv, ops[0], ops[1],
                           ops[2], glist, ngl, a.gT, a.xT, a.scr, a.its, a.res, a.LB, a.S, a.tol, a.maxit);
    GRF_LAUNCH_CHECK();
}

void launch_vertex_scatter(const MeshView &mv, const SchurArgs &a, hipStream_t st) {
    if (a.LB == 0 || a.S == 0) return;
    const dim3 grid((unsigned)((mv.V + 63) / 64), (unsigned)a.nb);
    if (a.ug32)  // FP32 copy for the FP32 recovery sweeps (mixed precision)
        hipLaunchKernelGGL(k_vertex_scatter<float>, grid, dim3(256), 0, st, mv, a.xT, a.LB, a.S, a.Sp, a.ug32, a.U);
    else
        hipLaunchKernelGGL(k_vertex_scatter<double>, grid, dim3(256), 0, st, mv, a.xT, a.LB, a.S, a.Sp, a.ug, a.U);
    GRF_LAUNCH_CHECK();
}

}  // namespace grf
