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
__global__ void __launch_bounds__(256) k_condense(MeshView mv, const double *__restrict__ X,
                                                  const double *__restrict__ ends, int32_t Sp, int64_t S,
                                                  double *__restrict__ gT) {
    __shared__ double tile[64][65];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int v0 = blockIdx.x * 64;
    const int b = blockIdx.y;
    const int l = blockIdx.z;
    const bool real = (int64_t)b * 64 + lane < S;  // padding samples load nothing
    const double *el = ends + (int64_t)l * 2 * mv.E * Sp + (int64_t)b * 64 + lane;  // row 2 e + side
    for (int vb = wv; vb < 64; vb += 16) {
        double g[4] = {0.0, 0.0, 0.0, 0.0};
        if (real) {  // one lane mask per step; inside it no branch until the loads are issued
            int vc[4], id[4][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int v = v0 + vb + 4 * q;
                vc[q] = min(v, mv.V - 1);
                const double x = X[((int64_t)b * mv.N + mv.NI + vc[q]) * 64 + lane];
                g[q] = v < mv.V ? x : 0.0;
#pragma unroll
                for (int j = 0; j < 4; ++j) id[q][j] = v < mv.V ? mv.eend[(int64_t)j * mv.V + vc[q]] : -1;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double e = el[(int64_t)max(id[q][j], 0) * Sp];  // a valid row even past the degree
                    g[q] += id[q][j] >= 0 ? e : 0.0;
                }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int v = v0 + vb + 4 * q;
                if (v < mv.V && mv.deg[vc[q]] > 4)
                    for (int64_t k = mv.vptr[v] + 4; k < mv.vptr[v + 1]; ++k)
                        g[q] += el[(int64_t)(2 * mv.adj_e[k] + mv.adj_s[k]) * Sp];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) tile[vb + 4 * q][lane] = g[q];
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
// Vertex operators of a shift block in ELL-4 form:
// (Op y)_u = diag[l][u] y_u + sum_{j<4} coef[l][u][j] y_{ell[j][u]} + sum over the
// CSR slots k >= vptr[u] + 4 of ovf[l][k] y_{adj_o[k]}  (a self-loop's coupling is
// in the diagonal; its slots carry 0).  For S^ the diagonal is 1 (not stored) and
// dh holds h; for P^ and Q^ diag holds their diagonal.
struct EllOp {
    double *diag, *dh, *coef, *ovf;  // [LB][V], [LB][V], [LB][V][4], [LB][2E]
};

// h = diag(S)^{-1/2} per (shift, vertex)
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
        dh[i] = 1.0 / sqrt(d);
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
        const double *hl = S.dh + (int64_t)l * mv.V;
        const double hu = hl[u];
        const int64_t k0 = mv.vptr[u], k1 = mv.vptr[u + 1];
        const double du = (double)(k1 - k0);
        double pdiag = 0.0;  // PM_NN: sum over the slots of (D^-1 S_e^-1 D^-1)_uu
        for (int64_t k = k0; k < k1; ++k) {
            const int e = mv.adj_e[k];
            const int o = mv.adj_o[k];
            const double c = (o == u) ? 0.0 : hu * sol[e] * hl[o];
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
                    cp = iso / (du * dov * hu * hl[o]);
                }
            }
            const int j = (int)(k - k0);
            if (j < 4) {
                S.coef[((int64_t)l * mv.V + u) * 4 + j] = c;
                if (opP) P.coef[((int64_t)l * mv.V + u) * 4 + j] = cp;
                if (lrn) Q.coef[((int64_t)l * mv.V + u) * 4 + j] = cq;
            } else {
                S.ovf[(int64_t)l * E2 + k] = c;
                if (opP) P.ovf[(int64_t)l * E2 + k] = cp;
                if (lrn) Q.ovf[(int64_t)l * E2 + k] = cq;
            }
        }
        for (int j = (int)(k1 - k0); j < 4; ++j) {
            S.coef[((int64_t)l * mv.V + u) * 4 + j] = 0.0;
            if (opP) P.coef[((int64_t)l * mv.V + u) * 4 + j] = 0.0;
            if (lrn) Q.coef[((int64_t)l * mv.V + u) * 4 + j] = 0.0;
        }
        if (lrn) {
            P.diag[i] = lo.Pd[i];
            Q.diag[i] = lo.Qd[i];
        } else if (pm == PM_NN) {
            P.diag[i] = pdiag / (hu * hu);
        }
    }
}

// (Op y)_u for the graph-local vector y (vertex u = u0 + local index); UNIT: the
// diagonal is 1
template <bool UNIT>
__device__ __forceinline__ double ell_apply(const MeshView &mv, const double *__restrict__ dg,
                                            const double *__restrict__ cf, const double *__restrict__ of,
                                            const double *y, int u, int u0) {
    double acc = UNIT ? y[u - u0] : dg[u] * y[u - u0];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc += cf[4 * (int64_t)u + j] * y[mv.ell[(int64_t)j * mv.V + u] - u0];
    const int d = mv.deg[u];
    if (d > 4) {
        const int64_t k0 = mv.vptr[u];
        for (int64_t k = k0 + 4; k < k0 + d; ++k) acc += of[k] * y[mv.adj_o[k] - u0];
    }
    return acc;
}

// One workgroup per (graph, shift, sample) system of the graphs glist[0 .. ngl-1],
// vectors in global scratch (x^, r^, p, q: 4 maxVg doubles per resident
// workgroup), for graphs too large for the on-chip kernel.  The vectors of
// system (g, l, s) are the graph's vertex range of gT / xT[l][s]; its
// statistics go to its / res[(g * LB + l) * S + s].  LRN: an operator
// preconditioner z^ = P^ r^ (learned or Neumann-Neumann) and the initial guess
// x0^ = Q^ g^ (learned; x0^ = 0 when Qop.diag is null), with the Jacobi
// fallback after maxit / 2 iterations (restart from the current iterate);
// otherwise CG on S^ (Jacobi) from x^ = 0.  Either way the residual g - S x
// recomputed from x decides convergence; the scaled recursive residual only
// triggers that test, at a threshold corrected by the ratio of the true to the
// scaled residual norm measured at the last test.
template <bool LRN>
__global__ void __launch_bounds__(256) k_pcg_ell(MeshView mv, EllOp Sop, EllOp Pop, EllOp Qop,
                                                 const int32_t *__restrict__ glist, int32_t ngl,
                                                 const double *__restrict__ gT, double *__restrict__ xT,
                                                 double *__restrict__ scr, int32_t *__restrict__ its,
                                                 double *__restrict__ res, int32_t LB, int64_t S, double tol,
                                                 int32_t maxit) {
    __shared__ double red[64];
    const int nw = blockDim.x >> 6;
    double *x = scr + (int64_t)blockIdx.x * 4 * mv.maxVg;
    double *r = x + mv.maxVg, *p = r + mv.maxVg, *q = p + mv.maxVg;
    const int64_t nsys = (int64_t)ngl * LB * S;
    const int64_t E2 = 2 * (int64_t)mv.E;
    const int switch_at = max(1, maxit / 2);
    for (int64_t lsys = blockIdx.x; lsys < nsys; lsys += gridDim.x) {
        const int64_t tl = lsys / S;
        const int64_t smp = lsys - tl * S;
        const int l = (int)(tl % LB);
        const int gi = glist[tl / LB];
        const int64_t sys = ((int64_t)gi * LB + l) * S + smp;
        const int u0 = mv.gv0[gi], V = mv.gv0[gi + 1] - u0;
        const double *g = gT + ((int64_t)l * S + smp) * mv.V + u0;
        const double *Sc = Sop.coef + (int64_t)l * 4 * mv.V, *So = Sop.ovf + (int64_t)l * E2,
                     *H = Sop.dh + (int64_t)l * mv.V + u0;
        const double *Pd = LRN ? Pop.diag + (int64_t)l * mv.V : nullptr;
        const double *Pc = LRN ? Pop.coef + (int64_t)l * 4 * mv.V : nullptr;
        const double *Po = LRN ? Pop.ovf + (int64_t)l * E2 : nullptr;
        bool learned = LRN;
        // g^ into r, ||g||^2, ||g^||^2
        double t0[2] = {0.0, 0.0};
        for (int v = threadIdx.x; v < V; v += blockDim.x) {
            const double gh = H[v] * g[v];
            r[v] = gh;
            t0[0] += g[v] * g[v];
            t0[1] += gh * gh;
        }
        block_sum<2>(t0, red, nw);
        const double gg = t0[0];
        const double tol2 = tol * tol * gg;
        double thr = tol * tol * t0[1];  // trigger on ||r^||^2
        const bool hq = LRN && Qop.diag != nullptr;
        for (int v = threadIdx.x; v < V; v += blockDim.x)
            x[v] = hq ? ell_apply<false>(mv, Qop.diag + (int64_t)l * mv.V, Qop.coef + (int64_t)l * 4 * mv.V,
                                         Qop.ovf + (int64_t)l * E2, r, u0 + v, u0)
                      : 0.0;
        int it = 0;
        double rel = 0.0;
        // r^ = g^ - S^ x^ and z^ = M r^ into p; returns (r^.z^, ||r||^2, ||r^||^2)
        auto restart = [&](double &rz, double &rr, double &rh) {
            __syncthreads();  // x^ complete, every read of r done
            double t[3] = {0.0, 0.0, 0.0};
            for (int v = threadIdx.x; v < V; v += blockDim.x) {
                const double rv = H[v] * g[v] - ell_apply<true>(mv, nullptr, Sc, So, x, u0 + v, u0);
                r[v] = rv;
                const double ru = rv / H[v];
                t[1] += ru * ru;
                t[2] += rv * rv;
                if (!learned) {
                    p[v] = rv;
                    t[0] += rv * rv;
                }
            }
            if (learned) {
                __syncthreads();  // r complete
                for (int v = threadIdx.x; v < V; v += blockDim.x) {
                    const double zv = ell_apply<false>(mv, Pd, Pc, Po, r, u0 + v, u0);
                    p[v] = zv;
                    t[0] += r[v] * zv;
                }
            }
            block_sum<3>(t, red, nw);
            rz = t[0];
            rr = t[1];
            rh = t[2];
        };
        if (gg > 0.0) {
            double rz, rr, rh;
            restart(rz, rr, rh);
            rel = sqrt(rr / gg);
            if (rh > 0.0) thr = tol2 * rh / rr;
            if (rr > tol2) {
                for (it = 1; it <= maxit; ++it) {
                    if (learned && it == switch_at) {  // fallback: Jacobi from the current iterate
                        learned = false;
                        restart(rz, rr, rh);
                    }
                    __syncthreads();  // p complete
                    double t1[1] = {0.0};
                    for (int v = threadIdx.x; v < V; v += blockDim.x) {
                        const double qv = ell_apply<true>(mv, nullptr, Sc, So, p, u0 + v, u0);
                        q[v] = qv;
                        t1[0] += p[v] * qv;
                    }
                    block_sum<1>(t1, red, nw);
                    const double alpha = rz / t1[0];
                    double t3[1] = {0.0};  // ||r^||^2 (= r^.z^ for Jacobi)
                    for (int v = threadIdx.x; v < V; v += blockDim.x) {
                        x[v] += alpha * p[v];
                        const double rv = r[v] - alpha * q[v];
                        r[v] = rv;
                        t3[0] += rv * rv;
                    }
                    block_sum<1>(t3, red, nw);
                    if (t3[0] <= thr) {
                        double rzt, rrt, rht;
                        restart(rzt, rrt, rht);  // true residual, and a fresh direction if it fails
                        rel = sqrt(rrt / gg);
                        if (rrt <= tol2) break;
                        if (rht > 0.0) thr = tol2 * rht / rrt;
                        rz = rzt;
                        continue;
                    }
                    rel = sqrt(t3[0] * rr / (rh > 0.0 ? rh : 1.0) / gg);
                    double rz_new = t3[0];
                    if (learned) {
                        __syncthreads();  // r complete: the preconditioner reads neighbours
                        double t4[1] = {0.0};
                        for (int v = threadIdx.x; v < V; v += blockDim.x) {
                            const double zv = ell_apply<false>(mv, Pd, Pc, Po, r, u0 + v, u0);
                            q[v] = zv;  // q is free until the next product
                            t4[0] += r[v] * zv;
                        }
                        block_sum<1>(t4, red, nw);
                        rz_new = t4[0];
                    }
                    const double beta = rz_new / rz;
                    rz = rz_new;
                    __syncthreads();  // all reads of p and q done
                    for (int v = threadIdx.x; v < V; v += blockDim.x) p[v] = (learned ? q[v] : r[v]) + beta * p[v];
                }
                if (it > maxit) it = maxit + 1;  // flags non-convergence
            }
        }
        __syncthreads();
        double *xo = xT + ((int64_t)l * S + smp) * mv.V + u0;
        for (int v = threadIdx.x; v < V; v += blockDim.x) xo[v] = (gg > 0.0) ? H[v] * x[v] : 0.0;
        if (threadIdx.x == 0) {
            its[sys] = it;
            res[sys] = rel;
        }
        __syncthreads();
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
                                                  const double *__restrict__ gT, double *__restrict__ xT,
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
    const uint32_t om = mv.ovfm[16 * (int64_t)gi + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6))];
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
#pragma unroll
        for (int i0 = 0; i0 < K; i0 += G) {
            if (!group_live<TPB>(i0, nv)) continue;
            const IG it(i0, nv);
            double sx[G];
            ell_group<G, true>(mv, nullptr, Sc, So, ps, it.vc, it.ok, u0, om, i0, sx);
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
                ell_group<G, false>(mv, Pd, Pc, Po, rs, it.vc, it.ok, u0, om, i0, z);
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
                                    Qop.ovf + (int64_t)l * E2, ps, it.vc, it.ok, u0, om, i0, xq);
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
    if (gg > 0.0) {
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
            if (LP && lz && it_n + 1 == switch_at) {  // fallback: Jacobi from the current iterate
                lz = false;
                fresh = true;
                continue;
            }
            ++it_n;
            __syncthreads();  // p complete
            double t1[1] = {0.0};
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
            gsum(t1);
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
                gsum(t4);
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
__global__ void __launch_bounds__(256) k_vertex_scatter(MeshView mv, const double *__restrict__ xT, int32_t LB,
                                                        int64_t S, int32_t Sp, double *__restrict__ ug,
                                                        double *__restrict__ U) {
    __shared__ double tile[64][65];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int v0 = blockIdx.x * 64;
    const int b = blockIdx.y;
    double acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0;
    for (int l = 0; l < LB; ++l) {
        __syncthreads();
        for (int si = wv; si < 64; si += 4) {
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
            if (v < mv.V) ug[((int64_t)l * mv.V + v) * Sp + (int64_t)b * 64 + lane] = val;
            acc[i] += val;
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int v = v0 + wv + 4 * i;
        if (v < mv.V) U[((int64_t)b * mv.N + mv.NI + v) * 64 + lane] += acc[i];
    }
}

}  // namespace

size_t pcg_scratch_bytes(const MeshView &mv, int32_t blocks) {
    return (size_t)blocks * 4 * mv.maxVg * sizeof(double);
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
    hipLaunchKernelGGL(k_condense, dim3((unsigned)((mv.V + 63) / 64), (unsigned)a.nb, (unsigned)a.LB), dim3(256), 0,
                       st, mv, a.X, a.ends, a.Sp, a.S, a.gT);
    GRF_LAUNCH_CHECK();
}

// the learned variant keeps two vectors in LDS and runs on the size classes
// 0 .. kChipLearned - 1 only; the Neumann-Neumann preconditioner needs both
// vectors in every class, so its graphs beyond class kChipNN - 1 take the
// global-memory kernel
constexpr int kChipLearned = 6;
constexpr int kChipNN = 5;

// the learned variant of the largest class applies the learned initial guess only (XP)
constexpr bool chip_xp(int c, bool lrn) { return lrn && kChipK[c] > 10; }
static size_t chip_lds(int c, bool lrn) {
    return (size_t)kPcgCap[c] * sizeof(double) * (lrn && !chip_xp(c, lrn) ? 2 : 1);
}

template <int C, bool LRN>
static void chip_class(const MeshView &mv, const SchurArgs *a, const EllOp *ops, hipStream_t st) {
    constexpr int TPB = kChipTpb[C], K = kChipK[C];
    static_assert(TPB * K >= kPcgCap[C], "class capacity");
    constexpr bool XG = K > 10;
    constexpr bool XP = chip_xp(C, LRN);
    const size_t lds = chip_lds(C, LRN);
    if (!a) {  // preparation: the dynamic LDS of the variant (not a stream operation)
        GRF_HIP(hipFuncSetAttribute((const void *)k_pcg_chip<TPB, K, LRN, XG, XP>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        return;
    }
    const int32_t n = mv.cls_off[C + 1] - mv.cls_off[C];
    if (n == 0) return;
    const int64_t groups = (int64_t)n * a->LB;
    const int64_t blocks = (groups + 7) / 8 * 8 * a->S;
    GRF_REQUIRE(blocks < ((int64_t)1 << 31), "too many systems in one shift block");
    hipLaunchKernelGGL((k_pcg_chip<TPB, K, LRN, XG, XP>), dim3((unsigned)blocks), dim3(TPB), lds, st, mv, ops[0],
                       ops[1], ops[2], mv.gord + mv.cls_off[C], n, kPcgCap[C], a->gT, a->xT, a->its, a->res, a->LB,
                       a->S, a->tol, a->maxit);
    GRF_LAUNCH_CHECK();
}

// the classes 0 .. nc - 1
template <bool LRN>
static void chip_all(const MeshView &mv, const SchurArgs *a, const EllOp *ops, hipStream_t st, int nc = kPcgClasses) {
    if (nc > 0) chip_class<0, LRN>(mv, a, ops, st);
    if (nc > 1) chip_class<1, LRN>(mv, a, ops, st);
    if (nc > 2) chip_class<2, LRN>(mv, a, ops, st);
    if (nc > 3) chip_class<3, LRN>(mv, a, ops, st);
    if (nc > 4) chip_class<4, LRN>(mv, a, ops, st);
    if (nc > 5) chip_class<5, LRN>(mv, a, ops, st);
}

void prepare_pcg(const MeshView &mv) {
    static bool done = false;  // the attributes hold for the process (every device)
    if (done) return;
    chip_all<false>(mv, nullptr, nullptr, nullptr);
    chip_all<true>(mv, nullptr, nullptr, nullptr);
    done = true;
}

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
    GRF_LAUNCH_CHECK();
    const int c0 = pm == PM_LEARNED ? kChipLearned : pm == PM_NN ? kChipNN : kPcgClasses;
    if (lrn)
        chip_all<true>(mv, &a, ops, st, c0);
    else
        chip_all<false>(mv, &a, ops, st);
    // graphs beyond the on-chip classes
    const int32_t ngl = mv.cls_off[kPcgClasses + 1] - mv.cls_off[c0];
    if (ngl == 0) return;
    const int64_t nsys = (int64_t)ngl * a.LB * a.S;
    const int64_t blocks = nsys < a.pcg_blocks ? nsys : a.pcg_blocks;
    const int32_t *glist = mv.gord + mv.cls_off[c0];
    if (lrn)
        hipLaunchKernelGGL(k_pcg_ell<true>, dim3((unsigned)blocks), dim3(256), 0, st, mv, ops[0], ops[1], ops[2],
                           glist, ngl, a.gT, a.xT, a.scr, a.its, a.res, a.LB, a.S, a.tol, a.maxit);
    else
        hipLaunchKernelGGL(k_pcg_ell<false>, dim3((unsigned)blocks), dim3(256), 0, st, mv, ops[0], ops[1], ops[2],
                           glist, ngl, a.gT, a.xT, a.scr, a.its, a.res, a.LB, a.S, a.tol, a.maxit);
    GRF_LAUNCH_CHECK();
}

void launch_vertex_scatter(const MeshView &mv, const SchurArgs &a, hipStream_t st) {
    if (a.LB == 0 || a.S == 0) return;
    hipLaunchKernelGGL(k_vertex_scatter, dim3((unsigned)((mv.V + 63) / 64), (unsigned)a.nb), dim3(256), 0, st, mv,
                       a.xT, a.LB, a.S, a.Sp, a.ug, a.U);
    GRF_LAUNCH_CHECK();
}

}  // namespace grf
