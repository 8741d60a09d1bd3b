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
// x 64 samples are transposed through LDS so both sides are contiguous.
__global__ void __launch_bounds__(256) k_condense(MeshView mv, const double *__restrict__ X,
                                                  const double *__restrict__ ends, int32_t Sp, int64_t S,
                                                  double *__restrict__ gT) {
    __shared__ double tile[64][65];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int v0 = blockIdx.x * 64;
    const int b = blockIdx.y;
    const int l = blockIdx.z;
    const int64_t E = mv.E;
    for (int vi = wv; vi < 64; vi += 4) {
        const int v = v0 + vi;
        double g = 0.0;
        if (v < mv.V) {
            g = X[((int64_t)b * mv.N + mv.NI + v) * 64 + lane];
            for (int64_t k = mv.vptr[v]; k < mv.vptr[v + 1]; ++k) {
                const int e = mv.adj_e[k];
                const int side = mv.adj_s[k];
                g += ends[(((int64_t)l * E + e) * 2 + side) * Sp + (int64_t)b * 64 + lane];
            }
        }
        tile[vi][lane] = g;
    }
    __syncthreads();
    for (int si = wv; si < 64; si += 4) {
        const int64_t s = (int64_t)b * 64 + si;
        const int v = v0 + lane;
        if (s < S && v < mv.V) gT[((int64_t)l * S + s) * mv.V + v] = tile[lane][si];
    }
}

// (S p)_u over the edge ends at vertex u; p holds the graph's vertices from u0
__device__ __forceinline__ double schur_apply(const MeshView &mv, const double *__restrict__ sdl,
                                              const double *__restrict__ sol, const double *p, int u, int u0) {
    const double pv = p[u - u0];
    double acc = 0.0;
    for (int64_t k = mv.vptr[u]; k < mv.vptr[u + 1]; ++k) {
        const int e = mv.adj_e[k];
        acc += sdl[e] * pv + sol[e] * p[mv.adj_o[k] - u0];
    }
    return acc;
}

// Vertex operators of a shift block in ELL-4 form, for the global-memory PCG:
// (Op y)_u = diag[l][u] y_u + sum_{j<4} coef[l][j][u] y_{ell[j][u]} + sum over the
// CSR slots k >= vptr[u] + 4 of ovf[l][k] y_{adj_o[k]}  (a self-loop's coupling is
// in the diagonal; its slots carry 0).  S is the Schur complement; with the
// learned preconditioner, P = Dh P_hat Dh and Q = Dh Q_hat Dh.
struct EllOp {
    double *diag, *coef, *ovf;  // [LB][V], [LB][4][V], [LB][2E]
};

__global__ void k_ell_ops(MeshView mv, const double *__restrict__ sd, const double *__restrict__ so, int32_t LB,
                          EllOp S, int32_t lrn, LearnedOps lo, EllOp P, EllOp Q) {
    const int64_t n = (int64_t)LB * mv.V;
    const int64_t E2 = 2 * (int64_t)mv.E;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(i / mv.V), u = (int)(i - (int64_t)l * mv.V);
        const double *sdl = sd + (int64_t)l * mv.E, *sol = so + (int64_t)l * mv.E;
        const int64_t k0 = mv.vptr[u], k1 = mv.vptr[u + 1];
        const double dhu = lrn ? lo.Dh[i] : 0.0;
        double d = 0.0;
        for (int64_t k = k0; k < k1; ++k) {
            const int e = mv.adj_e[k];
            const int o = mv.adj_o[k];
            d += sdl[e] + (o == u ? sol[e] : 0.0);
            const double c = (o == u) ? 0.0 : sol[e];
            const int j = (int)(k - k0);
            double cp = 0.0, cq = 0.0;
            if (lrn && o != u) {
                const double dho = lo.Dh[(int64_t)l * mv.V + o];
                cp = dhu * dho * lo.Pq[(int64_t)l * mv.E + e];
                cq = dhu * dho * lo.Qe[(int64_t)l * mv.E + e];
            }
            if (j < 4) {
                S.coef[((int64_t)l * 4 + j) * mv.V + u] = c;
                if (lrn) {
                    P.coef[((int64_t)l * 4 + j) * mv.V + u] = cp;
                    Q.coef[((int64_t)l * 4 + j) * mv.V + u] = cq;
                }
            } else {
                S.ovf[(int64_t)l * E2 + k] = c;
                if (lrn) {
                    P.ovf[(int64_t)l * E2 + k] = cp;
                    Q.ovf[(int64_t)l * E2 + k] = cq;
                }
            }
        }
        for (int j = (int)(k1 - k0); j < 4; ++j) {
            S.coef[((int64_t)l * 4 + j) * mv.V + u] = 0.0;
            if (lrn) {
                P.coef[((int64_t)l * 4 + j) * mv.V + u] = 0.0;
                Q.coef[((int64_t)l * 4 + j) * mv.V + u] = 0.0;
            }
        }
        S.diag[i] = d;
        if (lrn) {
            P.diag[i] = dhu * dhu * lo.Pd[i];
            Q.diag[i] = dhu * dhu * lo.Qd[i];
        }
    }
}

// (Op y)_u for the graph-local vector y (vertex u = u0 + local index)
__device__ __forceinline__ double ell_apply(const MeshView &mv, const double *__restrict__ dg,
                                            const double *__restrict__ cf, const double *__restrict__ of,
                                            const double *y, int u, int u0) {
    double acc = dg[u] * y[u - u0];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc += cf[(int64_t)j * mv.V + u] * y[mv.ell[(int64_t)j * mv.V + u] - u0];
    const int d = mv.deg[u];
    if (d > 4) {
        const int64_t k0 = mv.vptr[u];
        for (int64_t k = k0 + 4; k < k0 + d; ++k) acc += of[k] * y[mv.adj_o[k] - u0];
    }
    return acc;
}

// (Op y) for the four graph-local vertices v0 + i * stride (i < 4) of this thread:
// the ELL loads of all four are issued before any is consumed (indices past the
// graph are clamped to its last vertex and their results ignored).
__device__ __forceinline__ void ell_apply4(const MeshView &mv, const double *__restrict__ dg,
                                           const double *__restrict__ cf, const double *__restrict__ of,
                                           const double *y, int v0, int stride, int V, int u0, double (&out)[4]) {
    int uu[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) uu[i] = u0 + min(v0 + i * stride, V - 1);
    double acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = dg[uu[i]] * y[uu[i] - u0];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            acc[i] += cf[(int64_t)j * mv.V + uu[i]] * y[mv.ell[(int64_t)j * mv.V + uu[i]] - u0];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int d = mv.deg[uu[i]];
        if (d > 4) {
            const int64_t k0 = mv.vptr[uu[i]];
            for (int64_t k = k0 + 4; k < k0 + d; ++k) acc[i] += of[k] * y[mv.adj_o[k] - u0];
        }
        out[i] = acc[i];
    }
}

// One workgroup per (graph, shift, sample) system, vectors in global scratch
// (x, r, p, q: 4 maxVg doubles per resident workgroup).  Systems are numbered
// ((graph * LB) + shift) * S + sample; the vectors of system (g, l, s) are the
// graph's vertex range of gT / xT[l][s].  LRN: the learned preconditioner
// z = P r and initial guess x0 = Q g, with the Jacobi fallback after maxit / 2
// iterations (restart from the current iterate); otherwise Jacobi from x0 = 0.
// Either way the residual recomputed from x decides convergence.
template <bool LRN>
__global__ void __launch_bounds__(256) k_pcg_ell(MeshView mv, EllOp Sop, EllOp Pop, EllOp Qop,
                                                 const double *__restrict__ gT, double *__restrict__ xT,
                                                 double *__restrict__ scr, int32_t *__restrict__ its,
                                                 double *__restrict__ res, int32_t LB, int64_t S, double tol,
                                                 int32_t maxit) {
    __shared__ double red[64];
    const int nw = blockDim.x >> 6;
    double *x = scr + (int64_t)blockIdx.x * 4 * mv.maxVg;
    double *r = x + mv.maxVg, *p = r + mv.maxVg, *q = p + mv.maxVg;
    const int64_t nsys = (int64_t)mv.ng * LB * S;
    const int64_t E2 = 2 * (int64_t)mv.E;
    const int switch_at = max(1, maxit / 2);
    for (int64_t sys = blockIdx.x; sys < nsys; sys += gridDim.x) {
        const int64_t tl = sys / S;
        const int64_t smp = sys - tl * S;
        const int l = (int)(tl % LB);
        const int gi = (int)(tl / LB);
        const int u0 = mv.gv0[gi], V = mv.gv0[gi + 1] - u0;
        const double *g = gT + ((int64_t)l * S + smp) * mv.V + u0;
        const double *Sd = Sop.diag + (int64_t)l * mv.V, *Sc = Sop.coef + (int64_t)l * 4 * mv.V,
                     *So = Sop.ovf + (int64_t)l * E2;
        const double *Pd = LRN ? Pop.diag + (int64_t)l * mv.V : nullptr;
        const double *Pc = LRN ? Pop.coef + (int64_t)l * 4 * mv.V : nullptr;
        const double *Po = LRN ? Pop.ovf + (int64_t)l * E2 : nullptr;
        bool learned = LRN;
        double t0[1] = {0.0};
        for (int v = threadIdx.x; v < V; v += blockDim.x) {
            const int u = u0 + v;
            x[v] = LRN ? ell_apply(mv, Qop.diag + (int64_t)l * mv.V, Qop.coef + (int64_t)l * 4 * mv.V,
                                   Qop.ovf + (int64_t)l * E2, g, u, u0)
                       : 0.0;
            t0[0] += g[v] * g[v];
        }
        block_sum<1>(t0, red, nw);
        const double gg = t0[0];
        const double tol2 = tol * tol * gg;
        int it = 0;
        double rel = 0.0;
        // r = g - S x and z = M r into p; returns (r.z, r.r)
        auto restart = [&](double &rz, double &rr) {
            __syncthreads();  // x complete
            double t[2] = {0.0, 0.0};
            for (int v = threadIdx.x; v < V; v += blockDim.x) {
                const double rv = g[v] - ell_apply(mv, Sd, Sc, So, x, u0 + v, u0);
                r[v] = rv;
                t[1] += rv * rv;
                if (!learned) {
                    const double zv = rv / Sd[u0 + v];
                    p[v] = zv;
                    t[0] += rv * zv;
                }
            }
            if (learned) {
                __syncthreads();  // r complete
                for (int v = threadIdx.x; v < V; v += blockDim.x) {
                    const double zv = ell_apply(mv, Pd, Pc, Po, r, u0 + v, u0);
                    p[v] = zv;
                    t[0] += r[v] * zv;
                }
            }
            block_sum<2>(t, red, nw);
            rz = t[0];
            rr = t[1];
        };
        if (gg > 0.0) {
            double rz, rr;
            restart(rz, rr);
            rel = sqrt(rr / gg);
            if (rr > tol2) {
                for (it = 1; it <= maxit; ++it) {
                    if (learned && it == switch_at) {  // fallback: Jacobi from the current iterate
                        learned = false;
                        restart(rz, rr);
                    }
                    __syncthreads();  // p complete
                    double t1[1] = {0.0};
                    for (int v0 = threadIdx.x; v0 < V; v0 += 4 * blockDim.x) {
                        double qv[4];
                        ell_apply4(mv, Sd, Sc, So, p, v0, blockDim.x, V, u0, qv);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int v = v0 + i * (int)blockDim.x;
                            if (v < V) {
                                q[v] = qv[i];
                                t1[0] += p[v] * qv[i];
                            }
                        }
                    }
                    block_sum<1>(t1, red, nw);
                    const double alpha = rz / t1[0];
                    double t3[2] = {0.0, 0.0};  // r.z (Jacobi), r.r
                    for (int v = threadIdx.x; v < V; v += blockDim.x) {
                        x[v] += alpha * p[v];
                        const double rv = r[v] - alpha * q[v];
                        r[v] = rv;
                        t3[1] += rv * rv;
                        if (!learned) t3[0] += rv * (rv / Sd[u0 + v]);
                    }
                    block_sum<2>(t3, red, nw);
                    if (t3[1] <= tol2) {
                        double rzt, rrt;
                        restart(rzt, rrt);  // true residual, and a fresh direction if it fails
                        rel = sqrt(rrt / gg);
                        if (rrt <= tol2) break;
                        rz = rzt;
                        continue;
                    }
                    rel = sqrt(t3[1] / gg);
                    double rz_new = t3[0];
                    if (learned) {
                        __syncthreads();  // r complete: the preconditioner reads neighbours
                        double t4[1] = {0.0};
                        for (int v0 = threadIdx.x; v0 < V; v0 += 4 * blockDim.x) {
                            double zv[4];
                            ell_apply4(mv, Pd, Pc, Po, r, v0, blockDim.x, V, u0, zv);
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const int v = v0 + i * (int)blockDim.x;
                                if (v < V) {
                                    q[v] = zv[i];  // q is free until the next product
                                    t4[0] += r[v] * zv[i];
                                }
                            }
                        }
                        block_sum<1>(t4, red, nw);
                        rz_new = t4[0];
                    }
                    const double beta = rz_new / rz;
                    rz = rz_new;
                    __syncthreads();  // all reads of p and q done
                    for (int v = threadIdx.x; v < V; v += blockDim.x)
                        p[v] = (learned ? q[v] : r[v] / Sd[u0 + v]) + beta * p[v];
                }
                if (it > maxit) it = maxit + 1;  // flags non-convergence
            }
        }
        __syncthreads();
        double *xo = xT + ((int64_t)l * S + smp) * mv.V + u0;
        for (int v = threadIdx.x; v < V; v += blockDim.x) xo[v] = (gg > 0.0) ? x[v] : 0.0;
        if (threadIdx.x == 0) {
            its[sys] = it;
            res[sys] = rel;
        }
        __syncthreads();
    }
}

// Same algorithm with the vectors on chip, for graphs of at most TPB K
// vertices of degree <= D, fewer than 2^16 vertices and edges, and (2 V + E)
// doubles of LDS.  A workgroup takes a contiguous range of systems (mostly of
// one graph and shift).  LDS holds p, x and the shift's edge coefficients s_o
// of the graph (reloaded when the shift or the graph changes); each thread
// keeps, for its K vertices, the graph-local (neighbour, edge) pairs in CSR
// order packed in 16-bit halves, the Schur diagonal, the Jacobi inverse, r and
// q = S p in registers.  Only g is read and x written in HBM.
template <int K, int TPB, int D>
__global__ void __launch_bounds__(TPB) k_pcg_lds(MeshView mv, const double *__restrict__ sd,
                                                 const double *__restrict__ so, const double *__restrict__ gT,
                                                 double *__restrict__ xT, int32_t *__restrict__ its,
                                                 double *__restrict__ res, int32_t LB, int64_t S, double tol,
                                                 int32_t maxit) {
    extern __shared__ double sv[];  // p [maxVg], x [maxVg], s_o [maxEg]
    __shared__ double red[64];
    const int E = mv.E;
    double *ps = sv, *xs = sv + mv.maxVg, *sos = sv + 2 * mv.maxVg;
    const int nw = blockDim.x >> 6;
    const int64_t nsys = (int64_t)mv.ng * LB * S;
    const int64_t per = (nsys + gridDim.x - 1) / gridDim.x;
    const int64_t sys0 = (int64_t)blockIdx.x * per;
    const int64_t sys1 = min(nsys, sys0 + per);
    uint32_t nbr[K][D];  // local other vertex | local edge << 16
    int nd[K];
    double ds[K], ji[K];
    int gcur = -1, lcur = -1, u0 = 0, V = 0, e0 = 0, Eg = 0;
    for (int64_t sys = sys0; sys < sys1; ++sys) {
        const int64_t tl = sys / S;
        const int64_t smp = sys - tl * S;
        const int l = (int)(tl % LB);
        const int gi = (int)(tl / LB);
        if (gi != gcur) {  // uniform over the workgroup: the graph's adjacency, local ids
            gcur = gi;
            lcur = -1;
            u0 = mv.gv0[gi];
            V = mv.gv0[gi + 1] - u0;
            e0 = mv.ge0[gi];
            Eg = mv.ge0[gi + 1] - e0;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const int v = threadIdx.x + TPB * i;
                nd[i] = 0;
#pragma unroll
                for (int d = 0; d < D; ++d) nbr[i][d] = 0;
                if (v < V) {
                    const int k0 = (int)mv.vptr[u0 + v], k1 = (int)mv.vptr[u0 + v + 1];
                    nd[i] = k1 - k0;
#pragma unroll
                    for (int d = 0; d < D; ++d)
                        if (k0 + d < k1)
                            nbr[i][d] = (uint32_t)(mv.adj_o[k0 + d] - u0) | ((uint32_t)(mv.adj_e[k0 + d] - e0) << 16);
                }
            }
        }
        if (l != lcur) {  // uniform over the workgroup
            lcur = l;
            __syncthreads();  // previous coefficients no longer read
            const double *sdl = sd + (int64_t)l * E + e0;
            const double *sol = so + (int64_t)l * E + e0;
            for (int e = threadIdx.x; e < Eg; e += TPB) sos[e] = sol[e];
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const int v = threadIdx.x + TPB * i;
                double dsum = 0.0, dj = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    if (d < nd[i]) {
                        const int e = (int)(nbr[i][d] >> 16), o = (int)(nbr[i][d] & 0xffff);
                        dsum += sdl[e];
                        dj += (o == v) ? sol[e] : 0.0;
                    }
                }
                ds[i] = dsum;
                ji[i] = (v < V) ? 1.0 / (dsum + dj) : 0.0;
            }
            __syncthreads();  // s_o in LDS
        }
        // (S y)_v, y = sv[yo ..] in LDS, summed in CSR order.  The packed ids are
        // decoded at each use (the empty asm keeps the compiler from hoisting the
        // decoded ids and their LDS addresses out of the loop into registers).
        auto apply = [&](int yo, int i, int v) -> double {
            double acc = ds[i] * sv[yo + v];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                uint32_t pk = nbr[i][d];
                asm volatile("" : "+v"(pk));
                if (d < nd[i]) acc += sos[pk >> 16] * sv[yo + (int)(pk & 0xffff)];
            }
            return acc;
        };
        const double *g = gT + ((int64_t)l * S + smp) * mv.V + u0;
        double r[K], q[K];
        double t2[2] = {0.0, 0.0};
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int v = threadIdx.x + TPB * i;
            r[i] = 0.0;
            q[i] = 0.0;
            if (v < V) {
                const double gv = g[v];
                r[i] = gv;
                const double z = gv * ji[i];
                ps[v] = z;
                xs[v] = 0.0;
                t2[0] += gv * z;
                t2[1] += gv * gv;
            }
        }
        block_sum<2>(t2, red, nw);
        double rz = t2[0];
        const double gg = t2[1];
        const double tol2 = tol * tol * gg;
        int it = 0;
        double rel = 0.0;
        if (gg > 0.0) {
            rel = 1.0;
            for (it = 1; it <= maxit; ++it) {
                __syncthreads();  // p complete
                double t1[1] = {0.0};
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const int v = threadIdx.x + TPB * i;
                    if (v < V) {
                        q[i] = apply(0, i, v);
                        t1[0] += ps[v] * q[i];
                    }
                }
                block_sum<1>(t1, red, nw);
                const double alpha = rz / t1[0];
                double t3[2] = {0.0, 0.0};
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const int v = threadIdx.x + TPB * i;
                    if (v < V) {
                        xs[v] += alpha * ps[v];
                        r[i] -= alpha * q[i];
                        t3[0] += r[i] * r[i] * ji[i];
                        t3[1] += r[i] * r[i];
                    }
                }
                block_sum<2>(t3, red, nw);
                double rz_new = t3[0];
                double beta;
                if (t3[1] <= tol2) {
                    __syncthreads();  // x complete
                    double tt[2] = {0.0, 0.0};
#pragma unroll
                    for (int i = 0; i < K; ++i) {
                        const int v = threadIdx.x + TPB * i;
                        if (v < V) {
                            const double rv = g[v] - apply(mv.maxVg, i, v);
                            r[i] = rv;
                            tt[0] += rv * rv;
                            tt[1] += rv * rv * ji[i];
                        }
                    }
                    block_sum<2>(tt, red, nw);
                    rel = sqrt(tt[0] / gg);
                    if (tt[0] <= tol2) break;
                    rz_new = tt[1];
                    beta = 0.0;
                } else {
                    rel = sqrt(t3[1] / gg);
                    beta = rz_new / rz;
                }
                rz = rz_new;
                __syncthreads();  // every read of p done
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const int v = threadIdx.x + TPB * i;
                    if (v < V) ps[v] = r[i] * ji[i] + beta * ps[v];
                }
            }
            if (it > maxit) it = maxit + 1;
        }
        __syncthreads();  // x complete
        double *xo = xT + ((int64_t)l * S + smp) * mv.V + u0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int v = threadIdx.x + TPB * i;
            if (v < V) xo[v] = (gg > 0.0) ? xs[v] : 0.0;
        }
        if (threadIdx.x == 0) {
            its[sys] = it;
            res[sys] = rel;
        }
        __syncthreads();  // LDS reused by the next system
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

size_t pcg_ops_bytes(const MeshView &mv, int32_t LB, bool learned) {
    return (learned ? 3 : 1) * (size_t)LB * (5 * (size_t)mv.V + 2 * (size_t)mv.E) * sizeof(double) + 64;
}

void launch_condense(const MeshView &mv, const SchurArgs &a, hipStream_t st) {
    if (a.LB == 0 || a.S == 0) return;
    GRF_REQUIRE(a.LB < 65536 && a.nb < 65536, "internal: grid too large");
    hipLaunchKernelGGL(k_condense, dim3((unsigned)((mv.V + 63) / 64), (unsigned)a.nb, (unsigned)a.LB), dim3(256), 0,
                       st, mv, a.X, a.ends, a.Sp, a.S, a.gT);
    GRF_LAUNCH_CHECK();
}

constexpr size_t kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950

// Dynamic LDS needed by the on-chip kernel for this mesh, 0 if it does not fit.
size_t pcg_lds_bytes(const MeshView &mv) {
    const size_t lds = sizeof(double) * (2 * (size_t)mv.maxVg + (size_t)mv.maxEg);
    return lds > kMaxLds - 1024 ? 0 : lds;
}

// Grants the on-chip kernel variant its dynamic LDS (before any graph capture:
// the attribute call is not a stream operation).  Returns false if refused.
template <int K, int TPB, int D>
bool pcg_lds_attr(size_t lds) {
    static size_t granted = 0;  // largest dynamic LDS size granted so far
    if (lds <= granted) return true;
    if (hipFuncSetAttribute((const void *)k_pcg_lds<K, TPB, D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    granted = lds;
    return true;
}

template <int K, int TPB, int D>
static bool pcg_lds_d(const MeshView &mv, const SchurArgs *a, hipStream_t st) {
    const size_t lds = pcg_lds_bytes(mv);
    if (lds == 0 || !pcg_lds_attr<K, TPB, D>(lds)) return false;
    if (!a) return true;  // preparation only
    const int64_t nsys = (int64_t)mv.ng * a->LB * a->S;
    const int64_t blocks = std::min<int64_t>(nsys, 256 * (2048 / TPB));
    hipLaunchKernelGGL((k_pcg_lds<K, TPB, D>), dim3((unsigned)blocks), dim3(TPB), lds, st, mv, a->sd, a->so, a->gT,
                       a->xT, a->its, a->res, a->LB, a->S, a->tol, a->maxit);
    GRF_LAUNCH_CHECK();
    return true;
}

template <int K, int TPB>
static bool pcg_lds(const MeshView &mv, const SchurArgs *a, hipStream_t st) {
    if (mv.max_deg <= 4) return pcg_lds_d<K, TPB, 4>(mv, a, st);
    return pcg_lds_d<K, TPB, 8>(mv, a, st);
}

// the on-chip variant for this mesh (a = null: only grant its LDS); false if none applies
static bool pcg_onchip(const MeshView &mv, const SchurArgs *a, hipStream_t st) {
    // every neighbour of a vertex in registers, 16-bit graph-local vertex and edge ids
    if (!(mv.max_deg <= 8 && mv.maxVg < 65536 && mv.maxEg < 65536)) return false;
    if (mv.maxVg <= 256) return pcg_lds<1, 256>(mv, a, st);
    if (mv.maxVg <= 512) return pcg_lds<2, 256>(mv, a, st);
    if (mv.maxVg <= 1024) return pcg_lds<2, 512>(mv, a, st);
    if (mv.maxVg <= 2048) return pcg_lds<2, 1024>(mv, a, st);
    if (mv.maxVg <= 4096) return pcg_lds<4, 1024>(mv, a, st);
    return false;
}

static void pcg_global(const MeshView &mv, const SchurArgs &a, hipStream_t st) {
    const bool lrn = a.learned != nullptr;
    const size_t per = (size_t)a.LB * (5 * (size_t)mv.V + 2 * (size_t)mv.E);
    EllOp ops[3];
    for (int i = 0; i < 3; ++i) {
        double *base = a.ops + (lrn ? i : 0) * per;
        ops[i] = EllOp{base, base + (size_t)a.LB * mv.V, base + (size_t)a.LB * 5 * mv.V};
    }
    const LearnedOps lo = lrn ? *a.learned : LearnedOps{};
    const int64_t n = (int64_t)a.LB * mv.V;
    hipLaunchKernelGGL(k_ell_ops, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536))),
                       dim3(256), 0, st, mv, a.sd, a.so, a.LB, ops[0], lrn ? 1 : 0, lo, ops[1], ops[2]);
    GRF_LAUNCH_CHECK();
    const int64_t nsys = (int64_t)mv.ng * a.LB * a.S;
    const int64_t blocks = nsys < a.pcg_blocks ? nsys : a.pcg_blocks;
    if (lrn)
        hipLaunchKernelGGL(k_pcg_ell<true>, dim3((unsigned)blocks), dim3(256), 0, st, mv, ops[0], ops[1], ops[2],
                           a.gT, a.xT, a.scr, a.its, a.res, a.LB, a.S, a.tol, a.maxit);
    else
        hipLaunchKernelGGL(k_pcg_ell<false>, dim3((unsigned)blocks), dim3(256), 0, st, mv, ops[0], ops[1], ops[2],
                           a.gT, a.xT, a.scr, a.its, a.res, a.LB, a.S, a.tol, a.maxit);
    GRF_LAUNCH_CHECK();
}

void prepare_pcg(const MeshView &mv) { (void)pcg_onchip(mv, nullptr, nullptr); }

void launch_pcg(const MeshView &mv, const SchurArgs &a, hipStream_t st) {
    if (a.LB == 0 || a.S == 0) return;
    if (a.learned || !pcg_onchip(mv, &a, st)) pcg_global(mv, a, st);
}

void launch_vertex_scatter(const MeshView &mv, const SchurArgs &a, hipStream_t st) {
    if (a.LB == 0 || a.S == 0) return;
    hipLaunchKernelGGL(k_vertex_scatter, dim3((unsigned)((mv.V + 63) / 64), (unsigned)a.nb), dim3(256), 0, st, mv,
                       a.xT, a.LB, a.S, a.Sp, a.ug, a.U);
    GRF_LAUNCH_CHECK();
}

}  // namespace grf
