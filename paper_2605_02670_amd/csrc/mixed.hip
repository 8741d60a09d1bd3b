// FP64 residual and update kernels of the mixed-precision refinement.
//
// Paper: the shifted system of eq. spde_approx_fem, A = (c_I + c_L kappa_e^2) M_L
// + c_L G with the lumped mass ("Mass Lumping") and the stiffness of "Phase 2".
// Iterative refinement (x <- x + A^{-1}_FP32 (b - A x), residual in FP64) is
// this build's addition; the residual is evaluated row by row on the
// sample-interleaved layout [nb][N][64] (lanes = right-hand sides).
#include <algorithm>

#include "work.h"

namespace grf {
namespace {

// Interior rows of edge e (workgroup (e, b), lane = rhs):
//   (A x)_p = alpha h x_p + (gamma / h)(2 x_p - x_{p-1} - x_{p+1}),
// where x_{-1} / x_m are the tail / head vertex values.
__global__ void __launch_bounds__(64) k_residual_interior(MeshView mv, double cI, double cL,
                                                          const double *__restrict__ B, const double *__restrict__ X,
                                                          double *__restrict__ R) {
    const int e = blockIdx.x;
    const int64_t b = blockIdx.y;
    const int lane = threadIdx.x;
    const int m = mv.m[e];
    if (m == 0) return;
    const double h = mv.he[e];
    const double alpha = cI + cL * mv.kap2[e];
    const double a = alpha * h, c = cL / h;
    const int64_t base = b * mv.N * 64 + lane;
    const int64_t off = mv.off[e];
    double xl = X[base + (mv.NI + mv.eu[e]) * 64];
    double xc = X[base + off * 64];
    for (int p = 0; p < m; ++p) {
        const double xr = (p + 1 < m) ? X[base + (off + p + 1) * 64] : X[base + (mv.NI + mv.ev[e]) * 64];
        const int64_t row = base + (off + p) * 64;
        R[row] = B[row] - (a * xc + c * ((xc - xl) + (xc - xr)));
        xl = xc;
        xc = xr;
    }
}

// Vertex rows (thread = (vertex, lane)): sum over the edge ends at v of
//   alpha h / 2 x_v + (gamma / h)(x_v - x_next), x_next the adjacent node of the edge.
__global__ void __launch_bounds__(256) k_residual_vertex(MeshView mv, double cI, double cL,
                                                         const double *__restrict__ B, const double *__restrict__ X,
                                                         double *__restrict__ R) {
    const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t b = blockIdx.y;
    const int lane = threadIdx.x & 63;
    if (v >= mv.V) return;
    const int64_t base = b * mv.N * 64 + lane;
    const double xv = X[base + (mv.NI + v) * 64];
    double acc = 0.0;
    for (int64_t k = mv.vptr[v]; k < mv.vptr[v + 1]; ++k) {
        const int e = mv.adj_e[k];
        const double h = mv.he[e];
        const double alpha = cI + cL * mv.kap2[e];
        const int m = mv.m[e];
        int64_t nxt;
        if (m == 0)
            nxt = mv.NI + mv.adj_o[k];
        else
            nxt = mv.off[e] + (mv.adj_s[k] == 0 ? 0 : m - 1);
        acc += 0.5 * alpha * h * xv + (cL / h) * (xv - X[base + nxt * 64]);
    }
    const int64_t row = base + (mv.NI + v) * 64;
    R[row] = B[row] - acc;
}

// Y += X over n doubles
__global__ void k_axpy1(const double *__restrict__ X, double *__restrict__ Y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        Y[i] += X[i];
}

// partial sums of squares per (sample block, chunk of rows, lane): P[b][c][lane]
__global__ void __launch_bounds__(64) k_colnorm2(const double *__restrict__ X, int64_t N, int64_t rows_per,
                                                 double *__restrict__ P) {
    const int64_t c = blockIdx.x, b = blockIdx.y;
    const int lane = threadIdx.x;
    const int64_t r0 = c * rows_per, r1 = min(N, r0 + rows_per);
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const double x = X[(b * N + r) * 64 + lane];
        s += x * x;
    }
    P[(b * gridDim.x + c) * 64 + lane] = s;
}

}  // namespace

void launch_residual(const MeshView &mv, double cI, double cL, const double *B, const double *X, double *R, int32_t nb,
                     hipStream_t st) {
    if (nb == 0) return;
    if (mv.E > 0) {
        hipLaunchKernelGGL(k_residual_interior, dim3((unsigned)mv.E, (unsigned)nb), dim3(64), 0, st, mv, cI, cL, B, X,
                           R);
        GRF_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_residual_vertex, dim3((unsigned)((mv.V + 3) / 4), (unsigned)nb), dim3(256), 0, st, mv, cI,
                       cL, B, X, R);
    GRF_LAUNCH_CHECK();
}

void launch_axpy1(const double *X, double *Y, int64_t n, hipStream_t st) {
    if (n == 0) return;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_axpy1, dim3((unsigned)blocks), dim3(256), 0, st, X, Y, n);
    GRF_LAUNCH_CHECK();
}

int64_t colnorm_chunks(int64_t N) { return std::max<int64_t>(1, std::min<int64_t>(1024, (N + 4095) / 4096)); }

void launch_colnorm2(const double *X, int64_t N, int32_t nb, double *P, hipStream_t st) {
    if (nb == 0 || N == 0) return;
    const int64_t chunks = colnorm_chunks(N);
    const int64_t per = (N + chunks - 1) / chunks;
    hipLaunchKernelGGL(k_colnorm2, dim3((unsigned)chunks, (unsigned)nb), dim3(64), 0, st, X, N, per, P);
    GRF_LAUNCH_CHECK();
}

}  // namespace grf
