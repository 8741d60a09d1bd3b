// Layout changes between the canonical [S][N] vectors of the ABI and the
// sample-interleaved [nb][N][64] layout the sweeps use (lanes = samples, so a
// wavefront's access to one DOF is one contiguous 512-byte row).
#include <algorithm>

#include "work.h"

namespace grf {
namespace {

constexpr int kT = 64;  // tile: 64 DOFs x 64 samples, staged in LDS

// in[s][j] -> X[b][j][lane]; padded samples (s >= S) are written as 0
__global__ void __launch_bounds__(256) k_to_interleaved(const double *__restrict__ in, int64_t S, int64_t N,
                                                        double *__restrict__ X) {
    __shared__ double tile[kT][kT + 1];
    const int64_t j0 = (int64_t)blockIdx.x * kT;
    const int64_t b = blockIdx.y;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int si = ty; si < kT; si += 4) {
        int64_t s = b * kT + si, j = j0 + tx;
        tile[si][tx] = (s < S && j < N) ? in[s * N + j] : 0.0;
    }
    __syncthreads();
    for (int ji = ty; ji < kT; ji += 4) {
        int64_t j = j0 + ji;
        if (j < N) X[(b * N + j) * 64 + tx] = tile[tx][ji];
    }
}

// X[b][j][lane] -> out[s][j] for s < S (lanes of padding samples are not read)
__global__ void __launch_bounds__(256) k_from_interleaved(const double *__restrict__ X, int64_t S, int64_t N,
                                                          double *__restrict__ out) {
    __shared__ double tile[kT][kT + 1];
    const int64_t j0 = (int64_t)blockIdx.x * kT;
    const int64_t b = blockIdx.y;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int ji = ty; ji < kT; ji += 4) {
        int64_t j = j0 + ji;
        tile[ji][tx] = (j < N && b * kT + tx < S) ? X[(b * N + j) * 64 + tx] : 0.0;  // no padding lanes read
    }
    __syncthreads();
    for (int si = ty; si < kT; si += 4) {
        int64_t s = b * kT + si, j = j0 + tx;
        if (s < S && j < N) out[s * N + j] = tile[tx][si];
    }
}

__global__ void k_fill(double *__restrict__ p, size_t n, double v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// X[b][row][lane] -> outs[z][s][j] for every graph z of a batch, local DOF j of the
// graph at row ri + j (interior) or rv + j - ni (vertices).  Workgroup = one 64-DOF
// tile of one graph (the tiles of all graphs numbered in a row, tile0), 64 samples.
__global__ void __launch_bounds__(256) k_from_interleaved_seg(const double *__restrict__ X, int64_t S, int64_t N,
                                                              const int64_t *__restrict__ segs,
                                                              const int64_t *__restrict__ tile0, int32_t ng,
                                                              int64_t ntiles, double *const *__restrict__ outs) {
    __shared__ double tile[kT][kT + 1];
    const int64_t b = blockIdx.y;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    // a block of at most 32 real samples reads two DOF rows per wavefront step
    const int64_t Sb = S - b * kT < kT ? S - b * kT : kT;
    const int nvw = Sb <= 32 ? 2 : 1;
    const int sl = tx & (kT / nvw - 1), hv = tx / (kT / nvw);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int lo = 0, hi = ng;  // tile0[lo] <= t < tile0[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tile0[mid] <= t) lo = mid; else hi = mid;
        }
        const int64_t z = lo;
        const int64_t n = segs[4 * z], ni = segs[4 * z + 1], ri = segs[4 * z + 2], rv = segs[4 * z + 3];
        const int64_t j0 = (t - tile0[z]) * kT;
        double *out = outs[z];
        for (int ji = nvw * ty + hv; ji < kT; ji += 4 * nvw) {
            const int64_t j = j0 + ji;
            const int64_t row = j < ni ? ri + j : rv + (j - ni);
            tile[ji][sl] = (j < n && sl < Sb) ? X[(b * N + row) * 64 + sl] : 0.0;  // no padding lanes read
        }
        __syncthreads();
        for (int si = ty; si < Sb; si += 4) {
            const int64_t s = b * kT + si, j = j0 + tx;
            if (s < S && j < n) out[s * n + j] = tile[tx][si];
        }
        __syncthreads();  // the tile is rewritten by the next pass
    }
}

// rows [r0, r0 + nrows) of every 64-sample block of a [nb][N][64] array
__global__ void k_fill_rows(double *__restrict__ p, int64_t nb, int64_t N, int64_t r0, int64_t nrows) {
    const int64_t per = nrows * 64, n = nb * per;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / per, k = i - b * per;
        p[(b * N + r0) * 64 + k] = 0.0;
    }
}

}  // namespace

void launch_fill_rows(double *p, int64_t nb, int64_t N, int64_t r0, int64_t nrows, hipStream_t st) {
    const int64_t n = nb * nrows * 64;
    if (n == 0) return;
    GRF_REQUIRE(r0 >= 0 && r0 + nrows <= N, "internal: row range outside the array");
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_fill_rows, dim3((unsigned)blocks), dim3(256), 0, st, p, nb, N, r0, nrows);
    GRF_LAUNCH_CHECK();
}

void launch_from_interleaved_seg(const MeshView &mv, const double *X, int64_t S, double *const *outs,
                                 hipStream_t st) {
    const int64_t nb = (S + 63) / 64;
    if (nb == 0 || mv.ntiles == 0) return;
    GRF_REQUIRE(nb < 65536, "batch too large");
    const int64_t gx = std::min<int64_t>(mv.ntiles, int64_t(1) << 20);
    hipLaunchKernelGGL(k_from_interleaved_seg, dim3((unsigned)gx, (unsigned)nb), dim3(256), 0, st, X, S, mv.N,
                       mv.segs, mv.tile0, mv.ng, mv.ntiles, outs);
    GRF_LAUNCH_CHECK();
}

void launch_to_interleaved(const double *in, int64_t S, int64_t N, double *X, hipStream_t st) {
    int64_t nb = (S + 63) / 64;
    if (nb == 0 || N == 0) return;
    GRF_REQUIRE((N + kT - 1) / kT < (int64_t(1) << 31) && nb < 65536, "vector too large");
    hipLaunchKernelGGL(k_to_interleaved, dim3((unsigned)((N + kT - 1) / kT), (unsigned)nb), dim3(256), 0, st, in, S,
                       N, X);
    GRF_LAUNCH_CHECK();
}

void launch_from_interleaved(const double *X, int64_t S, int64_t N, double *out, hipStream_t st) {
    int64_t nb = (S + 63) / 64;
    if (nb == 0 || N == 0) return;
    GRF_REQUIRE((N + kT - 1) / kT < (int64_t(1) << 31) && nb < 65536, "vector too large");
    hipLaunchKernelGGL(k_from_interleaved, dim3((unsigned)((N + kT - 1) / kT), (unsigned)nb), dim3(256), 0, st, X,
                       S, N, out);
    GRF_LAUNCH_CHECK();
}

void launch_fill(double *p, size_t n, double v, hipStream_t st) {
    if (n == 0) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    GRF_LAUNCH_CHECK();
}

}  // namespace grf
