// Workspace of a graph handle and the kernel launchers of each step.
#pragma once

#include "common.h"

struct grf_graph::Work {
    grf::DevBuf X, U;             // sample-interleaved [nb][N][64]: input (noise / rhs) and accumulator
    grf::DevBuf rho;              // per-DOF multipliers [NI][LBp] (streamed sweeps)
    grf::DevBuf fwdt, bwdt;       // per-DOF step rows [NI][LBp] of (rho_{k-1}, dg_k) / (rho_{k-1}, of_k)
    grf::DevBuf btab;             // matrix-core operand tables per 16-position edge block
    grf::DevBuf ztab;             // pass-B operand tables per edge block
    grf::DevBuf boff;             // [E+1] first block of every edge
    grf::DevBuf bmap;             // [nblocks] int2: (edge, block index within the edge)
    grf::DevBuf babs, rhom;       // per-edge [E][LBp]: |b| = gamma/h_e, rho_{m-1}
    grf::DevBuf etab;             // per (edge, shift) closed-form scalars of the operand tables [E][10][LBp]
    grf::DevBuf sd, so;           // per-edge Schur 2x2 [LBp][E]: diagonal, off-diagonal
    grf::DevBuf shift;            // [LBp][2]: c_I, c_L of the shifts in the block
    grf::DevBuf ends;             // [LB][E][2][Sp]: |b| * (A_II^{-1} W_I) at both ends of every edge
                                  // (FP32 with mixed precision)
    grf::DevBuf gT, xT;           // [LB][S][V]: condensed right-hand sides / vertex solutions
    grf::DevBuf ug;               // [LB][V][Sp]: vertex solutions, sample-interleaved (FP32 with mixed precision)
    grf::DevBuf pcg_scr;          // PCG vectors in global memory (large graphs)
    grf::DevBuf pcg_ops;          // per-shift-block vertex operators of the global-memory PCG
    grf::DevBuf its, res;         // [LB][S] int32 iterations, double relative residual
    grf::DevBuf gexp;             // [ng][LB][S] int32: right-hand side scaled by 2^gexp for the PCG
    grf::DevBuf Bm, Xacc, nrm;    // mixed-precision refinement: right-hand sides, iterate, norm partials
    std::vector<int32_t> h_its;
    std::vector<double> h_res;
    std::vector<int32_t> h_gexp;
};

namespace grf {

void free_work(grf_graph &g);
grf_graph::Work &work(grf_graph &g);

// The whole path of grf_sample (noise null) and grf_sample_from_noise (noise given):
// status GRF_OK or GRF_ENOCONV; throws Error on any other failure.
int sample_impl(grf_graph *g, double kappa, double beta, double quad_step, int64_t n_samples, uint64_t seed,
                const double *noise, double *out, const grf_opts *opts);

// ---- launchers (each .hip file implements its own) -------------------------
// noise: X[b][j][lane] = msqrt[j] * Z(seed, soff + b*64 + lane, j) for b*64+lane < S, 0 otherwise
void launch_noise(const MeshView &mv, int64_t S, int64_t soff, uint64_t seed, double *X, hipStream_t st);

// layout transforms between canonical [S][N] and sample-interleaved [nb][N][64]
void launch_to_interleaved(const double *in, int64_t S, int64_t N, double *X, hipStream_t st);
void launch_from_interleaved(const double *X, int64_t S, int64_t N, double *out, hipStream_t st);
// batch: graph g's DOFs of X (mesh of the batch) -> outs[g][s][j] (device array of device pointers)
void launch_from_interleaved_seg(const MeshView &mv, const double *X, int64_t S, double *const *outs, hipStream_t st);
void launch_fill(double *p, size_t n, double v, hipStream_t st);
// zero rows [r0, r0 + nrows) of each of the nb sample blocks of a [nb][N][64] array
void launch_fill_rows(double *p, int64_t nb, int64_t N, int64_t r0, int64_t nrows, hipStream_t st);

// per-(shift, edge) coefficients: Thomas rows (streamed sweeps), |b|, rho_{m-1}, Schur 2x2
struct CoeffArgs {
    const double *shift;  // [LBp][2] c_I, c_L
    int32_t LB, LBp;
    double *rho;            // [NI][LBp] (streamed sweeps)
    double2 *fwdt, *bwdt;   // [NI][LBp] (streamed sweeps)
    double *babs, *rhom;    // [E][LBp]
    double *sd, *so;        // [LBp][E]
    double *etab;           // [E][10][LBp] scalars of the blocked operand tables (null: not written)
};
// recurrence form: Thomas rows and the per-edge quantities
void launch_coeff(const MeshView &mv, const CoeffArgs &a, hipStream_t st);
// closed form: the per-edge quantities only (the blocked sweeps build their operands in blocked.hip)
void launch_edge_coeff(const MeshView &mv, const CoeffArgs &a, hipStream_t st);
constexpr int kEdgeTabFields = 10;  // CoeffArgs::etab values per (edge, shift)

// sweeps over edge interiors (lanes = samples, shifts in registers)
struct SweepArgs {
    const double *X;        // [nb][N][64] right-hand sides (noise)
    double *U;              // [nb][N][64] accumulator (acc mode)
    const double *rho;      // [NI][LBp]
    const double2 *fwdt, *bwdt;  // [NI][LBp]
    const double *babs, *rhom;    // [E][LBp]
    const double *ug;       // [LB][V][Sp] vertex solutions (acc mode)
    double *ends;           // [LB][E][2][Sp] (ends mode)
    int32_t LB, LBp, nb, Sp;
    int32_t bl;             // shifts per wavefront: 8, 16, 32, 64
    int32_t fp32;           // run the recurrences in FP32
};
void launch_sweep_ends(const MeshView &mv, const SweepArgs &a, bool fwd, hipStream_t st);
void launch_sweep_acc(const MeshView &mv, const SweepArgs &a, bool fwd, hipStream_t st);

// blocked (matrix-core) sweeps: 16-position edge blocks, shifts padded to 16*NT
struct BlockArgs {
    const int32_t *boff;    // [E+1] first block of every edge
    const int2 *bmap;       // [nblocks] (edge, block index within the edge)
    int64_t nblocks;        // blocks of the whole graph
    int32_t NT;             // shift tiles of 16
    int32_t LB, LBp;        // real / padded shifts (LBp = 16 NT)
    const double *shift;    // [LBp][2] c_I, c_L
    const double *babs, *rhom;         // [E][LBp]
    const double *etab;     // [E][10][LBp] per-(edge, shift) scalars (k_edge_coeff)
    double *tab;            // pass-A operands, block_tab_doubles(NT) per block
    double *ztab;           // pass-B operands (first/last columns of T^{-1}), 512 NT per block
    const double *X;        // [nb][N][64]
    double *U;              // [nb][N][64]
    double *ends;           // [LB][E][2][Sp]
    float *ends32;          // the same, FP32 (mixed precision: written by the FP32 sweeps)
    const double *ug;       // [LB][V][Sp]
    const float *ug32;      // the same, FP32 (mixed precision: read by the FP32 recovery)
    int32_t nb, Sp;
    int32_t first;          // first shift block: the forward pass writes (not updates) the interior accumulator
    int32_t mixed;          // FP32 operand tables and matrix-core products (mixed precision)
    int64_t S;              // real samples (wavefronts of padding samples skip the products)
    float *tab32, *ztab32;  // the FP32 tables (same layout sizes as tab / ztab)
};
int64_t block_tab_doubles(int32_t NT);
void launch_block_map(const int32_t *boff, int64_t E, int2 *bmap, hipStream_t st);
void launch_blocktab(const MeshView &mv, const BlockArgs &a, hipStream_t st);
// pass A, both directions in one launch
void launch_sweep_blocked(const MeshView &mv, const BlockArgs &a, hipStream_t st);
void launch_corr_blocked(const MeshView &mv, const BlockArgs &a, hipStream_t st);

// mixed-precision refinement (mixed.hip): R = B - A X on the interleaved layout (A of one shift),
// Y += X, and per-column partial sums of squares P[nb][colnorm_chunks(N)][64]
void launch_residual(const MeshView &mv, double cI, double cL, const double *B, const double *X, double *R, int32_t nb,
                     hipStream_t st);
void launch_axpy1(const double *X, double *Y, int64_t n, hipStream_t st);
int64_t colnorm_chunks(int64_t N);
void launch_colnorm2(const double *X, int64_t N, int32_t nb, double *P, hipStream_t st);

// learned preconditioner (learned.hip): per shift of a block, D^{-1/2} [LB][V], the
// scale-free preconditioner (diagonal [LB][V], edge couplings [LB][E]) and
// initial-guess operator (same shapes)
struct LearnedOps {
    const double *Dh, *Pd, *Pq, *Qd, *Qe;
};
void learned_reserve(grf_learned &net, const MeshView &mv, int32_t LB);
// bf16act: bfloat16 hidden activations (the sampler's inference forward); false: FP32
// activations, as the training backward needs them
void learned_forward(grf_learned &net, const MeshView &mv, const double *shift, const double *sd, const double *so,
                     int32_t LB, hipStream_t st, bool bf16act);
LearnedOps learned_ops(grf_learned &net);
double learned_backward(grf_learned &net, const MeshView &mv, const double *g, const double *x, int32_t LB, int64_t S,
                        hipStream_t st);
void learned_adam(grf_learned &net, double lr, hipStream_t st);
void learned_copy_grad(grf_learned &net, float *host, hipStream_t st);
uint64_t learned_signature(const grf_learned &net);
size_t learned_held_bytes(const grf_learned &net);

// vertex Schur complement: condensed rhs, PCG, layout changes, accumulation
struct SchurArgs {
    const double *X;      // [nb][N][64] noise (vertex part used)
    const double *ends;   // [LB][E][2][Sp]
    const float *ends32;  // the same, FP32 (mixed precision), or null
    const double *sd, *so;  // [LBp][E]
    double *gT, *xT;      // [LB][S][V]
    double *ug;           // [LB][V][Sp]
    float *ug32;          // the same, FP32 (mixed precision, blocked sweeps), or null
    double *U;            // [nb][N][64]
    double *scr;          // PCG scratch (large graphs)
    double *ops;          // vertex operators of the block for the global-memory PCG (pcg_ops_bytes)
    int32_t *its;         // [LB][S]
    int32_t *gexp;        // [ng][LB][S] scale exponents of the right-hand sides (k_rhs_range)
    double *res;          // [LB][S]
    int32_t LB, LBp, nb, Sp;
    int64_t S;
    double tol;
    int32_t maxit;
    int32_t pcg_blocks;   // resident workgroups for the global-memory PCG
    int32_t precond;            // GRF_PRECOND_* of the solve
    const LearnedOps *learned;  // learned preconditioner and initial guess of this block (GRF_PRECOND_LEARNED)
    const int8_t *cls_mode;     // learned: ChipMode per size class, or null (default_chip_modes)
    KTimer *ctimer;             // optional: times each size class's launch under kClassTimerId + class
};

// On-chip PCG variant of a size class: the operator preconditioner (with the
// learned initial guess, if any), the learned initial guess with Jacobi, or Jacobi.
// CM_GLOBAL (reported only): the class runs the multi-system kernel instead.
enum ChipMode : int8_t { CM_OP = 0, CM_GUESS = 1, CM_JACOBI = 2, CM_GLOBAL = 3 };
constexpr int kChipOpClasses = 5;  // size classes whose LDS holds r^ and p (CM_OP)
constexpr int kMrhsSB = 4;         // samples per block of the multi-system PCG kernel
constexpr int32_t kRangeNonFinite = INT32_MIN;  // gexp of a system whose right-hand side holds NaN or Inf
constexpr int kClassTimerId = 100;  // + size class (kPcgClasses: the global-memory kernel)
void default_chip_modes(int32_t precond, int8_t *mode);  // [kPcgClasses]
bool chip_mode_valid(int c, int mode);
void launch_condense(const MeshView &mv, const SchurArgs &a, hipStream_t st);
void launch_pcg(const MeshView &mv, const SchurArgs &a, hipStream_t st);
void prepare_pcg(const MeshView &mv);  // one-time kernel attributes, before any graph capture
void launch_vertex_scatter(const MeshView &mv, const SchurArgs &a, hipStream_t st);
size_t pcg_scratch_bytes(const MeshView &mv, int32_t blocks);  // resident blocks of kMrhsSB samples
size_t pcg_ops_bytes(const MeshView &mv, int32_t LB, int32_t precond);

}  // namespace grf
