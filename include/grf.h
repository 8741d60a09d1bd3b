/*
 * grf.h -- C ABI of libgrf, a sampler for Gaussian random fields on metric
 * graphs for AMD Instinct MI355X (gfx950).
 *
 * A field solves the fractional SPDE (kappa^2 - Delta)^beta u = W on a metric
 * graph (paper: eq. fractional_spde).  A sample is the sinc-quadrature sum of
 * shifted lumped-mass finite-element solves
 *     u = sum_{l=-K^-}^{K^+} ((c_I + c_L kappa^2) M_L + c_L G)^{-1} W,
 * (paper: eq. balakrishnan_quadrature, eq. coefficients, eq. spde_approx_fem,
 * with the kappa^2 M term of the discretised operator written out), driven by
 * lumped white noise W = M_L^{1/2} xi (paper: eq. wh_def and "Mass Lumping").
 * Each shifted solve is done by static condensation onto the graph vertices
 * (paper: eq. global_schur and "Phase 3"-"Phase 5").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Status: every call returns a grf_status; no C++ exception crosses the
 *   ABI.  grf_last_error() returns a thread-local description of the most
 *   recent failure on the calling thread.
 * - Memory: host pointers are named "host", device pointers "device".  The
 *   caller owns every pointer it passes; the library copies what it keeps.
 *   Device pointers must be HIP allocations on the device the graph was
 *   created on.
 * - Streams: work is enqueued on opts->stream (NULL = the null stream) and
 *   the call returns after that stream has finished it (the library needs
 *   the solver's convergence flags on the host).  A graph handle must not be
 *   used from two threads at once.
 * - DOF order ("canonical order"): interior DOFs first, edge-major in input
 *   edge order, each edge's m_e = n_e - 1 interior nodes running from the
 *   tail vertex u_e (x = 0) to the head vertex v_e (x = l_e); then vertex v
 *   at index n_interior + v (paper: Phase 2, W = [W_I,1 ... W_I,|E| W_Gamma],
 *   and "Quadrature Accumulation and Global Assembly").
 * - Mesh (paper: "Phase 1: Initialization"): n_e = ceil(l_e / h) elements
 *   (GRF_MESH_CEIL) or n_e = floor(l_e / h + 1/2) (GRF_MESH_ROUND), at least
 *   1 (2 for a self-loop), h_e = l_e / n_e.
 */
#ifndef GRF_H
#define GRF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum grf_status {
    GRF_OK = 0,
    GRF_EINVAL = -1,  /* an argument is out of its documented domain */
    GRF_ENOMEM = -2,  /* device or host allocation failed */
    GRF_EDEVICE = -3, /* a HIP call failed (message names it) */
    GRF_ENOCONV = -4, /* some vertex Schur PCG hit maxit; output still written */
    GRF_EUNSUP = -5,  /* a documented-but-unsupported combination */
    GRF_ENONFINITE = -6 /* a vertex Schur system had a NaN or Inf right-hand side or
                           residual (a non-finite input reaches every vertex system
                           it touches); output still written, the vertex values of
                           those systems and the edges around them hold NaN.
                           Takes precedence over GRF_ENOCONV. */
} grf_status;

/* grf_graph_create flags */
#define GRF_MESH_CEIL 0u  /* n_e = ceil(l_e/h)  (paper, Phase 1) */
#define GRF_MESH_ROUND 1u /* n_e = floor(l_e/h + 1/2) */
/* OR-ed with a mesh rule: the shifted systems use the consistent mass matrix
   (element matrices (h_e/6)[[2,1],[1,2]], paper Phase 2, consistent entries)
   instead of the lumped one.  The noise of grf_sample / grf_noise stays the
   lumped W = M_L^{1/2} xi (grf_sample_from_noise takes any load).  Runs the
   streamed edge sweeps (sweep_block 0 picks their width); GRF_PREC_MIXED
   returns GRF_EUNSUP. */
#define GRF_MASS_CONSISTENT_SYS 2u
/* OR-ed with the others: grf_noise, grf_sample and grf_sample_batched draw the
   consistent-mass noise W = R xi with R R^T = M (the consistent mass above;
   paper eq. wh_def and Phase 2, consistent case) instead of M_L^{1/2} xi.  R is
   the assembly of per-element factors F_e = [[a, c], [a, -c]], a = sqrt(h_e/4),
   c = sqrt(h_e/12), F_e F_e^T = (h_e/6)[[2,1],[1,2]]: the same law as the
   paper's Cholesky factor, O(N), with two normals per element from the Philox
   block with counter (g / 2, 1, 0, 0) for element g (the element ordering and
   the summation order are fixed in the project documentation, so the values are
   reproducible bit for bit).  Works with either system mass. */
#define GRF_NOISE_CONSISTENT 4u

/* grf_opts.precision */
#define GRF_PREC_FP64 0  /* every step in FP64 */
#define GRF_PREC_MIXED 1 /* FP32 edge sweeps (products summed in FP32 within a tile of 16 shifts,
                            tiles added in FP64), FP64 noise, Schur blocks, PCG, residual and
                            accumulation; grf_solve_shifted refines against an FP64 residual
                            (opts->refine), grf_sample rejects refine > 0 */

/* grf_opts.pcg_class_modes: marks the per-class variants as given */
#define GRF_PCG_MODES_SET (1 << 12)

/* grf_opts.precond */
#define GRF_PRECOND_JACOBI 0  /* diagonal of the vertex Schur complement */
#define GRF_PRECOND_LEARNED 1 /* learned diagonal-plus-neighbour operator (opts->learned) */
#define GRF_PRECOND_NN 2      /* Neumann-Neumann: D^{-1} (sum_e S_e^{-1}) D^{-1}, D = diag(edge ends at v),
                                 S_e the edge's 2x2 Schur block (Phase 4, "The Neumann Step"); x0 = 0 */

typedef struct grf_graph grf_graph;
typedef struct grf_learned grf_learned;

/* Kernel classes of grf_stats.kernel_ms / kernel_launches. */
enum grf_kernel_id {
    GRF_K_NOISE = 0,     /* lumped white noise */
    GRF_K_COEFF = 1,     /* per-(shift, edge) Thomas rows and Schur blocks (k_edge_coeff, or the
                            streamed path's rows) */
    GRF_K_ENDS_FWD = 2,  /* condensed-rhs sweeps: blocked, both directions in one launch;
                            streamed, the forward sweep (head ends) */
    GRF_K_ENDS_BWD = 3,  /* condensed-rhs sweep, streamed: the backward sweep (tail ends) */
    GRF_K_CONDENSE = 4,  /* vertex right-hand sides */
    GRF_K_PCG = 5,       /* vertex Schur PCG */
    GRF_K_SCATTER = 6,   /* vertex solutions to the sample layout */
    GRF_K_ACC_FWD = 7,   /* interior recovery, forward part + accumulation */
    GRF_K_ACC_BWD = 8,   /* interior recovery, backward part + accumulation */
    GRF_K_LAYOUT = 9,    /* layout changes and fills */
    GRF_K_MIXED = 10,    /* mixed-precision residual and refinement kernels */
    GRF_K_LEARNED = 11,  /* learned preconditioner */
    GRF_K_TABLE = 12,    /* blocked sweeps: the per-(16-position block, shift) operand tables */
    GRF_K_COUNT = 13
};

/* Solver statistics, filled when grf_opts.stats is non-NULL (host struct). */
typedef struct grf_stats {
    int32_t n_shifts;           /* quadrature nodes used */
    int32_t n_systems;          /* vertex Schur systems solved (shifts x samples) */
    int32_t n_unconverged;      /* systems that hit maxit */
    int32_t max_iterations;     /* largest PCG iteration count */
    int64_t total_iterations;   /* sum over systems */
    double max_rel_residual;    /* max ||g - S u||_2 / ||g||_2 over systems */
    int32_t refine_steps;       /* mixed precision: refinement sweeps run */
    int32_t shift_block;        /* shifts processed per pass (as planned) */
    int32_t sweep_block;        /* shifts held per wavefront in the sweeps */
    int32_t pcg_class_modes;    /* grf_sample_batched: on-chip PCG variant of size class c in bits 2c..2c+1
                                   (0 operator preconditioner, 1 learned initial guess only, 2 Jacobi,
                                   3 the class runs the global-memory kernel) */
    double kernel_ms[16];       /* with opts.timing: summed HIP-event time per grf_kernel_id
                                   (entries from GRF_K_COUNT on stay 0) */
    int32_t kernel_launches[16];/* with opts.timing: launches per grf_kernel_id */
    /* Vertex PCG by graph size class c (vertex capacities 64, 256, 1024, 4096,
       10176, 20352 for c = 0..5; c = 6: the graphs that run the global-memory
       kernel, including a class the preconditioner sends there).  One launch per
       class and shift block. */
    double pcg_class_ms[7];          /* with opts.timing: HIP-event time of the class's launches */
    int32_t pcg_class_launches[7];   /* with opts.timing: launches */
    int32_t n_nonfinite;             /* systems with a NaN/Inf right-hand side or residual (GRF_ENONFINITE) */
    int64_t pcg_class_vertex_its[7]; /* sum over the class's systems of iterations x graph vertices */
    int64_t pcg_class_end_its[7];    /* sum over the class's systems of iterations x graph edge ends (2|E|) */
} grf_stats;

typedef struct grf_opts {
    double tol;            /* PCG: stop when ||g - S u||_2 <= tol ||g||_2 on the
                              recomputed residual; default 1e-12 */
    int32_t maxit;         /* PCG iteration cap per system; default 10000 */
    int32_t precision;     /* GRF_PREC_*; default GRF_PREC_FP64 */
    int32_t precond;       /* GRF_PRECOND_*; default GRF_PRECOND_JACOBI */
    int32_t k_minus;       /* quadrature limits; < 0 selects the paper's rule */
    int32_t k_plus;        /*   K^- = ceil(pi^2/(4k^2 beta)), K^+ = ceil(pi^2/(4k^2(1-beta))) */
    int32_t shift_block;   /* shifts per pass; 0 = plan from a memory budget */
    int32_t sweep_block;   /* shifts per wavefront in the sweeps: 0 (auto), 8, 16, 32, 64 */
    int32_t refine;        /* mixed precision, grf_solve_shifted: refinement sweeps; < 0 = default (2);
                              the sampling calls accept only < 0 or 0 */
    int32_t timing;        /* 1: time every kernel with HIP events into stats->kernel_ms (grf_sample_batched
                              then runs its launches uncaptured, each timed) */
    int32_t pcg_class_modes; /* learned preconditioner only: 0 = automatic (grf_sample_batched times the
                                three on-chip PCG variants per size class once and keeps the fastest;
                                elsewhere the default); or GRF_PCG_MODES_SET | (variant of class c)
                                << 2c, variants as in grf_stats.pcg_class_modes (0 only for c < 5) */
    int64_t sample_offset; /* global index of the first sample (noise key) */
    void *stream;          /* hipStream_t; NULL = null stream */
    const grf_learned *learned; /* required when precond = GRF_PRECOND_LEARNED */
    grf_stats *stats;      /* optional output, host */
} grf_opts;

/* Fill *opts with the defaults listed above. */
void grf_opts_init(grf_opts *opts);

/*
 * Create a graph and its mesh (paper: "Phase 1: Initialization").
 *   n_vertices  |V| >= 1
 *   n_edges     |E| >= 0
 *   edges       host, int64 [n_edges][2], 0-based (tail u_e, head v_e);
 *               self-loops and multi-edges are allowed
 *   lengths     host, float64 [n_edges], finite and > 0
 *   h           target mesh size, finite and > 0
 *   flags       GRF_MESH_CEIL or GRF_MESH_ROUND
 *   out         receives the handle; it owns device copies of the mesh
 * Errors: GRF_EINVAL for a bad size, endpoint, length or h, or a vertex with
 * no incident edge (its lumped mass is 0 and the shifted system singular).
 * Uses the current HIP device.
 */
int grf_graph_create(int64_t n_vertices, int64_t n_edges, const int64_t *edges,
                     const double *lengths, double h, uint32_t flags, grf_graph **out);

/* Sizes of the canonical DOF vector.  dof_offsets (host, int64 [n_edges+1],
 * may be NULL) receives the first interior DOF of every edge. */
int grf_graph_info(const grf_graph *g, int64_t *n_dof, int64_t *n_interior, int64_t *dof_offsets);

/* Diagonal of the lumped mass matrix M_L in canonical order (paper: "Phase 2",
 * lumped case): h_e at the interior nodes of edge e, the sum of h_e / 2 over
 * the edge ends at a vertex.  out: host, float64 [n_dof].  It defines the
 * norm ||u||_{M_L} in which sample errors are measured. */
int grf_graph_lumped_mass(const grf_graph *g, double *out);

/* Release a graph and every device buffer it holds.  NULL is accepted. */
int grf_graph_destroy(grf_graph *g);

/*
 * Quadrature limits for (beta, quad_step) on this graph: quad_step == 0
 * selects the paper's step k = -1/(beta ln h); opts->k_minus/k_plus >= 0
 * override the paper's limits (paper: "Strong error" subsection).  g may be
 * NULL when quad_step > 0 (h enters only the paper's step rule).  Host only.
 * Errors (here and in every sampling call): GRF_EINVAL for beta outside
 * (0, 1), more than 1e6 shifts, or limits so wide that some c_I or c_L is
 * not finite and positive.
 */
int grf_shift_count(const grf_graph *g, double beta, double quad_step, const grf_opts *opts,
                    int32_t *k_minus, int32_t *k_plus, double *step_used);

/*
 * Lumped white noise W[s][j] = sqrt(M_L[j,j]) * Z(seed, sample_offset + s, j)
 * (paper: eq. wh_def with R = M_L^{1/2}).  Z is Philox4x64-10 with key
 * (seed, global sample index) and counter (j/4, 0, 0, 0) followed by the
 * fixed-order Box-Muller transform specified in the project documentation;
 * the same (seed, sample, j) always gives the same bits.
 *   out   device, float64 [n_samples][n_dof], canonical order
 * A graph created with GRF_NOISE_CONSISTENT gets the consistent-mass noise
 * instead (see the flag).
 */
int grf_noise(grf_graph *g, int64_t n_samples, uint64_t seed, double *out, const grf_opts *opts);

/*
 * Draw n_samples fields: u[s] = sum_l A^(l)^{-1} W[s] with
 * A^(l) = (c_I^(l) + c_L^(l) kappa^2) M_L + c_L^(l) G, y_l = l k,
 * c_I = pi/(2 k sin(pi beta)) e^{-2 beta y_l}, c_L = c_I e^{2 y_l}, l
 * increasing from -K^- to K^+ (paper: eq. coefficients, eq. spde_approx_fem).
 *   kappa      > 0
 *   beta       in (0, 1)
 *   quad_step  k > 0, or 0 for the paper's k = -1/(beta ln h)
 *   out        device, float64 [n_samples][n_dof], canonical order
 * Returns GRF_ENOCONV (with out written) if a Schur system hit maxit, and
 * GRF_ENONFINITE (with out written, NaN in the affected samples) if one had a
 * NaN or Inf right-hand side or residual.
 */
int grf_sample(grf_graph *g, double kappa, double beta, double quad_step, int64_t n_samples,
               uint64_t seed, double *out, const grf_opts *opts);

/*
 * The same sum for caller-supplied noise, W[s] = noise[s] (eq. spde_approx_fem
 * with a given load): the path of grf_sample without the Philox draw, for noise
 * coupled across meshes (convergence studies, multilevel estimators).
 *   noise  device, float64 [n_samples][n_dof], canonical order (the layout
 *          grf_noise writes); read only, may not alias out
 *   out    device, float64 [n_samples][n_dof], canonical order
 * With noise = grf_noise(g, n_samples, seed) the result equals grf_sample's bit
 * for bit.  Returns GRF_ENOCONV (with out written) if a Schur system hit maxit,
 * GRF_ENONFINITE (with out written) if the noise holds a NaN or Inf: the
 * samples it reaches are NaN, the others are solved.
 */
int grf_sample_from_noise(grf_graph *g, double kappa, double beta, double quad_step, int64_t n_samples,
                          const double *noise, double *out, const grf_opts *opts);

/*
 * grf_sample for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, result and statuses as grf_sample; the call allocates nothing.
 * Its whole workspace lives in a fixed 128 MiB device array that the library
 * holds on every device it runs on until the process ends (the graph's own
 * mesh, uploaded by grf_graph_create, is not part of it).
 *   - GRF_EINVAL (before or during the call, message names the sizes) when the
 *     workspace of (graph, shifts, n_samples) needs more than the 128 MiB;
 *     roughly, 16 * ceil(n_samples/64) * 64 * n_dof bytes for the noise and
 *     accumulator plus per-shift tables must fit.
 *   - GRF_EINVAL for GRF_PRECOND_LEARNED (the network keeps its own workspace)
 *     or when the current device is not the graph's.
 *   - opts->timing is ignored (no per-kernel events are created).
 * Every call on a device shares that device's array: calls that overlap on one
 * device (two threads, or two streams running at once) race and give wrong
 * results.  The array keeps the last call's contents; the path clears what it
 * reads before writing it.
 */
int grf_sample_noalloc(grf_graph *g, double kappa, double beta, double quad_step, int64_t n_samples,
                       uint64_t seed, double *out, const grf_opts *opts);

/*
 * One shifted solve for n_rhs right-hand sides:
 *   out[r] = ((c_I + c_L kappa^2) M_L + c_L G)^{-1} rhs[r]
 * (paper: eq. spde_approx_fem for a single l, solved by eq. global_schur).
 *   c_I, c_L   > 0 and finite; kappa >= 0
 *   rhs, out   device, float64 [n_rhs][n_dof], canonical order; may not alias
 * Returns GRF_ENOCONV or GRF_ENONFINITE with out written, as grf_sample does;
 * a right-hand side holding NaN or Inf gives NaN in its row of out.  With
 * GRF_PREC_MIXED a finite value beyond the FP32 range counts as Inf.
 */
int grf_solve_shifted(grf_graph *g, double kappa, double c_I, double c_L, int64_t n_rhs,
                      const double *rhs, double *out, const grf_opts *opts);

/*
 * grf_sample for several graphs at once, one kappa per graph, sharing beta,
 * quad_step (0 = the paper's rule, from the graphs' common h), n_samples and
 * seed.  All graphs must share h and the mesh rule.  outs[i] is a device
 * pointer to float64 [n_samples][n_dof(graphs[i])].  The graphs are laid out
 * as one disjoint union and every step runs as one set of launches, captured
 * once into a HIP graph and replayed for repeated calls with the same inputs.
 */
int grf_sample_batched(grf_graph *const *graphs, int32_t n_graphs, const double *kappas,
                       double beta, double quad_step, int64_t n_samples, uint64_t seed,
                       double *const *outs, const grf_opts *opts);

/*
 * ---- Learned preconditioner of the vertex Schur solve ----------------------------
 * This build's addition to "Phase 4" (PCG on eq. global_schur).  A
 * message-passing network (3 layers of width 64 over vertex features: degree,
 * incident edge lengths, log(c_L / c_I), log kappa, Jacobi-scaled couplings)
 * predicts per (graph, shift) a scale-free SPD operator P_hat = diag(delta) +
 * sum over edges of PSD 2x2 blocks and an initial-guess operator Q_hat; the PCG
 * applies z = D^{-1/2} P_hat D^{-1/2} r and starts from x0 = D^{-1/2} Q_hat
 * D^{-1/2} g (D = diag S).  P_hat = I is exactly the Jacobi preconditioner,
 * which is also the fallback: a system not converged after maxit/2 iterations
 * restarts from its iterate with Jacobi; the recomputed true residual decides
 * convergence as for Jacobi.  Weights are bfloat16.  The sampler's forward keeps
 * the hidden activations in bfloat16 (64 -> 64 layer products on the bfloat16
 * matrix cores, FP32 accumulation); training runs on the GPU with FP32
 * activations (own forward / backward kernels, Adam) on the method's own
 * condensed right-hand sides and FP64 Schur solutions.
 * A network handle is used by one call at a time (its workspace is shared).
 */
/* Number of float parameters of the network. */
int grf_learned_param_count(int64_t *n_params);
/* Create from host FP32 parameters (copied; n_params must equal grf_learned_param_count). */
int grf_learned_create(const float *params, int64_t n_params, grf_learned **out);
/* Current FP32 master parameters to host memory. */
int grf_learned_params(const grf_learned *net, float *out, int64_t n_params);
int grf_learned_destroy(grf_learned *net);
/*
 * Training loss and its gradient (host FP32, n_params values) for the systems
 * S x_r = g_r of one shift (c_I, c_L) on graph g:
 *   rhs, sol   device, float64 [n_rhs][V] (g_r and the solutions x_r)
 *   loss       mean over r of (||P_hat g_hat - x_hat||^2 + ||Q_hat g_hat - x_hat||^2) / ||x_hat||^2,
 *              g_hat = D^{-1/2} g_r, x_hat = D^{1/2} x_r
 */
int grf_learned_loss_grad(grf_learned *net, grf_graph *g, double kappa, double c_I, double c_L,
                          int64_t n_rhs, const double *rhs, const double *sol, double *loss,
                          float *grad, const grf_opts *opts);
/*
 * The network's operators for one shift (c_I, c_L) on graph g, on the
 * Jacobi-scaled system (the learned operator above): device float64 outputs
 *   p_diag [V]  diagonal of P_hat (delta, the edge-end terms p and a self-loop's coupling)
 *   p_edge [E]  coupling q_e = rho sqrt(p_u p_v) of every edge
 *   q_diag [V]  diagonal of Q_hat (gamma, plus a self-loop's eta)
 *   q_edge [E]  coupling eta_e of every edge
 * activations: GRF_ACT_BF16 is the forward the sampler runs (bfloat16 hidden
 * activations and messages, 64 -> 64 products on the bfloat16 matrix cores),
 * GRF_ACT_FP32 the one training runs (FP32 activations).  p_edge and q_edge may
 * be NULL when E = 0.  Returns after the outputs are written.
 */
#define GRF_ACT_FP32 0
#define GRF_ACT_BF16 1
int grf_learned_operators(grf_learned *net, grf_graph *g, double kappa, double c_I, double c_L,
                          int32_t activations, double *p_diag, double *p_edge, double *q_diag, double *q_edge,
                          const grf_opts *opts);
/*
 * Train in place: draws n_samples noise samples per graph (seed + graph index),
 * runs the method with Jacobi PCG (FP64, opts->tol) over every shift of the
 * schedule (beta, quad_step) to collect (g, x) pairs, then takes n_steps Adam
 * steps (learning rate lr), step t on graph t mod n_graphs and a window of
 * shifts_per_step consecutive shifts.  losses (host, [n_steps]) may be NULL.
 * Each graph's sampling workspace is released once its pairs are collected (a
 * later grf_sample on it allocates again); the pairs stay on the device until
 * the call returns.
 */
int grf_learned_train(grf_learned *net, grf_graph *const *graphs, int32_t n_graphs,
                      const double *kappas, double beta, double quad_step, int64_t n_samples,
                      uint64_t seed, int32_t n_steps, int32_t shifts_per_step, double lr,
                      double *losses, const grf_opts *opts);

/* Thread-local text of the last error on this thread ("" if none). */
const char *grf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GRF_H */
