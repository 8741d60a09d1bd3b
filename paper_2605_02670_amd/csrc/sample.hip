// Entry points grf_noise, grf_sample, grf_solve_shifted and the pass that
// runs a block of quadrature shifts through the condensed solve.
//
// Paper: eq. spde_approx_fem (u = sum_l A^(l)^{-1} W, one W per sample for all
// shifts) organised as Phases 3-5 of "Algorithmic Implementation": per shift,
// the condensed right-hand side (eq. local_reduced_schur), the vertex Schur
// solve (eq. global_schur), the interior recovery (eq. internal_recovery) and
// the accumulation u = sum_l u^(l).  Here the shift loop is blocked: every
// step runs for a whole block of shifts before the next step starts, so the
// noise is read once per block instead of once per shift.
#include <algorithm>
#include <cmath>

#include "work.h"

namespace grf {

void free_work(grf_graph &g) {
    delete g.work;
    g.work = nullptr;
}

grf_graph::Work &work(grf_graph &g) {
    if (!g.work) g.work = new grf_graph::Work();
    return *g.work;
}

static void set_kappa2(grf_graph &g, double kappa, hipStream_t st) {
    const double k2 = kappa * kappa;
    if (g.kap2_loaded == k2) return;
    std::vector<double> v(g.E + 1, k2);
    GRF_HIP(hipMemcpyAsync(g.d_kap2.ptr, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, st));
    GRF_HIP(hipStreamSynchronize(st));
    g.kap2_loaded = k2;
}

struct Plan {
    bool blocked = true;  // matrix-core sweeps (otherwise streamed recurrences)
    int32_t LB = 0;       // shifts per pass
    int32_t BL = 0;       // streamed: shifts per wavefront; blocked: padding granule (16)
    int32_t pcg_blocks = 0;
};

static int32_t auto_bl(int32_t L) {
    if (L >= 40) return 64;
    if (L >= 20) return 32;
    if (L >= 10) return 16;
    return 8;
}

static Plan plan_pass(const grf_graph &g, int32_t L, int64_t S, const grf_opts &o) {
    Plan p;
    p.blocked = (o.sweep_block == 0);
    p.BL = p.blocked ? 16 : o.sweep_block;
    const int64_t nb = (S + 63) / 64, Sp = 64 * nb;
    // bytes per shift of the per-pass buffers
    // streamed: rho + two double2 step rows per interior DOF; blocked: per-block operand tables
    const double rows = p.blocked ? 0.0 : 5.0;
    const double btab = p.blocked ? (1296.0 / 16.0 + 32.0) * ((double)g.NI / 16.0 + (double)g.E) : 0.0;
    const double per_shift = 8.0 * (rows * g.NI + btab + 4.0 * g.E + 2.0 * g.E * Sp + 2.0 * S * g.V +
                                    (double)g.V * Sp) + 12.0 * S;
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) freeb = (size_t)64 << 30;
    double budget = 0.5 * (double)freeb;
    int64_t lb = o.shift_block > 0 ? o.shift_block : (int64_t)std::floor(budget / per_shift);
    if (p.blocked) lb = std::min<int64_t>(lb, 128);
    lb = std::min<int64_t>(lb, L);
    if (lb < L) lb = std::max<int64_t>(p.BL, (lb / p.BL) * p.BL);
    lb = std::max<int64_t>(1, std::min<int64_t>(lb, L));
    p.LB = (int32_t)lb;
    const double vbytes = 40.0 * std::max<int64_t>(g.V, 1);
    int64_t blocks = (int64_t)std::min(2048.0, std::max(1.0, std::floor((2.0 * (1 << 30)) / vbytes)));
    p.pcg_blocks = (int32_t)blocks;
    return p;
}

static void ensure_block_offsets(grf_graph &g, grf_graph::Work &w, hipStream_t st, int64_t &nblocks) {
    std::vector<int32_t> bo(g.E + 1, 0);
    for (int64_t e = 0; e < g.E; ++e) bo[e + 1] = bo[e] + (g.m[e] + 15) / 16;
    nblocks = bo[g.E];
    upload(w.boff, bo, st);
}

// Runs shifts (cI[i], cL[i]) on the right-hand sides in w.X, accumulating into
// w.U (zeroed here: the blocked forward pass of the first shift block writes
// the interior rows, so only the vertex rows are cleared).
static void run_shifts(grf_graph &g, const std::vector<double> &cI, const std::vector<double> &cL, int64_t S,
                       const grf_opts &o, hipStream_t st, grf_stats *stats, KTimer &T) {
    grf_graph::Work &w = work(g);
    const MeshView mv = g.view();
    const int32_t L = (int32_t)cI.size();
    const int32_t nb = (int32_t)((S + 63) / 64), Sp = 64 * nb;
    const Plan p = plan_pass(g, L, S, o);
    int64_t n_unconv = 0, tot_it = 0;
    int32_t max_it = 0;
    double max_res = 0.0;
    T.begin(GRF_K_LAYOUT);
    if (p.blocked)
        launch_fill_rows(w.U.as<double>(), nb, g.N, g.NI, g.V, st);
    else
        launch_fill(w.U.as<double>(), (size_t)nb * g.N * 64, 0.0, st);
    T.end();
    for (int32_t l0 = 0; l0 < L; l0 += p.LB) {
        const int32_t lb = std::min(p.LB, L - l0);
        const int32_t LBp = ((lb + p.BL - 1) / p.BL) * p.BL;  // blocked: multiple of 16
        std::vector<double> sh(2 * (size_t)LBp, 0.0);
        for (int32_t i = 0; i < lb; ++i) {
            sh[2 * i] = cI[l0 + i];
            sh[2 * i + 1] = cL[l0 + i];
        }
        for (int32_t i = lb; i < LBp; ++i) sh[2 * i + 1] = 1.0;  // padding: never used as a divisor of 0
        upload(w.shift, sh, st);
        const size_t nir = (size_t)std::max<int64_t>(g.NI, 1) * LBp;
        if (!p.blocked) {
            w.rho.reserve(8 * nir);
            w.fwdt.reserve(16 * nir);
            w.bwdt.reserve(16 * nir);
        }
        w.babs.reserve(8 * (size_t)g.E * LBp + 8);
        w.rhom.reserve(8 * (size_t)g.E * LBp + 8);
        w.sd.reserve(8 * (size_t)g.E * LBp + 8);
        w.so.reserve(8 * (size_t)g.E * LBp + 8);
        w.ends.reserve(8 * (size_t)lb * g.E * 2 * Sp + 8);
        w.gT.reserve(8 * (size_t)lb * S * g.V);
        w.xT.reserve(8 * (size_t)lb * S * g.V);
        w.ug.reserve(8 * (size_t)lb * g.V * Sp);
        w.its.reserve(4 * (size_t)lb * S);
        w.res.reserve(8 * (size_t)lb * S);
        w.pcg_scr.reserve(pcg_scratch_bytes(mv, p.pcg_blocks));

        CoeffArgs ca{};
        ca.shift = w.shift.as<double>();
        ca.LB = lb;
        ca.LBp = LBp;
        ca.rho = p.blocked ? nullptr : w.rho.as<double>();
        ca.fwdt = p.blocked ? nullptr : w.fwdt.as<double2>();
        ca.bwdt = p.blocked ? nullptr : w.bwdt.as<double2>();
        ca.babs = w.babs.as<double>();
        ca.rhom = w.rhom.as<double>();
        ca.sd = w.sd.as<double>();
        ca.so = w.so.as<double>();
        T.begin(GRF_K_COEFF);
        if (p.blocked)
            launch_edge_coeff(mv, ca, st);
        else
            launch_coeff(mv, ca, st);
        T.end();

        SweepArgs sa{};
        sa.X = w.X.as<double>();
        sa.U = w.U.as<double>();
        sa.rho = ca.rho;
        sa.fwdt = ca.fwdt;
        sa.bwdt = ca.bwdt;
        sa.babs = ca.babs;
        sa.rhom = ca.rhom;
        sa.ug = w.ug.as<double>();
        sa.ends = w.ends.as<double>();
        sa.LB = lb;
        sa.LBp = LBp;
        sa.nb = nb;
        sa.Sp = Sp;
        sa.bl = p.BL;

        BlockArgs ba{};
        if (p.blocked) {
            int64_t nblocks = 0;
            ensure_block_offsets(g, w, st, nblocks);
            ba.boff = w.boff.as<int32_t>();
            ba.nblocks = nblocks;
            ba.NT = LBp / 16;
            ba.LB = lb;
            ba.LBp = LBp;
            ba.shift = ca.shift;
            ba.babs = ca.babs;
            ba.rhom = ca.rhom;
            w.btab.reserve(8 * (size_t)std::max<int64_t>(nblocks, 1) * block_tab_doubles(ba.NT));
            w.ztab.reserve(8 * (size_t)std::max<int64_t>(nblocks, 1) * 512 * ba.NT);
            ba.tab = w.btab.as<double>();
            ba.ztab = w.ztab.as<double>();
            ba.X = sa.X;
            ba.U = sa.U;
            ba.ends = sa.ends;
            ba.ug = sa.ug;
            ba.nb = nb;
            ba.Sp = Sp;
            ba.first = (l0 == 0) ? 1 : 0;
            ba.mixed = (o.precision == GRF_PREC_MIXED) ? 1 : 0;
            ba.tab32 = w.btab.as<float>();
            ba.ztab32 = w.ztab.as<float>();
            T.begin(GRF_K_COEFF);
            launch_blocktab(mv, ba, st);
            T.end();
            T.begin(GRF_K_ENDS_FWD);
            launch_sweep_blocked(mv, ba, true, st);
            T.end();
            T.begin(GRF_K_ENDS_BWD);
            launch_sweep_blocked(mv, ba, false, st);
            T.end();
        } else {
            T.begin(GRF_K_ENDS_FWD);
            launch_sweep_ends(mv, sa, true, st);
            T.end();
            T.begin(GRF_K_ENDS_BWD);
            launch_sweep_ends(mv, sa, false, st);
            T.end();
        }

        SchurArgs sc{};
        sc.X = sa.X;
        sc.ends = sa.ends;
        sc.sd = ca.sd;
        sc.so = ca.so;
        sc.gT = w.gT.as<double>();
        sc.xT = w.xT.as<double>();
        sc.ug = w.ug.as<double>();
        sc.U = sa.U;
        sc.scr = w.pcg_scr.as<double>();
        sc.its = w.its.as<int32_t>();
        sc.res = w.res.as<double>();
        sc.LB = lb;
        sc.LBp = LBp;
        sc.nb = nb;
        sc.Sp = Sp;
        sc.S = S;
        sc.tol = o.tol;
        sc.maxit = o.maxit;
        sc.pcg_blocks = p.pcg_blocks;
        T.begin(GRF_K_CONDENSE);
        launch_condense(mv, sc, st);
        T.end();
        T.begin(GRF_K_PCG);
        launch_pcg(mv, sc, st);
        T.end();
        T.begin(GRF_K_SCATTER);
        launch_vertex_scatter(mv, sc, st);
        T.end();
        if (p.blocked) {
            T.begin(GRF_K_ACC_FWD);
            launch_corr_blocked(mv, ba, st);
            T.end();
        } else {
            T.begin(GRF_K_ACC_FWD);
            launch_sweep_acc(mv, sa, true, st);
            T.end();
            T.begin(GRF_K_ACC_BWD);
            launch_sweep_acc(mv, sa, false, st);
            T.end();
        }

        w.h_its.resize((size_t)lb * S);
        w.h_res.resize((size_t)lb * S);
        GRF_HIP(hipMemcpyAsync(w.h_its.data(), w.its.ptr, 4 * (size_t)lb * S, hipMemcpyDeviceToHost, st));
        GRF_HIP(hipMemcpyAsync(w.h_res.data(), w.res.ptr, 8 * (size_t)lb * S, hipMemcpyDeviceToHost, st));
        GRF_HIP(hipStreamSynchronize(st));
        for (size_t i = 0; i < w.h_its.size(); ++i) {
            const int32_t it = w.h_its[i];
            if (it > o.maxit) n_unconv++;
            tot_it += std::min(it, o.maxit);
            max_it = std::max(max_it, std::min(it, o.maxit));
            max_res = std::max(max_res, w.h_res[i]);
        }
    }
    if (stats) {
        stats->n_shifts = L;
        stats->n_systems = (int32_t)std::min<int64_t>((int64_t)L * S, INT32_MAX);
        stats->n_unconverged = (int32_t)n_unconv;
        stats->max_iterations = max_it;
        stats->total_iterations = tot_it;
        stats->max_rel_residual = max_res;
        stats->refine_steps = 0;
        stats->shift_block = p.LB;
        stats->sweep_block = p.blocked ? 0 : p.BL;
    }
    if (n_unconv > 0) {
        set_error("%lld vertex Schur systems did not reach tol=%g within maxit=%d", (long long)n_unconv, o.tol,
                  o.maxit);
        throw Error{GRF_ENOCONV};
    }
}

}  // namespace grf

using namespace grf;

#define GRF_API_BEGIN try {
#define GRF_API_END                                       \
    }                                                     \
    catch (const ::grf::Error &err) { return err.code; }  \
    catch (const std::bad_alloc &) {                      \
        ::grf::set_error("host allocation failed");        \
        return GRF_ENOMEM;                                \
    }                                                     \
    catch (...) {                                         \
        ::grf::set_error("unexpected internal error");     \
        return GRF_EDEVICE;                               \
    }                                                     \
    return GRF_OK;

extern "C" {

int grf_noise(grf_graph *g, int64_t n_samples, uint64_t seed, double *out, const grf_opts *opts) {
    GRF_API_BEGIN
    GRF_REQUIRE(g, "graph is NULL");
    GRF_REQUIRE(n_samples >= 0, "n_samples must be >= 0");
    grf_opts o = resolve_opts(opts);
    if (n_samples == 0) return GRF_OK;
    GRF_REQUIRE(out, "out is NULL");
    hipStream_t st = (hipStream_t)o.stream;
    grf_graph::Work &w = work(*g);
    const int64_t nb = (n_samples + 63) / 64;
    w.X.reserve(8 * (size_t)nb * g->N * 64);
    const MeshView mv = g->view();
    launch_noise(mv, n_samples, o.sample_offset, seed, w.X.as<double>(), st);
    launch_from_interleaved(w.X.as<double>(), n_samples, g->N, out, st);
    GRF_HIP(hipStreamSynchronize(st));
    GRF_API_END
}

int grf_sample(grf_graph *g, double kappa, double beta, double quad_step, int64_t n_samples, uint64_t seed,
               double *out, const grf_opts *opts) {
    GRF_API_BEGIN
    GRF_REQUIRE(g, "graph is NULL");
    GRF_REQUIRE(std::isfinite(kappa) && kappa > 0, "kappa must be finite and > 0");
    GRF_REQUIRE(n_samples >= 0, "n_samples must be >= 0");
    grf_opts o = resolve_opts(opts);
    Shifts sh = make_shifts(beta, quad_step, g->h, o);
    if (n_samples == 0) return GRF_OK;
    GRF_REQUIRE(out, "out is NULL");
    GRF_REQUIRE(o.precision == GRF_PREC_FP64 || o.sweep_block == 0,
                "mixed precision runs with the blocked edge sweeps (sweep_block = 0)");
    GRF_REQUIRE(o.precond == GRF_PRECOND_JACOBI, "learned preconditioner is not available in this build");
    hipStream_t st = (hipStream_t)o.stream;
    set_kappa2(*g, kappa, st);
    grf_graph::Work &w = work(*g);
    const int64_t nb = (n_samples + 63) / 64;
    w.X.reserve(8 * (size_t)nb * g->N * 64);
    w.U.reserve(8 * (size_t)nb * g->N * 64);
    const MeshView mv = g->view();
    if (o.stats) *o.stats = grf_stats{};
    KTimer T(o.timing != 0, st);
    T.begin(GRF_K_NOISE);
    launch_noise(mv, n_samples, o.sample_offset, seed, w.X.as<double>(), st);
    T.end();
    int code = GRF_OK;
    try {
        run_shifts(*g, sh.cI, sh.cL, n_samples, o, st, o.stats, T);
    } catch (const Error &err) {
        if (err.code != GRF_ENOCONV) throw;
        code = GRF_ENOCONV;
    }
    T.begin(GRF_K_LAYOUT);
    launch_from_interleaved(w.U.as<double>(), n_samples, g->N, out, st);
    T.end();
    GRF_HIP(hipStreamSynchronize(st));
    T.collect(o.stats);
    return code;
    GRF_API_END
}

int grf_solve_shifted(grf_graph *g, double kappa, double c_I, double c_L, int64_t n_rhs, const double *rhs,
                      double *out, const grf_opts *opts) {
    GRF_API_BEGIN
    GRF_REQUIRE(g, "graph is NULL");
    GRF_REQUIRE(std::isfinite(kappa) && kappa >= 0, "kappa must be finite and >= 0");
    GRF_REQUIRE(std::isfinite(c_I) && c_I > 0 && std::isfinite(c_L) && c_L > 0, "c_I and c_L must be finite and > 0");
    GRF_REQUIRE(n_rhs >= 0, "n_rhs must be >= 0");
    grf_opts o = resolve_opts(opts);
    if (n_rhs == 0) return GRF_OK;
    GRF_REQUIRE(rhs && out, "rhs/out is NULL");
    GRF_REQUIRE(rhs != out, "rhs and out may not alias");
    GRF_REQUIRE(o.precision == GRF_PREC_FP64 || o.sweep_block == 0,
                "mixed precision runs with the blocked edge sweeps (sweep_block = 0)");
    GRF_REQUIRE(o.precond == GRF_PRECOND_JACOBI, "learned preconditioner is not available in this build");
    hipStream_t st = (hipStream_t)o.stream;
    set_kappa2(*g, kappa, st);
    grf_graph::Work &w = work(*g);
    const int64_t nb = (n_rhs + 63) / 64;
    const size_t nel = (size_t)nb * g->N * 64;
    w.X.reserve(8 * nel);
    w.U.reserve(8 * nel);
    const bool mixed = o.precision == GRF_PREC_MIXED;
    const int32_t nref = mixed ? (o.refine < 0 ? 2 : o.refine) : 0;
    if (o.stats) *o.stats = grf_stats{};
    KTimer T(o.timing != 0, st);
    T.begin(GRF_K_LAYOUT);
    launch_to_interleaved(rhs, n_rhs, g->N, w.X.as<double>(), st);
    T.end();
    std::vector<double> cI(1, c_I), cL(1, c_L);
    const MeshView mv = g->view();
    int code = GRF_OK;
    auto solve = [&]() {
        try {
            run_shifts(*g, cI, cL, n_rhs, o, st, o.stats, T);
        } catch (const Error &err) {
            if (err.code != GRF_ENOCONV) throw;
            code = GRF_ENOCONV;
        }
    };
    double *result = w.U.as<double>();
    if (nref > 0) {
        // x_0 = A^{-1} b with FP32 sweeps; then x <- x + A^{-1} (b - A x), residual in FP64
        w.Bm.reserve(8 * nel);
        w.Xacc.reserve(8 * nel);
        const int64_t chunks = colnorm_chunks(g->N);
        w.nrm.reserve(8 * (size_t)nb * chunks * 64);
        GRF_HIP(hipMemcpyAsync(w.Bm.ptr, w.X.ptr, 8 * nel, hipMemcpyDeviceToDevice, st));
        solve();
        GRF_HIP(hipMemcpyAsync(w.Xacc.ptr, w.U.ptr, 8 * nel, hipMemcpyDeviceToDevice, st));
        auto rel_residual = [&]() -> double {  // max over rhs of ||b - A x|| / ||b||
            std::vector<double> pr((size_t)nb * chunks * 64), pb((size_t)nb * chunks * 64);
            launch_colnorm2(w.X.as<double>(), g->N, (int32_t)nb, w.nrm.as<double>(), st);
            GRF_HIP(hipMemcpyAsync(pr.data(), w.nrm.ptr, 8 * pr.size(), hipMemcpyDeviceToHost, st));
            GRF_HIP(hipStreamSynchronize(st));
            launch_colnorm2(w.Bm.as<double>(), g->N, (int32_t)nb, w.nrm.as<double>(), st);
            GRF_HIP(hipMemcpyAsync(pb.data(), w.nrm.ptr, 8 * pb.size(), hipMemcpyDeviceToHost, st));
            GRF_HIP(hipStreamSynchronize(st));
            double worst = 0.0;
            for (int64_t s = 0; s < n_rhs; ++s) {
                const int64_t b = s / 64, lane = s % 64;
                double rr = 0.0, bb = 0.0;
                for (int64_t c = 0; c < chunks; ++c) {
                    rr += pr[(b * chunks + c) * 64 + lane];
                    bb += pb[(b * chunks + c) * 64 + lane];
                }
                if (bb > 0.0) worst = std::max(worst, std::sqrt(rr / bb));
            }
            return worst;
        };
        double rel = 0.0;
        int32_t done = 0;
        for (int32_t it = 0; it < nref; ++it) {
            T.begin(GRF_K_MIXED);
            launch_residual(mv, c_I, c_L, w.Bm.as<double>(), w.Xacc.as<double>(), w.X.as<double>(), (int32_t)nb, st);
            T.end();
            solve();
            T.begin(GRF_K_MIXED);
            launch_axpy1(w.U.as<double>(), w.Xacc.as<double>(), (int64_t)nel, st);
            T.end();
            done++;
        }
        launch_residual(mv, c_I, c_L, w.Bm.as<double>(), w.Xacc.as<double>(), w.X.as<double>(), (int32_t)nb, st);
        rel = rel_residual();
        if (o.stats) {
            o.stats->refine_steps = done;
            o.stats->max_rel_residual = rel;  // of the refined solution in the full system
        }
        result = w.Xacc.as<double>();
    } else {
        solve();
    }
    T.begin(GRF_K_LAYOUT);
    launch_from_interleaved(result, n_rhs, g->N, out, st);
    T.end();
    GRF_HIP(hipStreamSynchronize(st));
    T.collect(o.stats);
    return code;
    GRF_API_END
}

int grf_sample_batched(grf_graph *const *graphs, int32_t n_graphs, const double *kappas, double beta,
                       double quad_step, int64_t n_samples, uint64_t seed, double *const *outs, const grf_opts *opts) {
    GRF_API_BEGIN
    (void)graphs; (void)n_graphs; (void)kappas; (void)beta; (void)quad_step; (void)n_samples; (void)seed;
    (void)outs; (void)opts;
    set_error("grf_sample_batched is not available in this build");
    return GRF_EUNSUP;
    GRF_API_END
}

}  // extern "C"
