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
#include <mutex>
#include <memory>
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

// FP32 matrix-core sweeps and the mixed refinement residual are written for the lumped system
static void require_supported(const grf_graph &g, const grf_opts &o) {
    if ((g.flags & GRF_MASS_CONSISTENT_SYS) && o.precision != GRF_PREC_FP64) {
        set_error("mixed precision is not available for a graph with GRF_MASS_CONSISTENT_SYS");
        throw Error{GRF_EUNSUP};
    }
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

// bytes this graph's per-pass buffers already hold: a new plan reuses them (they grow
// by release-then-allocate), so they count as free; otherwise a second call would see
// the first call's buffers as used and plan smaller shift blocks into them
static size_t held_pass_bytes(const grf_graph &g) {
    if (!g.work) return 0;
    const grf_graph::Work &w = *g.work;
    const DevBuf *bufs[] = {&w.rho,  &w.fwdt, &w.bwdt, &w.btab, &w.ztab, &w.babs, &w.rhom,   &w.etab, &w.sd,
                            &w.so,   &w.ends, &w.gT,   &w.xT,   &w.ug,   &w.its,  &w.res,    &w.gexp, &w.pcg_ops};
    size_t t = 0;
    for (const DevBuf *b : bufs) t += b->bytes;
    return t;
}

static Plan plan_pass(const grf_graph &g, int32_t L, int64_t S, const grf_opts &o) {
    Plan p;
    // the matrix-core sweeps' closed forms need the lumped system's b < 0; a
    // consistent-mass system runs the streamed sweeps (width picked here when not given)
    const bool consistent = (g.flags & GRF_MASS_CONSISTENT_SYS) != 0;
    p.blocked = (o.sweep_block == 0) && !consistent;
    p.BL = p.blocked ? 16 : (o.sweep_block != 0 ? o.sweep_block : auto_bl(L));
    const int64_t nb = (S + 63) / 64, Sp = 64 * nb;
    // bytes per shift of the per-pass buffers
    // streamed: rho + two double2 step rows per interior DOF; blocked: per-block operand tables
    // (table elements are FP32 with mixed precision)
    const double rows = p.blocked ? 0.0 : 5.0;
    const double btab = p.blocked ? (1296.0 / 16.0 + 32.0) * ((double)g.NI / 16.0 + (double)g.E) : 0.0;
    const double tbytes = o.precision == GRF_PREC_MIXED ? 4.0 : 8.0;
    const double edge_scalars = p.blocked ? 14.0 : 4.0;  // per (edge, shift): |b|, rho, s_d, s_o (+ table scalars)
    const double per_shift = 8.0 * (rows * g.NI + edge_scalars * g.E + 2.0 * g.E * Sp + 2.0 * S * g.V +
                                    (double)g.V * Sp) +
                             tbytes * btab + 12.0 * S * (double)(g.gv0.size() - 1);
    double budget;
    if (const Arena *a = current_arena()) {
        // lent memory: most of what is left of it (the estimate above is not exact)
        budget = 0.75 * (double)(a->size - std::min(a->size, a->used));
    } else {
        size_t freeb = 0, totalb = 0;
        if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) freeb = (size_t)64 << 30;
        // the graph's pass buffers and the network's forward workspace are reused by the new plan
        const size_t lrn = (o.precond == GRF_PRECOND_LEARNED && o.learned) ? learned_held_bytes(*o.learned) : 0;
        budget = 0.5 * (double)(freeb + held_pass_bytes(g) + lrn);
    }
    int64_t lb = o.shift_block > 0 ? o.shift_block : (int64_t)std::floor(budget / per_shift);
    if (p.blocked) lb = std::min<int64_t>(lb, 128);
    lb = std::min<int64_t>(lb, L);
    if (lb < L) lb = std::max<int64_t>(p.BL, (lb / p.BL) * p.BL);
    lb = std::max<int64_t>(1, std::min<int64_t>(lb, L));
    p.LB = (int32_t)lb;
    // multi-system PCG (graphs no on-chip variant takes): resident blocks of
    // kMrhsSB samples, 5 vectors each, up to one per block of the pass and 16 GiB
    const int c0 = o.precond == GRF_PRECOND_NN ? kChipOpClasses : kPcgClasses;
    const int64_t nglob = g.cls_off[kPcgClasses + 1] - g.cls_off[c0];
    const int64_t units = nglob * lb * ((S + kMrhsSB - 1) / kMrhsSB);
    const double ubytes = 5.0 * kMrhsSB * sizeof(double) * std::max<int32_t>(g.maxVg, 1);
    const double scr_budget = current_arena() ? 0.25 * budget : 16.0 * (double)(1ull << 30);
    const int64_t cap = (int64_t)std::max(1.0, std::floor(scr_budget / ubytes));
    p.pcg_blocks = (int32_t)std::min<int64_t>(std::min<int64_t>(units, cap), 4096);
    return p;
}

static void ensure_block_offsets(grf_graph &g, grf_graph::Work &w, hipStream_t st, int64_t &nblocks) {
    std::vector<int32_t> bo(g.E + 1, 0);
    for (int64_t e = 0; e < g.E; ++e) bo[e + 1] = bo[e] + (g.m[e] + 15) / 16;
    nblocks = bo[g.E];
    upload(w.boff, bo, st);
    w.bmap.reserve(sizeof(int2) * (size_t)std::max<int64_t>(nblocks, 1));
    launch_block_map(w.boff.as<int32_t>(), g.E, w.bmap.as<int2>(), st);
}

// One run of the shift schedule over the right-hand sides in w.X, in three
// phases: prepare (planning, buffers, every upload), enqueue (kernels only, no
// host synchronisation: the part a caller may capture in a HIP graph) and
// finish (iteration counts back to the host).
struct Pass {
    Plan p;
    int32_t L = 0, nb = 0, Sp = 0, ng = 1;
    int64_t S = 0, nblocks = 0;
    int32_t LBmax = 0;  // padded shifts of the largest shift block
    std::vector<int32_t> l0s, lbs, LBps;
};

static Pass prepare_pass(grf_graph &g, const std::vector<double> &cI, const std::vector<double> &cL, int64_t S,
                         const grf_opts &o, hipStream_t st) {
    grf_graph::Work &w = work(g);
    const MeshView mv = g.view();
    Pass ps;
    ps.L = (int32_t)cI.size();
    ps.S = S;
    ps.nb = (int32_t)((S + 63) / 64);
    ps.Sp = 64 * ps.nb;
    ps.ng = mv.ng;
    ps.p = plan_pass(g, ps.L, S, o);
    for (int32_t l0 = 0; l0 < ps.L; l0 += ps.p.LB) {
        const int32_t lb = std::min(ps.p.LB, ps.L - l0);
        ps.l0s.push_back(l0);
        ps.lbs.push_back(lb);
        ps.LBps.push_back(((lb + ps.p.BL - 1) / ps.p.BL) * ps.p.BL);  // blocked: multiple of 16
        ps.LBmax = std::max(ps.LBmax, ps.LBps.back());
    }
    // all shift blocks' (c_I, c_L), block k at 2 LBmax k; padding c_L = 1 (never a divisor of 0)
    std::vector<double> sh(2 * (size_t)ps.LBmax * ps.l0s.size(), 0.0);
    for (size_t k = 0; k < ps.l0s.size(); ++k) {
        double *d = sh.data() + 2 * (size_t)ps.LBmax * k;
        for (int32_t i = 0; i < ps.LBps[k]; ++i) {
            d[2 * i] = i < ps.lbs[k] ? cI[ps.l0s[k] + i] : 0.0;
            d[2 * i + 1] = i < ps.lbs[k] ? cL[ps.l0s[k] + i] : 1.0;
        }
    }
    upload(w.shift, sh, st);
    const int32_t LBp = ps.LBmax, lb = ps.p.LB;
    const size_t nir = (size_t)std::max<int64_t>(g.NI, 1) * LBp;
    if (!ps.p.blocked) {
        w.rho.reserve(8 * nir);
        w.fwdt.reserve(16 * nir);
        w.bwdt.reserve(16 * nir);
    } else {
        ensure_block_offsets(g, w, st, ps.nblocks);
        const size_t tb = o.precision == GRF_PREC_MIXED ? sizeof(float) : sizeof(double);  // table element
        w.btab.reserve(tb * (size_t)std::max<int64_t>(ps.nblocks, 1) * block_tab_doubles(LBp / 16));
        w.ztab.reserve(tb * (size_t)std::max<int64_t>(ps.nblocks, 1) * 512 * (LBp / 16));
        w.etab.reserve(8 * (size_t)g.E * kEdgeTabFields * LBp + 8);
    }
    w.babs.reserve(8 * (size_t)g.E * LBp + 8);
    w.rhom.reserve(8 * (size_t)g.E * LBp + 8);
    w.sd.reserve(8 * (size_t)g.E * LBp + 8);
    w.so.reserve(8 * (size_t)g.E * LBp + 8);
    // end values: FP32 where the FP32 sweeps write them (mixed precision, blocked)
    const size_t eb = (ps.p.blocked && o.precision == GRF_PREC_MIXED) ? sizeof(float) : sizeof(double);
    w.ends.reserve(eb * (size_t)lb * g.E * 2 * ps.Sp + 8);
    w.gT.reserve(8 * (size_t)lb * S * g.V);
    w.xT.reserve(8 * (size_t)lb * S * g.V);
    w.ug.reserve(eb * (size_t)lb * g.V * ps.Sp);  // FP32 where the FP32 recovery reads it
    w.its.reserve(4 * (size_t)ps.ng * ps.L * S);
    w.gexp.reserve(4 * (size_t)ps.ng * ps.L * S);
    w.res.reserve(8 * (size_t)ps.ng * ps.L * S);
    w.pcg_scr.reserve(pcg_scratch_bytes(mv, ps.p.pcg_blocks));
    w.pcg_ops.reserve(pcg_ops_bytes(mv, lb, o.precond));
    prepare_pcg(mv);
    if (o.precond == GRF_PRECOND_LEARNED) learned_reserve(*const_cast<grf_learned *>(o.learned), mv, LBp);
    GRF_HIP(hipStreamSynchronize(st));  // uploads from host memory complete
    return ps;
}

static void enqueue_pass(grf_graph &g, const Pass &ps, const grf_opts &o, hipStream_t st, KTimer &T,
                         const int8_t *cls_mode = nullptr, KTimer *ct = nullptr) {
    grf_graph::Work &w = work(g);
    const MeshView mv = g.view();
    const Plan &p = ps.p;
    const int32_t nb = ps.nb, Sp = ps.Sp;
    const int64_t S = ps.S;
    T.begin(GRF_K_LAYOUT);
    if (p.blocked)
        launch_fill_rows(w.U.as<double>(), nb, g.N, g.NI, g.V, st);
    else
        launch_fill(w.U.as<double>(), (size_t)nb * g.N * 64, 0.0, st);
    T.end();
    for (size_t k = 0; k < ps.l0s.size(); ++k) {
        const int32_t l0 = ps.l0s[k], lb = ps.lbs[k], LBp = ps.LBps[k];
        CoeffArgs ca{};
        ca.shift = w.shift.as<double>() + 2 * (size_t)ps.LBmax * k;
        ca.LB = lb;
        ca.LBp = LBp;
        ca.rho = p.blocked ? nullptr : w.rho.as<double>();
        ca.fwdt = p.blocked ? nullptr : w.fwdt.as<double2>();
        ca.bwdt = p.blocked ? nullptr : w.bwdt.as<double2>();
        ca.babs = w.babs.as<double>();
        ca.rhom = w.rhom.as<double>();
        ca.sd = w.sd.as<double>();
        ca.so = w.so.as<double>();
        ca.etab = p.blocked ? w.etab.as<double>() : nullptr;
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
            ba.boff = w.boff.as<int32_t>();
            ba.bmap = w.bmap.as<int2>();
            ba.nblocks = ps.nblocks;
            ba.NT = LBp / 16;
            ba.LB = lb;
            ba.LBp = LBp;
            ba.shift = ca.shift;
            ba.babs = ca.babs;
            ba.rhom = ca.rhom;
            ba.etab = ca.etab;
            ba.tab = w.btab.as<double>();
            ba.ztab = w.ztab.as<double>();
            ba.X = sa.X;
            ba.U = sa.U;
            ba.ends = sa.ends;
            ba.ends32 = w.ends.as<float>();
            ba.ug32 = w.ug.as<float>();
            ba.ug = sa.ug;
            ba.nb = nb;
            ba.Sp = Sp;
            ba.first = (l0 == 0) ? 1 : 0;
            ba.S = S;
            ba.mixed = (o.precision == GRF_PREC_MIXED) ? 1 : 0;
            ba.tab32 = w.btab.as<float>();
            ba.ztab32 = w.ztab.as<float>();
            T.begin(GRF_K_TABLE);
            launch_blocktab(mv, ba, st);
            T.end();
            T.begin(GRF_K_ENDS_FWD);  // both directions
            launch_sweep_blocked(mv, ba, st);
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
        sc.ends32 = (p.blocked && o.precision == GRF_PREC_MIXED) ? w.ends.as<float>() : nullptr;
        sc.ug32 = (p.blocked && o.precision == GRF_PREC_MIXED) ? w.ug.as<float>() : nullptr;
        sc.sd = ca.sd;
        sc.so = ca.so;
        sc.gT = w.gT.as<double>();
        sc.xT = w.xT.as<double>();
        sc.ug = w.ug.as<double>();
        sc.U = sa.U;
        sc.scr = w.pcg_scr.as<double>();
        sc.ops = w.pcg_ops.as<double>();
        sc.its = w.its.as<int32_t>() + (size_t)ps.ng * l0 * S;  // [ng][lb][S] per shift block
        sc.gexp = w.gexp.as<int32_t>() + (size_t)ps.ng * l0 * S;
        sc.res = w.res.as<double>() + (size_t)ps.ng * l0 * S;
        sc.LB = lb;
        sc.LBp = LBp;
        sc.nb = nb;
        sc.Sp = Sp;
        sc.S = S;
        sc.tol = o.tol;
        sc.maxit = o.maxit;
        sc.pcg_blocks = p.pcg_blocks;
        sc.precond = o.precond;
        sc.cls_mode = cls_mode;
        sc.ctimer = ct;
        LearnedOps lops{};
        // the network runs only where its outputs are read: a size class with a learned
        // variant, or a graph beyond the on-chip classes
        bool net_used = false;
        if (o.precond == GRF_PRECOND_LEARNED) {
            int8_t md[kPcgClasses];
            default_chip_modes(o.precond, md);
            if (cls_mode) std::copy(cls_mode, cls_mode + kPcgClasses, md);
            net_used = mv.cls_off[kPcgClasses + 1] > mv.cls_off[kPcgClasses];
            for (int c = 0; c < kPcgClasses; ++c)
                net_used |= md[c] != CM_JACOBI && mv.cls_off[c + 1] > mv.cls_off[c];
            if (!net_used) sc.precond = GRF_PRECOND_JACOBI;
        }
        if (net_used) {
            grf_learned &net = *const_cast<grf_learned *>(o.learned);
            T.begin(GRF_K_LEARNED);
            learned_forward(net, mv, ca.shift, ca.sd, ca.so, lb, st, true);
            T.end();
            lops = learned_ops(net);
            sc.learned = &lops;
        }
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
    }
}

// the errors after which a call still writes its output
static bool soft_error(int code) { return code == GRF_ENOCONV || code == GRF_ENONFINITE; }

// Copies the iteration counts back, fills stats, throws GRF_ENONFINITE if any
// system had a NaN/Inf right-hand side or residual, else GRF_ENOCONV if any
// hit maxit.  Per-graph iteration totals go to graph_its if given.
static void finish_pass(grf_graph &g, const Pass &ps, const grf_opts &o, hipStream_t st, grf_stats *stats,
                        std::vector<int64_t> *graph_its = nullptr) {
    grf_graph::Work &w = work(g);
    const size_t n = (size_t)ps.ng * ps.L * ps.S;
    w.h_its.resize(n);
    w.h_res.resize(n);
    w.h_gexp.resize(n);
    if (n > 0) {
        GRF_HIP(hipMemcpyAsync(w.h_its.data(), w.its.ptr, 4 * n, hipMemcpyDeviceToHost, st));
        GRF_HIP(hipMemcpyAsync(w.h_res.data(), w.res.ptr, 8 * n, hipMemcpyDeviceToHost, st));
        GRF_HIP(hipMemcpyAsync(w.h_gexp.data(), w.gexp.ptr, 4 * n, hipMemcpyDeviceToHost, st));
    }
    GRF_HIP(hipStreamSynchronize(st));
    int64_t n_unconv = 0, n_bad = 0, tot_it = 0;
    int32_t max_it = 0;
    double max_res = 0.0;
    std::vector<int64_t> own_its;
    if (!graph_its && stats) graph_its = &own_its;
    if (graph_its) graph_its->assign(ps.ng, 0);
    for (size_t k = 0; k < ps.l0s.size(); ++k) {
        const size_t base = (size_t)ps.ng * ps.l0s[k] * ps.S, cnt = (size_t)ps.ng * ps.lbs[k] * ps.S;
        for (size_t i = 0; i < cnt; ++i) {
            const int32_t it = w.h_its[base + i];
            if (w.h_gexp[base + i] == kRangeNonFinite || !std::isfinite(w.h_res[base + i])) {
                n_bad++;
                continue;
            }
            if (it > o.maxit) n_unconv++;
            tot_it += std::min(it, o.maxit);
            max_it = std::max(max_it, std::min(it, o.maxit));
            max_res = std::max(max_res, w.h_res[base + i]);
            if (graph_its) (*graph_its)[i / ((size_t)ps.lbs[k] * ps.S)] += std::min(it, o.maxit);
        }
    }
    if (stats) {
        stats->n_shifts = ps.L;
        stats->n_systems = (int32_t)std::min<int64_t>((int64_t)n, INT32_MAX);
        stats->n_unconverged = (int32_t)n_unconv;
        stats->n_nonfinite = (int32_t)n_bad;
        stats->max_iterations = max_it;
        stats->total_iterations = tot_it;
        stats->max_rel_residual = max_res;
        stats->refine_steps = 0;
        stats->shift_block = ps.p.LB;
        stats->sweep_block = ps.p.blocked ? 0 : ps.p.BL;
        // iterations x vertices and x edge ends per PCG size class (the kernel that ran them)
        for (int c = 0; c <= kPcgClasses; ++c) {
            stats->pcg_class_vertex_its[c] = 0;
            stats->pcg_class_end_its[c] = 0;
        }
        for (int c = 0; c <= kPcgClasses; ++c) {
            const bool global = c == kPcgClasses || (o.precond == GRF_PRECOND_NN && c >= kChipOpClasses);
            const int bucket = global ? kPcgClasses : c;
            for (int32_t i = g.cls_off[c]; i < g.cls_off[c + 1]; ++i) {
                const int32_t gi = g.gord[i];
                const int64_t it = (*graph_its)[gi];
                stats->pcg_class_vertex_its[bucket] += it * (g.gv0[gi + 1] - g.gv0[gi]);
                stats->pcg_class_end_its[bucket] += it * 2 * (int64_t)(g.ge0[gi + 1] - g.ge0[gi]);
            }
        }
    }
    if (n_bad > 0) {
        set_error("%lld vertex Schur systems had a NaN or Inf right-hand side or residual (a non-finite input, or "
                  "with mixed precision a value beyond the FP32 range); their vertex values are NaN",
                  (long long)n_bad);
        throw Error{GRF_ENONFINITE};
    }
    if (n_unconv > 0) {
        set_error("%lld vertex Schur systems did not reach tol=%g within maxit=%d", (long long)n_unconv, o.tol,
                  o.maxit);
        throw Error{GRF_ENOCONV};
    }
}

// the per-class PCG variants the caller fixed (grf_opts.pcg_class_modes), if any
static bool given_modes(const grf_opts &o, int8_t *md) {
    if (!(o.pcg_class_modes & GRF_PCG_MODES_SET)) return false;
    for (int c = 0; c < kPcgClasses; ++c) md[c] = (int8_t)((o.pcg_class_modes >> (2 * c)) & 3);
    return true;
}

// Runs shifts (cI[i], cL[i]) on the right-hand sides in w.X into w.U (zeroed
// here: the blocked forward pass of the first shift block writes the interior
// rows, so only the vertex rows are cleared).
static void run_shifts(grf_graph &g, const std::vector<double> &cI, const std::vector<double> &cL, int64_t S,
                       const grf_opts &o, hipStream_t st, grf_stats *stats, KTimer &T) {
    const Pass ps = prepare_pass(g, cI, cL, S, o, st);
    int8_t md[kPcgClasses];
    KTimer CT(o.timing != 0, st);  // per PCG size class
    enqueue_pass(g, ps, o, st, T, given_modes(o, md) ? md : nullptr, o.timing ? &CT : nullptr);
    try {
        finish_pass(g, ps, o, st, stats);
    } catch (const Error &err) {
        if (soft_error(err.code)) CT.collect(stats);
        throw;
    }
    CT.collect(stats);
}

// ---- batches of graphs ----------------------------------------------------------
// A batch is the disjoint union of its graphs (graph k's edges and vertices in
// order after those of graphs 0..k-1), with its own workspace, the options the
// autotuner chose, and the HIP graph of its last run.
namespace {

struct Batch {
    std::vector<uint64_t> ids;
    grf_graph U;
    std::vector<double> kap2;     // per-edge kappa^2 on the device
    bool tuned = false;
    std::vector<double> tuned_key;  // (precision, preconditioner, network) the tuning was done for
    int32_t sweep_block = 0, shift_block = 0;
    int8_t tuned_mode[kPcgClasses] = {};  // learned: the tuner's PCG variant per size class (ChipMode)
    bool modes_tuned = false;             // tuned_mode was measured (not the default)
    int8_t cls_mode[kPcgClasses] = {};    // the variants of this call
    hipStream_t stream = nullptr;  // capture and replay stream (default priority)
    hipGraphExec_t exec = nullptr;
    std::vector<double> exec_key;  // parameters the captured graph was recorded with
    Pass exec_pass;
    DevBuf d_outs;
    ~Batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (stream) (void)hipStreamDestroy(stream);
        free_work(U);
    }
};

std::mutex g_batch_mu;
std::vector<std::unique_ptr<Batch>> g_batches;  // least recently used first
constexpr size_t kMaxBatches = 4;

Batch *get_batch(grf_graph *const *graphs, int32_t ng) {
    std::vector<uint64_t> ids(ng);
    for (int32_t k = 0; k < ng; ++k) ids[k] = graphs[k]->serial;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (size_t i = 0; i < g_batches.size(); ++i)
        if (g_batches[i]->ids == ids) {
            std::unique_ptr<Batch> b = std::move(g_batches[i]);
            g_batches.erase(g_batches.begin() + i);
            g_batches.push_back(std::move(b));
            return g_batches.back().get();
        }
    const grf_graph &g0 = *graphs[0];
    int64_t V = 0, E = 0;
    for (int32_t k = 0; k < ng; ++k) {
        const grf_graph &g = *graphs[k];
        GRF_REQUIRE(g.h == g0.h && g.flags == g0.flags, "the graphs of a batch must share h and the mesh rule");
        GRF_REQUIRE(g.device == g0.device, "the graphs of a batch must live on one device");
        V += g.V;
        E += g.E;
    }
    GRF_REQUIRE(V < (int64_t(1) << 31) && 2 * E < (int64_t(1) << 31), "batch too large");
    std::vector<int64_t> edges(2 * (size_t)E);
    std::vector<double> lengths(E);
    std::vector<int32_t> gv0(ng + 1, 0), ge0(ng + 1, 0);
    for (int32_t k = 0; k < ng; ++k) {
        const grf_graph &g = *graphs[k];
        for (int64_t e = 0; e < g.E; ++e) {
            edges[2 * (ge0[k] + e)] = g.eu[e] + gv0[k];
            edges[2 * (ge0[k] + e) + 1] = g.ev[e] + gv0[k];
            lengths[ge0[k] + e] = g.len[e];
        }
        gv0[k + 1] = gv0[k] + (int32_t)g.V;
        ge0[k + 1] = ge0[k] + (int32_t)g.E;
    }
    auto b = std::make_unique<Batch>();
    b->ids = ids;
    build_mesh(b->U, V, E, edges.data(), lengths.data(), g0.h, g0.flags);
    b->U.device = g0.device;
    b->U.gv0 = gv0;
    b->U.ge0 = ge0;
    upload_mesh(b->U, nullptr);
    GRF_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    g_batches.push_back(std::move(b));
    if (g_batches.size() > kMaxBatches) g_batches.erase(g_batches.begin());
    return g_batches.back().get();
}

// One uncaptured run of the batch with the given options; returns its device time in ms.
// One run of the batch on its stream; returns its time in ms.  With cls_ms, also the
// PCG time of each size class (cls_ms[kPcgClasses], summed over the shift blocks).
double timed_run(Batch &B, const Shifts &sh, int64_t S, uint64_t seed, const grf_opts &o,
                 const int8_t *cls_mode = nullptr, double *cls_ms = nullptr) {
    grf_graph &U = B.U;
    grf_graph::Work &w = work(U);
    hipStream_t cs = B.stream;
    const Pass ps = prepare_pass(U, sh.cI, sh.cL, S, o, cs);
    hipEvent_t a, b;
    GRF_HIP(hipEventCreate(&a));
    GRF_HIP(hipEventCreate(&b));
    KTimer T(false, cs);
    KTimer CT(cls_ms != nullptr, cs);
    GRF_HIP(hipEventRecord(a, cs));
    launch_noise(U.view(), S, o.sample_offset, seed, w.X.as<double>(), cs);
    enqueue_pass(U, ps, o, cs, T, cls_mode, cls_ms ? &CT : nullptr);
    GRF_HIP(hipEventRecord(b, cs));
    GRF_HIP(hipEventSynchronize(b));
    if (cls_ms) {
        for (int c = 0; c < kPcgClasses; ++c) cls_ms[c] = 0.0;
        for (const KTimer::Rec &r : CT.recs) {
            float t = 0.0f;
            GRF_HIP(hipEventElapsedTime(&t, r.a, r.b));
            if (r.id - kClassTimerId < kPcgClasses) cls_ms[r.id - kClassTimerId] += t;
        }
    }
    float ms = 0.0f;
    GRF_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

}  // namespace

void batch_forget(uint64_t serial) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (size_t i = 0; i < g_batches.size();) {
        const auto &ids = g_batches[i]->ids;
        if (std::find(ids.begin(), ids.end(), serial) != ids.end())
            g_batches.erase(g_batches.begin() + i);
        else
            ++i;
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

}  // extern "C"

namespace grf {
// grf_sample and grf_sample_from_noise: W from the Philox draw (noise null) or the caller
int sample_impl(grf_graph *g, double kappa, double beta, double quad_step, int64_t n_samples, uint64_t seed,
                       const double *noise, double *out, const grf_opts *opts) {
    GRF_REQUIRE(g, "graph is NULL");
    GRF_REQUIRE(std::isfinite(kappa) && kappa > 0, "kappa must be finite and > 0");
    GRF_REQUIRE(n_samples >= 0, "n_samples must be >= 0");
    grf_opts o = resolve_opts(opts);
    Shifts sh = make_shifts(beta, quad_step, g->h, o);
    if (n_samples == 0) return GRF_OK;
    GRF_REQUIRE(out, "out is NULL");
    GRF_REQUIRE(noise != out, "noise and out may not alias");
    require_supported(*g, o);
    GRF_REQUIRE(o.precision == GRF_PREC_FP64 || o.sweep_block == 0,
                "mixed precision runs with the blocked edge sweeps (sweep_block = 0)");
    GRF_REQUIRE(o.refine <= 0, "refinement (opts.refine > 0) applies to grf_solve_shifted only");
    hipStream_t st = (hipStream_t)o.stream;
    set_kappa2(*g, kappa, st);
    grf_graph::Work &w = work(*g);
    const int64_t nb = (n_samples + 63) / 64;
    w.X.reserve(8 * (size_t)nb * g->N * 64);
    w.U.reserve(8 * (size_t)nb * g->N * 64);
    const MeshView mv = g->view();
    if (o.stats) *o.stats = grf_stats{};
    KTimer T(o.timing != 0, st);
    if (noise) {
        T.begin(GRF_K_LAYOUT);
        launch_to_interleaved(noise, n_samples, g->N, w.X.as<double>(), st);
    } else {
        T.begin(GRF_K_NOISE);
        launch_noise(mv, n_samples, o.sample_offset, seed, w.X.as<double>(), st);
    }
    T.end();
    int code = GRF_OK;
    try {
        run_shifts(*g, sh.cI, sh.cL, n_samples, o, st, o.stats, T);
    } catch (const Error &err) {
        if (!soft_error(err.code)) throw;
        code = err.code;
    }
    T.begin(GRF_K_LAYOUT);
    launch_from_interleaved(w.U.as<double>(), n_samples, g->N, out, st);
    T.end();
    GRF_HIP(hipStreamSynchronize(st));
    T.collect(o.stats);
    return code;
}
}  // namespace grf

extern "C" {

int grf_sample(grf_graph *g, double kappa, double beta, double quad_step, int64_t n_samples, uint64_t seed,
               double *out, const grf_opts *opts) {
    GRF_API_BEGIN
    return sample_impl(g, kappa, beta, quad_step, n_samples, seed, nullptr, out, opts);
    GRF_API_END
}

int grf_sample_from_noise(grf_graph *g, double kappa, double beta, double quad_step, int64_t n_samples,
                          const double *noise, double *out, const grf_opts *opts) {
    GRF_API_BEGIN
    GRF_REQUIRE(noise || n_samples == 0, "noise is NULL");
    return sample_impl(g, kappa, beta, quad_step, n_samples, 0, noise, out, opts);
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
    require_supported(*g, o);
    GRF_REQUIRE(o.precision == GRF_PREC_FP64 || o.sweep_block == 0,
                "mixed precision runs with the blocked edge sweeps (sweep_block = 0)");
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
            if (!soft_error(err.code)) throw;
            if (code != GRF_ENONFINITE) code = err.code;
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
    GRF_REQUIRE(graphs && n_graphs > 0, "graphs must be a non-empty array");
    GRF_REQUIRE(kappas, "kappas is NULL");
    for (int32_t k = 0; k < n_graphs; ++k) {
        GRF_REQUIRE(graphs[k], "graphs[%d] is NULL", k);
        GRF_REQUIRE(std::isfinite(kappas[k]) && kappas[k] > 0, "kappas[%d] must be finite and > 0", k);
    }
    GRF_REQUIRE(n_samples >= 0, "n_samples must be >= 0");
    grf_opts o = resolve_opts(opts);
    if (n_samples == 0) return GRF_OK;
    GRF_REQUIRE(outs, "outs is NULL");
    for (int32_t k = 0; k < n_graphs; ++k) GRF_REQUIRE(outs[k], "outs[%d] is NULL", k);
    require_supported(*graphs[0], o);
    GRF_REQUIRE(o.precision == GRF_PREC_FP64 || o.sweep_block == 0,
                "mixed precision runs with the blocked edge sweeps (sweep_block = 0)");
    GRF_REQUIRE(o.refine <= 0, "refinement (opts.refine > 0) applies to grf_solve_shifted only");
    hipStream_t st = (hipStream_t)o.stream;
    Batch &B = *get_batch(graphs, n_graphs);
    grf_graph &U = B.U;
    const Shifts sh = make_shifts(beta, quad_step, U.h, o);
    const MeshView mv = U.view();
    // per-edge kappa^2 of each edge's graph
    std::vector<double> k2(U.E + 1, 0.0);
    for (int32_t k = 0; k < n_graphs; ++k)
        for (int32_t e = U.ge0[k]; e < U.ge0[k + 1]; ++e) k2[e] = kappas[k] * kappas[k];
    if (k2 != B.kap2) {
        upload(U.d_kap2, k2, B.stream);
        GRF_HIP(hipStreamSynchronize(B.stream));
        B.kap2 = k2;
    }
    grf_graph::Work &w = work(U);
    const int64_t nb = (n_samples + 63) / 64;
    w.X.reserve(8 * (size_t)nb * U.N * 64);
    w.U.reserve(8 * (size_t)nb * U.N * 64);
    GRF_HIP(hipStreamSynchronize(st));  // the caller's earlier work on its stream
    // options: the autotuner picks the sweep form and shift block unless the caller fixed them
    grf_opts run = o;
    run.timing = 0;
    auto tune_key = [&]() {
        const uint64_t ls = o.precond == GRF_PRECOND_LEARNED ? learned_signature(*o.learned) : 0;
        return std::vector<double>{(double)o.precision, (double)o.precond, (double)(ls >> 32),
                                   (double)(ls & 0xffffffffu)};
    };
    int8_t given[kPcgClasses];
    const bool has_given = given_modes(o, given);
    if (o.sweep_block == 0 && o.shift_block == 0) {
        if (!B.tuned || tune_key() != B.tuned_key) {
            std::vector<std::pair<int32_t, int32_t>> cand = {{0, 0}, {0, 64}};
            if (o.precision == GRF_PREC_FP64) {
                cand.push_back({32, 0});
                cand.push_back({64, 0});
            }
            if (U.flags & GRF_MASS_CONSISTENT_SYS) cand = {{32, 0}, {64, 0}, {32, 64}};  // streamed sweeps only
            grf_opts t = run;
            if (has_given) t.pcg_class_modes = 0;
            // the sweeps are tuned with Jacobi PCG in every size class (the choice of sweep form
            // and shift block does not depend on the PCG variant, and the learned variants would
            // add their forward pass and their own run-to-run spread to every trial)
            int8_t jac[kPcgClasses];
            for (int c = 0; c < kPcgClasses; ++c) jac[c] = CM_JACOBI;
            const int8_t *tmode = o.precond == GRF_PRECOND_LEARNED ? jac : nullptr;
            double best = 0.0;
            for (size_t c = 0; c < cand.size(); ++c) {
                t.sweep_block = cand[c].first;
                t.shift_block = cand[c].second;
                if (c == 0) (void)timed_run(B, sh, n_samples, seed, t, tmode);  // first launches of the kernels
                // the faster of two runs (a single run's spread can exceed the candidates' difference)
                const double ms = std::min(timed_run(B, sh, n_samples, seed, t, tmode),
                                           timed_run(B, sh, n_samples, seed, t, tmode));
                if (c == 0 || ms < best) {
                    best = ms;
                    B.sweep_block = t.sweep_block;
                    B.shift_block = t.shift_block;
                }
            }
            default_chip_modes(o.precond, B.tuned_mode);
            B.modes_tuned = false;
            B.tuned = true;
            B.tuned_key = tune_key();  // after the runs: the preparation may grow the network's buffers
            if (B.exec) {
                (void)hipGraphExecDestroy(B.exec);
                B.exec = nullptr;
            }
        }
        run.sweep_block = B.sweep_block;
        run.shift_block = B.shift_block;
        if (o.precond == GRF_PRECOND_LEARNED && !has_given && !B.modes_tuned) {
            // per size class, the fastest PCG variant: the learned operator and initial
            // guess, the initial guess only, or Jacobi.  Each class is its own launch,
            // so one timed run per variant (after one that loads it) times every class.
            // Any learned variant also costs the network's forward pass, which only the
            // whole run sees: a mix is kept only if it beats Jacobi everywhere (where the
            // forward pass is skipped) as a whole.
            double cms[3][kPcgClasses], tot[3];
            for (int m = 0; m < 3; ++m) {
                int8_t md[kPcgClasses];
                for (int c = 0; c < kPcgClasses; ++c) md[c] = (int8_t)(chip_mode_valid(c, m) ? m : CM_GUESS);
                (void)timed_run(B, sh, n_samples, seed, run, md);
                tot[m] = timed_run(B, sh, n_samples, seed, run, md, cms[m]);
            }
            bool all_jacobi = true;
            for (int c = 0; c < kPcgClasses; ++c) {
                int bm = CM_JACOBI;
                for (int m = 0; m < 3; ++m)
                    if (chip_mode_valid(c, m) && cms[m][c] < cms[bm][c]) bm = m;
                B.tuned_mode[c] = (int8_t)bm;
                all_jacobi &= bm == CM_JACOBI || mv.cls_off[c + 1] == mv.cls_off[c];
            }
            if (!all_jacobi) {
                const double tmix = timed_run(B, sh, n_samples, seed, run, B.tuned_mode);
                if (tmix >= tot[CM_JACOBI])
                    for (int c = 0; c < kPcgClasses; ++c) B.tuned_mode[c] = CM_JACOBI;
            }
            B.modes_tuned = true;
            B.tuned_key = tune_key();
        }
        std::copy(B.tuned_mode, B.tuned_mode + kPcgClasses, B.cls_mode);
    } else {
        default_chip_modes(o.precond, B.cls_mode);
    }
    if (has_given) std::copy(given, given + kPcgClasses, B.cls_mode);
    // everything the captured graph depends on; with the learned preconditioner also
    // the network's buffers (taken again after the capture: the preparation may grow them)
    auto make_key = [&]() {
        std::vector<double> k = {beta, sh.k, (double)sh.kminus, (double)sh.kplus, (double)n_samples,
                                 (double)(seed >> 32), (double)(seed & 0xffffffffu), (double)run.sample_offset,
                                 run.tol, (double)run.maxit, (double)run.precision, (double)run.sweep_block,
                                 (double)run.shift_block, (double)run.precond, (double)run.refine};
        const uint64_t ls = run.precond == GRF_PRECOND_LEARNED ? learned_signature(*run.learned) : 0;
        k.push_back((double)(ls >> 32));
        k.push_back((double)(ls & 0xffffffffu));
        k.insert(k.end(), kappas, kappas + n_graphs);
        k.insert(k.end(), B.cls_mode, B.cls_mode + kPcgClasses);
        return k;
    };
    const std::vector<double> key = make_key();
    hipStream_t cs = B.stream;
    if (!B.exec || key != B.exec_key) {
        if (B.exec) {
            (void)hipGraphExecDestroy(B.exec);
            B.exec = nullptr;
        }
        // every upload and allocation happens here, before the capture
        B.exec_pass = prepare_pass(U, sh.cI, sh.cL, n_samples, run, cs);
        KTimer T(false, cs);
        hipGraph_t graph = nullptr;
        GRF_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        try {
            launch_noise(mv, n_samples, run.sample_offset, seed, w.X.as<double>(), cs);
            enqueue_pass(U, B.exec_pass, run, cs, T, B.cls_mode);
        } catch (...) {
            (void)hipStreamEndCapture(cs, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        GRF_HIP(hipStreamEndCapture(cs, &graph));
        const hipError_t ie = hipGraphInstantiate(&B.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            B.exec = nullptr;
            set_error("HIP graph instantiation failed: %s", hipGetErrorString(ie));
            throw Error{GRF_EDEVICE};
        }
        B.exec_key = make_key();
    }
    // with timing the same launches run uncaptured, each bracketed by HIP events
    KTimer T(o.timing != 0, cs), CT(o.timing != 0, cs);
    if (o.timing) {
        T.begin(GRF_K_NOISE);
        launch_noise(mv, n_samples, run.sample_offset, seed, w.X.as<double>(), cs);
        T.end();
        enqueue_pass(U, B.exec_pass, run, cs, T, B.cls_mode, &CT);
    } else {
        GRF_HIP(hipGraphLaunch(B.exec, cs));
    }
    if (o.stats) *o.stats = grf_stats{};
    int code = GRF_OK;
    try {
        finish_pass(U, B.exec_pass, run, cs, o.stats);
    } catch (const Error &err) {
        if (!soft_error(err.code)) throw;
        code = err.code;
    }
    T.collect(o.stats);
    CT.collect(o.stats);
    if (o.stats) {
        int32_t mw = 0;
        for (int c = 0; c < kPcgClasses; ++c) mw |= (int32_t)B.cls_mode[c] << (2 * c);
        o.stats->pcg_class_modes = mw;
    }
    // outputs, on the caller's stream
    std::vector<double *> op(outs, outs + n_graphs);
    upload(B.d_outs, op, st);
    launch_from_interleaved_seg(mv, w.U.as<double>(), n_samples, B.d_outs.as<double *>(), st);
    GRF_HIP(hipStreamSynchronize(st));
    return code;
    GRF_API_END
}

int grf_learned_loss_grad(grf_learned *net, grf_graph *g, double kappa, double c_I, double c_L, int64_t n_rhs,
                          const double *rhs, const double *sol, double *loss, float *grad, const grf_opts *opts) {
    GRF_API_BEGIN
    GRF_REQUIRE(net && g, "net/graph is NULL");
    GRF_REQUIRE(std::isfinite(kappa) && kappa > 0, "kappa must be finite and > 0");
    GRF_REQUIRE(std::isfinite(c_I) && c_I > 0 && std::isfinite(c_L) && c_L > 0, "c_I and c_L must be finite and > 0");
    GRF_REQUIRE(n_rhs > 0 && rhs && sol && loss && grad, "need n_rhs > 0 and rhs, sol, loss, grad");
    grf_opts o = resolve_opts(opts);
    hipStream_t st = (hipStream_t)o.stream;
    set_kappa2(*g, kappa, st);
    grf_graph::Work &w = work(*g);
    const MeshView mv = g->view();
    std::vector<double> sh = {c_I, c_L};
    upload(w.shift, sh, st);
    w.babs.reserve(8 * (size_t)g->E + 8);
    w.rhom.reserve(8 * (size_t)g->E + 8);
    w.sd.reserve(8 * (size_t)g->E + 8);
    w.so.reserve(8 * (size_t)g->E + 8);
    CoeffArgs ca{};
    ca.shift = w.shift.as<double>();
    ca.LB = 1;
    ca.LBp = 1;
    ca.babs = w.babs.as<double>();
    ca.rhom = w.rhom.as<double>();
    ca.sd = w.sd.as<double>();
    ca.so = w.so.as<double>();
    launch_edge_coeff(mv, ca, st);
    learned_reserve(*net, mv, 1);
    learned_forward(*net, mv, ca.shift, ca.sd, ca.so, 1, st, false);
    *loss = learned_backward(*net, mv, rhs, sol, 1, n_rhs, st);
    learned_copy_grad(*net, grad, st);
    GRF_API_END
}

int grf_learned_operators(grf_learned *net, grf_graph *g, double kappa, double c_I, double c_L, int32_t activations,
                          double *p_diag, double *p_edge, double *q_diag, double *q_edge, const grf_opts *opts) {
    GRF_API_BEGIN
    GRF_REQUIRE(net && g, "net/graph is NULL");
    GRF_REQUIRE(std::isfinite(kappa) && kappa > 0, "kappa must be finite and > 0");
    GRF_REQUIRE(std::isfinite(c_I) && c_I > 0 && std::isfinite(c_L) && c_L > 0, "c_I and c_L must be finite and > 0");
    GRF_REQUIRE(activations == GRF_ACT_FP32 || activations == GRF_ACT_BF16, "unknown activations %d", activations);
    GRF_REQUIRE(p_diag && q_diag && (g->E == 0 || (p_edge && q_edge)), "output pointers are NULL");
    grf_opts o = resolve_opts(opts);
    hipStream_t st = (hipStream_t)o.stream;
    set_kappa2(*g, kappa, st);
    grf_graph::Work &w = work(*g);
    const MeshView mv = g->view();
    std::vector<double> sh = {c_I, c_L};
    upload(w.shift, sh, st);
    w.babs.reserve(8 * (size_t)g->E + 8);
    w.rhom.reserve(8 * (size_t)g->E + 8);
    w.sd.reserve(8 * (size_t)g->E + 8);
    w.so.reserve(8 * (size_t)g->E + 8);
    CoeffArgs ca{};
    ca.shift = w.shift.as<double>();
    ca.LB = 1;
    ca.LBp = 1;
    ca.babs = w.babs.as<double>();
    ca.rhom = w.rhom.as<double>();
    ca.sd = w.sd.as<double>();
    ca.so = w.so.as<double>();
    launch_edge_coeff(mv, ca, st);
    learned_reserve(*net, mv, 1);
    learned_forward(*net, mv, ca.shift, ca.sd, ca.so, 1, st, activations == GRF_ACT_BF16);
    const LearnedOps ops = learned_ops(*net);
    GRF_HIP(hipMemcpyAsync(p_diag, ops.Pd, 8 * (size_t)g->V, hipMemcpyDeviceToDevice, st));
    GRF_HIP(hipMemcpyAsync(q_diag, ops.Qd, 8 * (size_t)g->V, hipMemcpyDeviceToDevice, st));
    if (g->E > 0) {
        GRF_HIP(hipMemcpyAsync(p_edge, ops.Pq, 8 * (size_t)g->E, hipMemcpyDeviceToDevice, st));
        GRF_HIP(hipMemcpyAsync(q_edge, ops.Qe, 8 * (size_t)g->E, hipMemcpyDeviceToDevice, st));
    }
    GRF_HIP(hipStreamSynchronize(st));
    GRF_API_END
}

int grf_learned_train(grf_learned *net, grf_graph *const *graphs, int32_t n_graphs, const double *kappas,
                      double beta, double quad_step, int64_t n_samples, uint64_t seed, int32_t n_steps,
                      int32_t shifts_per_step, double lr, double *losses, const grf_opts *opts) {
    GRF_API_BEGIN
    GRF_REQUIRE(net && graphs && kappas && n_graphs > 0, "need a network, graphs and kappas");
    GRF_REQUIRE(n_samples > 0 && n_steps >= 0 && shifts_per_step > 0, "need n_samples > 0, n_steps >= 0, "
                "shifts_per_step > 0");
    GRF_REQUIRE(std::isfinite(lr) && lr > 0, "lr must be > 0");
    for (int32_t k = 0; k < n_graphs; ++k) {
        GRF_REQUIRE(graphs[k], "graphs[%d] is NULL", k);
        GRF_REQUIRE(std::isfinite(kappas[k]) && kappas[k] > 0, "kappas[%d] must be finite and > 0", k);
    }
    grf_opts o = resolve_opts(opts);
    hipStream_t st = (hipStream_t)o.stream;
    // training data: the method's own condensed right-hand sides and FP64 Jacobi-PCG solutions
    grf_opts gen = o;
    gen.precond = GRF_PRECOND_JACOBI;
    gen.precision = GRF_PREC_FP64;
    gen.stats = nullptr;
    gen.sample_offset = 0;
    struct Data {
        Shifts sh;
        DevBuf G, X;
    };
    std::vector<std::unique_ptr<Data>> data;
    for (int32_t k = 0; k < n_graphs; ++k) {
        grf_graph &g = *graphs[k];
        auto d = std::make_unique<Data>();
        d->sh = make_shifts(beta, quad_step, g.h, o);
        const int32_t L = (int32_t)d->sh.cI.size();
        const size_t per_shift = (size_t)n_samples * g.V;
        d->G.reserve(8 * per_shift * L);
        d->X.reserve(8 * per_shift * L);
        set_kappa2(g, kappas[k], st);
        grf_graph::Work &w = work(g);
        const int64_t nb = (n_samples + 63) / 64;
        w.X.reserve(8 * (size_t)nb * g.N * 64);
        w.U.reserve(8 * (size_t)nb * g.N * 64);
        const MeshView mv = g.view();
        launch_noise(mv, n_samples, 0, seed + (uint64_t)k, w.X.as<double>(), st);
        KTimer T(false, st);
        for (int32_t l0 = 0; l0 < L; l0 += 64) {
            const int32_t lb = std::min(64, L - l0);
            std::vector<double> cI(d->sh.cI.begin() + l0, d->sh.cI.begin() + l0 + lb);
            std::vector<double> cL(d->sh.cL.begin() + l0, d->sh.cL.begin() + l0 + lb);
            gen.shift_block = lb;
            run_shifts(g, cI, cL, n_samples, gen, st, nullptr, T);
            GRF_HIP(hipMemcpyAsync(d->G.as<double>() + per_shift * l0, w.gT.ptr, 8 * per_shift * lb,
                                   hipMemcpyDeviceToDevice, st));
            GRF_HIP(hipMemcpyAsync(d->X.as<double>() + per_shift * l0, w.xT.ptr, 8 * per_shift * lb,
                                   hipMemcpyDeviceToDevice, st));
        }
        GRF_HIP(hipStreamSynchronize(st));
        data.push_back(std::move(d));
        free_work(g);  // the sampling workspace (block tables of up to 64 shifts) is not needed for the steps
    }
    // Adam steps: graph t mod n_graphs, a window of consecutive shifts cycling through the schedule
    for (int32_t t = 0; t < n_steps; ++t) {
        const int32_t k = t % n_graphs;
        grf_graph &g = *graphs[k];
        Data &d = *data[k];
        const int32_t L = (int32_t)d.sh.cI.size();
        const int32_t lw = std::min(shifts_per_step, L);
        const int32_t ws = (int32_t)(((int64_t)(t / n_graphs) * lw) % L);
        const int32_t l1 = std::min(L, ws + lw), nl = l1 - ws;
        set_kappa2(g, kappas[k], st);
        grf_graph::Work &w = work(g);
        const MeshView mv = g.view();
        std::vector<double> sh(2 * (size_t)nl);
        for (int32_t i = 0; i < nl; ++i) {
            sh[2 * i] = d.sh.cI[ws + i];
            sh[2 * i + 1] = d.sh.cL[ws + i];
        }
        upload(w.shift, sh, st);
        w.babs.reserve(8 * (size_t)g.E * nl + 8);
        w.rhom.reserve(8 * (size_t)g.E * nl + 8);
        w.sd.reserve(8 * (size_t)g.E * nl + 8);
        w.so.reserve(8 * (size_t)g.E * nl + 8);
        CoeffArgs ca{};
        ca.shift = w.shift.as<double>();
        ca.LB = nl;
        ca.LBp = nl;
        ca.babs = w.babs.as<double>();
        ca.rhom = w.rhom.as<double>();
        ca.sd = w.sd.as<double>();
        ca.so = w.so.as<double>();
        launch_edge_coeff(mv, ca, st);
        learned_reserve(*net, mv, nl);
        learned_forward(*net, mv, ca.shift, ca.sd, ca.so, nl, st, false);
        const size_t off = (size_t)ws * n_samples * g.V;
        const double L_t = learned_backward(*net, mv, d.G.as<double>() + off, d.X.as<double>() + off, nl, n_samples, st);
        learned_adam(*net, lr, st);
        if (losses) losses[t] = L_t;
    }
    GRF_HIP(hipStreamSynchronize(st));
    GRF_API_END
}

}  // extern "C"
