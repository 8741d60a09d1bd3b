// Graph handle, mesh and DOF numbering, quadrature schedule (host side).
//
// Mesh: paper section "Algorithmic Implementation", "Phase 1: Initialization"
// (n_e uniform elements per edge, h_e = l_e / n_e, N = |V| + sum_e (N_e - 2)).
// Lumped mass: "Phase 2", lumped case (h_e inside an edge, sum of h_e/2 at a
// vertex) and "Mass Lumping" (R = element-wise square root).
// Shift schedule: eq. coefficients and the limits K^-, K^+ of the "Strong
// error" subsection.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "common.h"
#include <algorithm>
#include <atomic>

#include "work.h"

namespace grf {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

static thread_local Arena *g_arena = nullptr;

Arena *current_arena() { return g_arena; }

ArenaScope::ArenaScope(Arena *a) : prev(g_arena) { g_arena = a; }

ArenaScope::~ArenaScope() { g_arena = prev; }

DevBuf::~DevBuf() { release(); }

void DevBuf::release() {
    if (ptr && !borrowed) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
    borrowed = false;
}

void DevBuf::reserve(size_t n) {
    if (n <= bytes) return;
    release();
    if (n == 0) return;
    if (Arena *a = g_arena) {
        const size_t at = (a->used + 255) & ~(size_t)255;
        if (at > a->size || n > a->size - at) {
            set_error("%s: the workspace needs more than its %zu-byte scratch (%zu bytes more requested with "
                      "%zu in use)", a->owner, a->size, n, at);
            throw Error{GRF_EINVAL};
        }
        ptr = a->base + at;
        bytes = n;
        borrowed = true;
        a->used = at + n;
        return;
    }
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
        ptr = nullptr;
        set_error("hipMalloc(%zu bytes) failed: %s", n, hipGetErrorString(e));
        throw Error{GRF_ENOMEM};
    }
    bytes = n;
}

KTimer::~KTimer() {
    for (auto &r : recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
}

static_assert(GRF_K_COUNT <= 16, "kernel ids fit grf_stats.kernel_ms");
static_assert(offsetof(grf_stats, pcg_class_ms) == 240 && sizeof(grf_stats) == 440, "grf_stats layout");

void KTimer::begin(int id) {
    if (!on) return;
    Rec r{id, nullptr, nullptr};
    GRF_HIP(hipEventCreate(&r.a));
    GRF_HIP(hipEventCreate(&r.b));
    GRF_HIP(hipEventRecord(r.a, st));
    recs.push_back(r);
}

void KTimer::end() {
    if (!on || recs.empty()) return;
    GRF_HIP(hipEventRecord(recs.back().b, st));
}

void KTimer::collect(grf_stats *stats) {
    if (!on || !stats) return;
    for (auto &r : recs) {
        float ms = 0.f;
        GRF_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        if (r.id >= 0 && r.id < GRF_K_COUNT) {
            stats->kernel_ms[r.id] += ms;
            stats->kernel_launches[r.id] += 1;
        } else if (r.id >= kClassTimerId && r.id <= kClassTimerId + kPcgClasses) {
            stats->pcg_class_ms[r.id - kClassTimerId] += ms;
            stats->pcg_class_launches[r.id - kClassTimerId] += 1;
        }
    }
}

void build_mesh(grf_graph &g, int64_t V, int64_t E, const int64_t *edges, const double *lengths, double h,
                uint32_t flags) {
    GRF_REQUIRE(V >= 1 && V < (int64_t(1) << 31), "n_vertices must be in [1, 2^31)");
    GRF_REQUIRE(E >= 0 && E < (int64_t(1) << 30), "n_edges must be in [0, 2^30)");
    GRF_REQUIRE(E == 0 || (edges && lengths), "edges and lengths must be non-NULL");
    GRF_REQUIRE(std::isfinite(h) && h > 0, "h must be finite and > 0");
    GRF_REQUIRE((flags & ~(GRF_MESH_ROUND | GRF_MASS_CONSISTENT_SYS | GRF_NOISE_CONSISTENT)) == 0,
                "unknown mesh flag %u", flags);
    g.V = V;
    g.E = E;
    g.h = h;
    g.flags = flags;
    g.eu.resize(E);
    g.ev.resize(E);
    g.len.resize(E);
    g.m.resize(E);
    g.he.resize(E);
    g.off.resize(E + 1);
    std::vector<int64_t> deg(V, 0);
    g.off[0] = 0;
    for (int64_t e = 0; e < E; ++e) {
        int64_t u = edges[2 * e], v = edges[2 * e + 1];
        double L = lengths[e];
        GRF_REQUIRE(u >= 0 && u < V && v >= 0 && v < V, "edge %lld endpoint out of range", (long long)e);
        GRF_REQUIRE(std::isfinite(L) && L > 0, "edge %lld length must be finite and > 0", (long long)e);
        double q = L / h;
        double n = (flags & GRF_MESH_ROUND) ? std::floor(q + 0.5) : std::ceil(q);
        double nmin = (u == v) ? 2.0 : 1.0;
        if (n < nmin) n = nmin;
        GRF_REQUIRE(n < 1e9, "edge %lld needs too many elements", (long long)e);
        g.eu[e] = u;
        g.ev[e] = v;
        g.len[e] = L;
        g.m[e] = (int32_t)(n - 1);
        g.he[e] = L / n;
        g.off[e + 1] = g.off[e] + g.m[e];
        deg[u]++;
        deg[v]++;
    }
    for (int64_t v = 0; v < V; ++v)
        GRF_REQUIRE(deg[v] > 0, "vertex %lld has no incident edge (zero lumped mass, singular system)",
                    (long long)v);
    g.NI = g.off[E];
    g.N = g.NI + V;
    GRF_REQUIRE(g.N < (int64_t(1) << 40), "too many DOFs");
    // lumped mass diagonal: interior h_e, vertices summed over edges in order, tail end first
    g.ml.assign(g.N, 0.0);
    for (int64_t e = 0; e < E; ++e)
        for (int64_t p = g.off[e]; p < g.off[e + 1]; ++p) g.ml[p] = g.he[e];
    for (int64_t e = 0; e < E; ++e) {
        double half = g.he[e] * 0.5;
        g.ml[g.NI + g.eu[e]] += half;
        g.ml[g.NI + g.ev[e]] += half;
    }
    // CSR over edge ends, ends listed in increasing edge order
    g.vptr.assign(V + 1, 0);
    for (int64_t v = 0; v < V; ++v) g.vptr[v + 1] = g.vptr[v] + deg[v];
    std::vector<int64_t> fill(g.vptr.begin(), g.vptr.end() - 1);
    g.adj_e.resize(2 * E);
    g.adj_o.resize(2 * E);
    g.adj_s.resize(2 * E);
    for (int64_t e = 0; e < E; ++e) {
        int64_t a = fill[g.eu[e]]++;
        g.adj_e[a] = (int32_t)e;
        g.adj_o[a] = (int32_t)g.ev[e];
        g.adj_s[a] = 0;
        int64_t b = fill[g.ev[e]]++;
        g.adj_e[b] = (int32_t)e;
        g.adj_o[b] = (int32_t)g.eu[e];
        g.adj_s[b] = 1;
    }
}

void prepare_mesh(grf_graph &g, Uploads &up) {
    std::vector<int32_t> eu(g.E), ev(g.E);
    for (int64_t e = 0; e < g.E; ++e) {
        eu[e] = (int32_t)g.eu[e];
        ev[e] = (int32_t)g.ev[e];
    }
    std::vector<double> msq(g.N);
    for (int64_t j = 0; j < g.N; ++j) msq[j] = std::sqrt(g.ml[j]);
    up.add(g.d_off, g.off);
    up.add(g.d_m, g.m);
    up.add(g.d_eu, std::move(eu));
    up.add(g.d_ev, std::move(ev));
    up.add(g.d_he, g.he);
    up.add(g.d_vptr, g.vptr);
    up.add(g.d_adj_e, g.adj_e);
    up.add(g.d_adj_o, g.adj_o);
    up.add(g.d_adj_s, g.adj_s);
    up.add(g.d_msqrt, std::move(msq));
    if (g.gv0.empty()) {
        g.gv0 = {0, (int32_t)g.V};
        g.ge0 = {0, (int32_t)g.E};
    }
    const int64_t ng = (int64_t)g.gv0.size() - 1;
    g.segs.assign(4 * ng, 0);
    g.tile0.assign(ng + 1, 0);
    g.maxVg = g.maxEg = 0;
    g.maxNg = 0;
    for (int64_t k = 0; k < ng; ++k) {
        const int64_t i0 = g.off[g.ge0[k]], i1 = g.off[g.ge0[k + 1]];
        const int64_t vk = g.gv0[k + 1] - g.gv0[k];
        g.segs[4 * k + 0] = (i1 - i0) + vk;
        g.segs[4 * k + 1] = i1 - i0;
        g.segs[4 * k + 2] = i0;
        g.segs[4 * k + 3] = g.NI + g.gv0[k];
        g.maxVg = std::max<int32_t>(g.maxVg, (int32_t)vk);
        g.maxEg = std::max<int32_t>(g.maxEg, g.ge0[k + 1] - g.ge0[k]);
        g.maxNg = std::max<int64_t>(g.maxNg, g.segs[4 * k]);
        g.tile0[k + 1] = g.tile0[k] + (g.segs[4 * k] + 63) / 64;
    }
    g.max_deg = 0;
    for (int64_t u = 0; u < g.V; ++u) g.max_deg = std::max<int32_t>(g.max_deg, (int32_t)(g.vptr[u + 1] - g.vptr[u]));
    std::vector<int32_t> ell(4 * (size_t)g.V), eend(4 * (size_t)g.V), deg(g.V);
    for (int64_t u = 0; u < g.V; ++u) {
        deg[u] = (int32_t)(g.vptr[u + 1] - g.vptr[u]);
        for (int j = 0; j < 4; ++j) {
            const int64_t k = g.vptr[u] + j;
            ell[(size_t)j * g.V + u] = j < deg[u] ? g.adj_o[k] : (int32_t)u;
            eend[(size_t)j * g.V + u] = j < deg[u] ? 2 * g.adj_e[k] + g.adj_s[k] : -1;
        }
    }
    up.add(g.d_ell, ell);
    up.add(g.d_eend, std::move(eend));
    up.add(g.d_deg, deg);
    // PCG size classes, each ordered largest graph first
    std::vector<int32_t> cls(ng);
    for (int64_t k = 0; k < ng; ++k) {
        const int32_t vk = g.gv0[k + 1] - g.gv0[k];
        int c = 0;
        while (c < kPcgClasses && vk > kPcgCap[c]) ++c;
        cls[k] = c;
    }
    g.gord.resize(ng);
    for (int64_t k = 0; k < ng; ++k) g.gord[k] = (int32_t)k;
    std::stable_sort(g.gord.begin(), g.gord.end(), [&](int32_t a, int32_t b) {
        if (cls[a] != cls[b]) return cls[a] < cls[b];
        return g.gv0[a + 1] - g.gv0[a] > g.gv0[b + 1] - g.gv0[b];
    });
    for (int c = 0; c <= kPcgClasses + 1; ++c) {
        int32_t n = 0;
        for (int64_t k = 0; k < ng; ++k) n += cls[k] < c ? 1 : 0;
        g.cls_off[c] = n;
    }
    up.add(g.d_gord, g.gord);
    // 16-bit local neighbour ids and overflow masks for the graphs of an on-chip class
    std::vector<uint32_t> e16(2 * (size_t)g.V, 0), om(16 * (size_t)ng, 0);
    for (int64_t k = 0; k < ng; ++k) {
        const int c = cls[k];
        if (c >= kPcgClasses) continue;
        const int32_t u0 = g.gv0[k], nv = g.gv0[k + 1] - u0;
        for (int32_t v = 0; v < nv; ++v) {
            const int64_t u = u0 + v;
            uint32_t id[4];
            for (int j = 0; j < 4; ++j) id[j] = (uint32_t)(ell[(size_t)j * g.V + u] - u0);
            e16[2 * u] = id[0] | (id[1] << 16);
            e16[2 * u + 1] = id[2] | (id[3] << 16);
            if (deg[u] > 4) {
                const int tpb = kChipTpb[c];
                const int t = v % tpb, i = v / tpb;
                om[16 * k + t / 64] |= 1u << i;
            }
        }
    }
    up.add(g.d_ell16, std::move(e16));
    up.add(g.d_ovfm, std::move(om));
    // overflow slots as pieces of at most 64 packed into chunks of 64 entries (MeshView::ovent)
    {
        std::vector<int32_t> ent, ent0(ng + 1, 0), np(ng, 0), pc(2 * (size_t)g.V, 0);
        for (int64_t k = 0; k < ng; ++k) {
            ent0[k] = (int32_t)(ent.size() / 4);
            if (cls[k] >= kPcgClasses) continue;
            const int32_t u0 = g.gv0[k], nv = g.gv0[k + 1] - u0;
            int32_t piece = 0, fill = 0;  // entries used in the current chunk
            for (int32_t v = 0; v < nv; ++v) {
                const int64_t u = u0 + v;
                if (deg[u] <= 4) continue;
                const int64_t q0 = g.vptr[u] + 4, q1 = g.vptr[u + 1];
                pc[2 * u] = piece;
                for (int64_t a = q0; a < q1; a += 64) {
                    const int32_t len = (int32_t)std::min<int64_t>(64, q1 - a);
                    if (fill + len > 64) {  // pad the chunk
                        for (; fill < 64; ++fill) ent.insert(ent.end(), {0, -1, 0, 0});
                        fill = 0;
                    }
                    for (int64_t q = a; q < a + len; ++q)
                        ent.insert(ent.end(), {(int32_t)q, piece, v, g.adj_o[q] - u0});
                    fill = (fill + len) % 64;
                    ++piece;
                }
                pc[2 * u + 1] = piece;
            }
            for (; fill > 0 && fill < 64; ++fill) ent.insert(ent.end(), {0, -1, 0, 0});
            np[k] = piece;
        }
        ent0[ng] = (int32_t)(ent.size() / 4);
        ent.insert(ent.end(), {0, -1, 0, 0});  // never empty
        up.add(g.d_ovent, std::move(ent));
        up.add(g.d_ovent0, std::move(ent0));
        up.add(g.d_ovnp, std::move(np));
        up.add(g.d_ovpc, std::move(pc));
    }
    // vertex PCG row order: reverse Cuthill-McKee for the graphs beyond every on-chip
    // class (their neighbour gathers then stay close in memory), vertex order otherwise
    std::vector<int32_t> prow(g.V), pvtx(g.V), pell(4 * (size_t)g.V), padj(g.adj_o.size());
    for (int64_t u = 0; u < g.V; ++u) prow[u] = pvtx[u] = (int32_t)u;
    for (int64_t k = 0; k < ng; ++k) {
        if (cls[k] < kPcgClasses) continue;
        const int32_t u0 = g.gv0[k], nv = g.gv0[k + 1] - u0;
        std::vector<int32_t> byd(nv), order;
        order.reserve(nv);
        for (int32_t v = 0; v < nv; ++v) byd[v] = v;
        std::stable_sort(byd.begin(), byd.end(), [&](int32_t a, int32_t b) { return deg[u0 + a] < deg[u0 + b]; });
        std::vector<char> seen(nv, 0);
        std::vector<int32_t> nb;
        for (int32_t st0 : byd) {  // each component from its least-connected vertex, breadth first
            if (seen[st0]) continue;
            seen[st0] = 1;
            size_t head = order.size();
            order.push_back(st0);
            while (head < order.size()) {
                const int32_t v = order[head++];
                nb.clear();
                for (int64_t q = g.vptr[u0 + v]; q < g.vptr[u0 + v + 1]; ++q) {
                    const int32_t w = g.adj_o[q] - u0;
                    if (!seen[w]) {
                        seen[w] = 1;
                        nb.push_back(w);
                    }
                }
                std::stable_sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg[u0 + a] < deg[u0 + b]; });
                order.insert(order.end(), nb.begin(), nb.end());
            }
        }
        GRF_REQUIRE((int32_t)order.size() == nv, "internal: vertex order incomplete");
        for (int32_t r = 0; r < nv; ++r) {  // reversed
            const int32_t v = order[nv - 1 - r];
            pvtx[u0 + r] = u0 + v;
            prow[u0 + v] = u0 + r;
        }
    }
    for (int64_t k = 0; k < ng; ++k) {
        const int32_t u0 = g.gv0[k];
        for (int32_t r = u0; r < g.gv0[k + 1]; ++r) {
            const int32_t u = pvtx[r];
            for (int j = 0; j < 4; ++j) pell[(size_t)j * g.V + r] = prow[ell[(size_t)j * g.V + u]] - u0;
        }
        for (int32_t u = u0; u < g.gv0[k + 1]; ++u)
            for (int64_t q = g.vptr[u]; q < g.vptr[u + 1]; ++q) padj[q] = prow[g.adj_o[q]] - u0;
    }
    up.add(g.d_prow, std::move(prow));
    up.add(g.d_pvtx, std::move(pvtx));
    up.add(g.d_pell, std::move(pell));
    up.add(g.d_padj, std::move(padj));
    up.add(g.d_gv0, g.gv0);
    up.add(g.d_ge0, g.ge0);
    up.add(g.d_segs, g.segs);
    up.add(g.d_tile0, g.tile0);
}

void finish_upload(grf_graph &g, Uploads &up, hipStream_t s) {
    up.flush(s);
    g.d_kap2.reserve(sizeof(double) * (g.E + 1));
    g.kap2_loaded = -1.0;
    GRF_HIP(hipStreamSynchronize(s));
}

void upload_mesh(grf_graph &g, hipStream_t s) {
    Uploads up;
    prepare_mesh(g, up);
    finish_upload(g, up, s);
}

Shifts make_shifts(double beta, double step, double h, const grf_opts &o) {
    GRF_REQUIRE(std::isfinite(beta) && beta > 0 && beta < 1, "beta must lie in (0, 1)");
    GRF_REQUIRE(std::isfinite(step) && step >= 0, "quad_step must be >= 0 (0 = paper rule)");
    Shifts sh;
    sh.k = (step == 0) ? -1.0 / (beta * std::log(h)) : step;
    GRF_REQUIRE(std::isfinite(sh.k) && sh.k > 0, "paper step rule needs h < 1; pass quad_step > 0");
    const double pi = 3.14159265358979323846;
    double km = std::ceil(pi * pi / (4.0 * sh.k * sh.k * beta));
    double kp = std::ceil(pi * pi / (4.0 * sh.k * sh.k * (1.0 - beta)));
    GRF_REQUIRE(km < 1e6 && kp < 1e6, "quadrature step too small: %g shifts", km + kp + 1);
    sh.kminus = o.k_minus >= 0 ? o.k_minus : (int32_t)km;
    sh.kplus = o.k_plus >= 0 ? o.k_plus : (int32_t)kp;
    GRF_REQUIRE((int64_t)sh.kminus + (int64_t)sh.kplus + 1 <= 1000000,
                "k_minus + k_plus + 1 = %lld shifts: at most 1e6", (long long)sh.kminus + sh.kplus + 1);
    double cconst = pi / (2.0 * sh.k * std::sin(pi * beta));
    for (int32_t l = -sh.kminus; l <= sh.kplus; ++l) {
        double y = (double)l * sh.k;
        double ci = cconst * std::exp(-2.0 * beta * y);
        double cl = ci * std::exp(2.0 * y);
        GRF_REQUIRE(std::isfinite(ci) && ci > 0 && std::isfinite(cl) && cl > 0,
                    "shift l = %d: c_I = %g, c_L = %g are not finite and positive (limits too wide for step %g)",
                    l, ci, cl, sh.k);
        sh.cI.push_back(ci);
        sh.cL.push_back(cl);
    }
    return sh;
}

grf_opts resolve_opts(const grf_opts *o) {
    grf_opts r;
    grf_opts_init(&r);
    if (o) r = *o;
    GRF_REQUIRE(std::isfinite(r.tol) && r.tol > 0, "tol must be > 0");
    GRF_REQUIRE(r.maxit >= 1, "maxit must be >= 1");
    GRF_REQUIRE(r.precision == GRF_PREC_FP64 || r.precision == GRF_PREC_MIXED, "unknown precision");
    GRF_REQUIRE(r.precond == GRF_PRECOND_JACOBI || r.precond == GRF_PRECOND_LEARNED || r.precond == GRF_PRECOND_NN,
                "unknown precond");
    GRF_REQUIRE(r.precond != GRF_PRECOND_LEARNED || r.learned, "learned preconditioner needs opts->learned");
    GRF_REQUIRE(r.sample_offset >= 0, "sample_offset must be >= 0");
    if (r.pcg_class_modes != 0) {
        GRF_REQUIRE(r.precond == GRF_PRECOND_LEARNED, "pcg_class_modes is for the learned preconditioner");
        GRF_REQUIRE((r.pcg_class_modes & ~(GRF_PCG_MODES_SET | 0xfff)) == 0 && (r.pcg_class_modes & GRF_PCG_MODES_SET),
                    "pcg_class_modes: GRF_PCG_MODES_SET | 2-bit variants of the 6 size classes");
        for (int c = 0; c < kPcgClasses; ++c)
            GRF_REQUIRE(chip_mode_valid(c, (r.pcg_class_modes >> (2 * c)) & 3),
                        "pcg_class_modes: variant %d is not available in size class %d", (r.pcg_class_modes >> (2 * c)) & 3, c);
    }
    GRF_REQUIRE(r.sweep_block == 0 || r.sweep_block == 8 || r.sweep_block == 16 || r.sweep_block == 32 ||
                    r.sweep_block == 64,
                "sweep_block must be 0, 8, 16, 32 or 64");
    GRF_REQUIRE(r.shift_block >= 0, "shift_block must be >= 0");
    return r;
}

}  // namespace grf

grf::MeshView grf_graph::view() const {
    grf::MeshView v;
    v.V = (int32_t)V;
    v.E = (int32_t)E;
    v.max_deg = max_deg;
    v.NI = NI;
    v.N = N;
    v.off = d_off.as<int64_t>();
    v.m = d_m.as<int32_t>();
    v.eu = d_eu.as<int32_t>();
    v.ev = d_ev.as<int32_t>();
    v.he = d_he.as<double>();
    v.kap2 = d_kap2.as<double>();
    v.vptr = d_vptr.as<int64_t>();
    v.adj_e = d_adj_e.as<int32_t>();
    v.adj_o = d_adj_o.as<int32_t>();
    v.adj_s = d_adj_s.as<int8_t>();
    v.msqrt = d_msqrt.as<double>();
    v.ng = (int32_t)gv0.size() - 1;
    v.consistent = (flags & GRF_MASS_CONSISTENT_SYS) ? 1 : 0;
    v.cnoise = (flags & GRF_NOISE_CONSISTENT) ? 1 : 0;
    v.gv0 = d_gv0.as<int32_t>();
    v.ge0 = d_ge0.as<int32_t>();
    v.segs = d_segs.as<int64_t>();
    v.maxVg = maxVg;
    v.maxEg = maxEg;
    v.maxNg = maxNg;
    v.tile0 = d_tile0.as<int64_t>();
    v.ntiles = tile0.empty() ? 0 : tile0.back();
    v.ell = d_ell.as<int32_t>();
    v.eend = d_eend.as<int32_t>();
    v.deg = d_deg.as<int32_t>();
    v.gord = d_gord.as<int32_t>();
    v.ell16 = d_ell16.as<uint2>();
    v.ovfm = d_ovfm.as<uint32_t>();
    v.ovent = d_ovent.as<int4>();
    v.ovent0 = d_ovent0.as<int32_t>();
    v.ovnp = d_ovnp.as<int32_t>();
    v.ovpc = d_ovpc.as<int2>();
    v.prow = d_prow.as<int32_t>();
    v.pvtx = d_pvtx.as<int32_t>();
    v.pell = d_pell.as<int32_t>();
    v.padj = d_padj.as<int32_t>();
    for (int c = 0; c <= grf::kPcgClasses + 1; ++c) v.cls_off[c] = cls_off[c];
    return v;
}

using namespace grf;

#define GRF_API_BEGIN try {
#define GRF_API_END                                     \
    }                                                   \
    catch (const ::grf::Error &err) { return err.code; } \
    catch (const std::bad_alloc &) {                    \
        ::grf::set_error("host allocation failed");      \
        return GRF_ENOMEM;                              \
    }                                                   \
    catch (...) {                                       \
        ::grf::set_error("unexpected internal error");   \
        return GRF_EDEVICE;                             \
    }                                                   \
    return GRF_OK;

extern "C" {

const char *grf_last_error(void) { return g_err; }

void grf_opts_init(grf_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-12;
    o->maxit = 10000;
    o->precision = GRF_PREC_FP64;
    o->precond = GRF_PRECOND_JACOBI;
    o->k_minus = -1;
    o->k_plus = -1;
    o->refine = -1;
}

int grf_graph_create(int64_t n_vertices, int64_t n_edges, const int64_t *edges, const double *lengths, double h,
                     uint32_t flags, grf_graph **out) {
    GRF_API_BEGIN
    GRF_REQUIRE(out, "out must be non-NULL");
    *out = nullptr;
    static std::atomic<uint64_t> next_serial{1};
    grf_graph *g = new grf_graph();
    g->serial = next_serial++;
    try {
        build_mesh(*g, n_vertices, n_edges, edges, lengths, h, flags);
        Uploads up;
        prepare_mesh(*g, up);  // every host step before the first HIP call
        GRF_HIP(hipGetDevice(&g->device));
        finish_upload(*g, up, nullptr);
    } catch (...) {
        delete g;
        throw;
    }
    *out = g;
    GRF_API_END
}

int grf_graph_info(const grf_graph *g, int64_t *n_dof, int64_t *n_interior, int64_t *dof_offsets) {
    GRF_API_BEGIN
    GRF_REQUIRE(g, "graph is NULL");
    if (n_dof) *n_dof = g->N;
    if (n_interior) *n_interior = g->NI;
    if (dof_offsets)
        for (int64_t e = 0; e <= g->E; ++e) dof_offsets[e] = g->off[e];
    GRF_API_END
}

int grf_graph_lumped_mass(const grf_graph *g, double *out) {
    GRF_API_BEGIN
    GRF_REQUIRE(g, "graph is NULL");
    GRF_REQUIRE(out || g->N == 0, "out is NULL");
    std::copy(g->ml.begin(), g->ml.end(), out);
    GRF_API_END
}

int grf_graph_destroy(grf_graph *g) {
    GRF_API_BEGIN
    if (g) {
        batch_forget(g->serial);
        free_work(*g);
        delete g;
    }
    GRF_API_END
}

int grf_shift_count(const grf_graph *g, double beta, double quad_step, const grf_opts *opts, int32_t *k_minus,
                    int32_t *k_plus, double *step_used) {
    GRF_API_BEGIN
    GRF_REQUIRE(g || quad_step > 0, "graph is NULL (it may be NULL only with quad_step > 0)");
    grf_opts o = resolve_opts(opts);
    Shifts sh = make_shifts(beta, quad_step, g ? g->h : 0.5, o);
    if (k_minus) *k_minus = sh.kminus;
    if (k_plus) *k_plus = sh.kplus;
    if (step_used) *step_used = sh.k;
    GRF_API_END
}

}  // extern "C"
