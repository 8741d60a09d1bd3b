// Drives the host code of libgrf through the C ABI, for a build whose host
// side carries AddressSanitizer (device code is not part of that build).
// Every call here runs its host steps before its first HIP call: mesh
// construction and preparation (edge meshing, adjacency, size classes,
// overflow pieces, reverse Cuthill-McKee order, tiles), argument validation,
// the quadrature schedule and the network's parameter checks.  Without a GPU
// the valid graphs end in GRF_EDEVICE after all of that; with one they are
// created, queried and destroyed.  Prints one line per case and exits 1 if a
// status is not the expected one (AddressSanitizer aborts on its own).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "grf.h"

static int g_fail = 0;

struct GraphCase {
    const char *name;
    int64_t V;
    std::vector<int64_t> edges;  // [E][2]
    std::vector<double> lengths;
    double h;
    uint32_t flags;
    bool valid;
};

static void add_edge(GraphCase &c, int64_t u, int64_t v, double L) {
    c.edges.push_back(u);
    c.edges.push_back(v);
    c.lengths.push_back(L);
}

static GraphCase lattice(const char *name, int n, double h, uint32_t seed) {
    GraphCase c{name, (int64_t)n * n, {}, {}, h, 0u, true};
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> len(0.02, 1.5);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int64_t u = (int64_t)i * n + j;
            if (j + 1 < n) add_edge(c, u, u + 1, len(rng));
            if (i + 1 < n) add_edge(c, u, u + n, len(rng));
        }
    return c;
}

static void run_graph(const GraphCase &c) {
    grf_graph *g = nullptr;
    const int64_t E = (int64_t)c.lengths.size();
    const int rc = grf_graph_create(c.V, E, c.edges.empty() ? nullptr : c.edges.data(),
                                    c.lengths.empty() ? nullptr : c.lengths.data(), c.h, c.flags, &g);
    const char *msg = grf_last_error();
    bool ok;
    if (c.valid) {
        ok = rc == GRF_OK || rc == GRF_EDEVICE;
        if (rc == GRF_OK) {
            int64_t n_dof = 0, n_int = 0;
            std::vector<int64_t> off(E + 1);
            ok = ok && grf_graph_info(g, &n_dof, &n_int, off.data()) == GRF_OK && off[E] == n_int;
            std::vector<double> ml(n_dof);
            ok = ok && grf_graph_lumped_mass(g, ml.data()) == GRF_OK;
            int32_t km = 0, kp = 0;
            double step = 0;
            grf_opts o;
            grf_opts_init(&o);
            ok = ok && grf_shift_count(g, 0.6, 0.0, &o, &km, &kp, &step) == GRF_OK;
            ok = ok && grf_graph_destroy(g) == GRF_OK;
        } else {
            ok = ok && g == nullptr && msg && std::strlen(msg) > 0;
        }
    } else {
        ok = rc == GRF_EINVAL && g == nullptr && msg && std::strlen(msg) > 0;
    }
    std::printf("graph %-26s V=%-7lld E=%-7lld rc=%d %s\n", c.name, (long long)c.V, (long long)E, rc,
                ok ? "ok" : "UNEXPECTED");
    if (!ok) g_fail = 1;
}

int main() {
    grf_opts o;
    grf_opts_init(&o);
    std::vector<GraphCase> cases;
    {  // edges of 0, 1, 2, ... interior points, a multi-edge, a self-loop, a pendant vertex
        GraphCase c{"ragged", 13, {}, {}, 0.07, GRF_MESH_ROUND, true};
        const double L[] = {0.013, 0.05, 0.09, 0.16, 0.31, 0.9, 1.7, 0.44, 0.21, 0.6, 1.1, 0.07};
        for (int i = 0; i < 12; ++i) add_edge(c, i, (i + 1) % 12, L[i]);
        add_edge(c, 0, 1, 0.5);
        add_edge(c, 5, 5, 0.9);
        add_edge(c, 3, 12, 0.31);
        cases.push_back(c);
        c.name = "ragged-ceil-consistent";
        c.flags = GRF_MESH_CEIL | GRF_MASS_CONSISTENT_SYS;
        cases.push_back(c);
        c.name = "ragged-consistent-noise";
        c.flags = GRF_MESH_ROUND | GRF_MASS_CONSISTENT_SYS | GRF_NOISE_CONSISTENT;
        cases.push_back(c);
    }
    cases.push_back(lattice("lattice-30", 30, 0.05, 1));
    {  // a hub of degree 3000 (overflow pieces), on-chip size class
        GraphCase c{"hub-3000", 3001, {}, {}, 0.1, 0u, true};
        for (int i = 1; i <= 3000; ++i) {
            add_edge(c, 0, i, 0.3 + 0.001 * i);
            add_edge(c, i, i % 3000 + 1, 0.2);
        }
        cases.push_back(c);
    }
    {  // beyond every on-chip class (reverse Cuthill-McKee order), with two hubs
        GraphCase c = lattice("lattice-150-hubs", 150, 0.2, 2);
        for (int i = 0; i < 400; ++i) {
            add_edge(c, 7, 53 * i + 11, 0.4);
            add_edge(c, 22000, 37 * i + 5, 0.7);
        }
        cases.push_back(c);
    }
    {  // two components, long edges
        GraphCase c{"two-triangles-long", 6, {}, {}, 0.05, 0u, true};
        add_edge(c, 0, 1, 50.0);
        add_edge(c, 1, 2, 0.01);
        add_edge(c, 2, 0, 7.3);
        add_edge(c, 3, 4, 1.0);
        add_edge(c, 4, 5, 12.0);
        add_edge(c, 5, 3, 0.2);
        cases.push_back(c);
    }
    {
        GraphCase c{"isolated-vertex", 3, {}, {}, 0.1, 0u, false};
        add_edge(c, 0, 1, 1.0);
        cases.push_back(c);
        GraphCase d{"endpoint-out-of-range", 2, {}, {}, 0.1, 0u, false};
        add_edge(d, 0, 2, 1.0);
        cases.push_back(d);
        GraphCase e{"negative-endpoint", 2, {}, {}, 0.1, 0u, false};
        add_edge(e, -1, 1, 1.0);
        cases.push_back(e);
        GraphCase f{"nan-length", 2, {}, {}, 0.1, 0u, false};
        add_edge(f, 0, 1, std::nan(""));
        cases.push_back(f);
        GraphCase z{"zero-length", 2, {}, {}, 0.1, 0u, false};
        add_edge(z, 0, 1, 0.0);
        cases.push_back(z);
        GraphCase hz{"h-zero", 2, {}, {}, 0.0, 0u, false};
        add_edge(hz, 0, 1, 1.0);
        cases.push_back(hz);
        GraphCase hn{"h-nan", 2, {}, {}, std::nan(""), 0u, false};
        add_edge(hn, 0, 1, 1.0);
        cases.push_back(hn);
        GraphCase fl{"unknown-flag", 2, {}, {}, 0.1, 0x80u, false};
        add_edge(fl, 0, 1, 1.0);
        cases.push_back(fl);
        GraphCase nv{"no-vertices", 0, {}, {}, 0.1, 0u, false};
        cases.push_back(nv);
    }
    for (const GraphCase &c : cases) run_graph(c);

    // quadrature schedule without a graph (quad_step > 0)
    struct Q {
        double beta, step;
        int expect;
    } qs[] = {{0.6, 0.35, GRF_OK}, {0.85, 0.2, GRF_OK}, {0.1, 1.0, GRF_OK}, {1.0, 0.3, GRF_EINVAL},
              {0.0, 0.3, GRF_EINVAL}, {0.5, -1.0, GRF_EINVAL}, {0.5, 0.0, GRF_EINVAL}, {std::nan(""), 0.3, GRF_EINVAL}};
    for (const Q &q : qs) {
        int32_t km = -7, kp = -7;
        double used = 0;
        const int rc = grf_shift_count(nullptr, q.beta, q.step, &o, &km, &kp, &used);
        const bool ok = rc == q.expect && (rc != GRF_OK || (km >= 0 && kp >= 0 && used == q.step));
        std::printf("shift_count beta=%g step=%g rc=%d K-=%d K+=%d %s\n", q.beta, q.step, rc, km, kp,
                    ok ? "ok" : "UNEXPECTED");
        if (!ok) g_fail = 1;
    }
    {  // explicit limits, too many shifts
        grf_opts w = o;
        w.k_minus = 600000;
        w.k_plus = 600000;
        int32_t km = 0, kp = 0;
        double used = 0;
        const int rc = grf_shift_count(nullptr, 0.5, 0.3, &w, &km, &kp, &used);
        std::printf("shift_count too-many rc=%d %s\n", rc, rc == GRF_EINVAL ? "ok" : "UNEXPECTED");
        if (rc != GRF_EINVAL) g_fail = 1;
    }

    // the network's parameter checks
    int64_t np = 0;
    if (grf_learned_param_count(&np) != GRF_OK || np <= 0) g_fail = 1;
    std::vector<float> p((size_t)np, 0.01f);
    grf_learned *net = nullptr;
    int rc = grf_learned_create(p.data(), np - 1, &net);
    std::printf("learned_create short rc=%d %s\n", rc, rc == GRF_EINVAL && !net ? "ok" : "UNEXPECTED");
    if (rc != GRF_EINVAL || net) g_fail = 1;
    p[(size_t)np / 2] = INFINITY;
    rc = grf_learned_create(p.data(), np, &net);
    std::printf("learned_create inf rc=%d %s\n", rc, rc == GRF_EINVAL && !net ? "ok" : "UNEXPECTED");
    if (rc != GRF_EINVAL || net) g_fail = 1;

    // NULL handles
    const int nulls[] = {grf_graph_info(nullptr, nullptr, nullptr, nullptr),
                         grf_sample(nullptr, 1.0, 0.5, 0.3, 1, 0, nullptr, nullptr),
                         grf_noise(nullptr, 1, 0, nullptr, nullptr),
                         grf_solve_shifted(nullptr, 1.0, 1.0, 1.0, 1, nullptr, nullptr, nullptr),
                         grf_sample_batched(nullptr, 0, nullptr, 0.5, 0.3, 1, 0, nullptr, nullptr)};
    for (int r : nulls)
        if (r != GRF_EINVAL) g_fail = 1;
    std::printf("null handles %s\n", g_fail ? "UNEXPECTED" : "ok");
    std::printf("%s\n", g_fail ? "FAILED" : "PASSED");
    return g_fail;
}
