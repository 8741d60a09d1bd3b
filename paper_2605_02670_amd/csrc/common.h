// Internal declarations shared by the libgrf translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>
#include <memory>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/grf.h"

namespace grf {

constexpr int kWave = 64;  // CDNA wavefront width; samples are laid out in blocks of 64

// ---- error handling -------------------------------------------------------
void set_error(const char *fmt, ...);

struct Error {
    int code;
};

#define GRF_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ::grf::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),      \
                             __FILE__, __LINE__);                                        \
            throw ::grf::Error{e_ == hipErrorOutOfMemory ? GRF_ENOMEM : GRF_EDEVICE};    \
        }                                                                                \
    } while (0)

#define GRF_REQUIRE(cond, ...)               \
    do {                                     \
        if (!(cond)) {                       \
            ::grf::set_error(__VA_ARGS__);   \
            throw ::grf::Error{GRF_EINVAL};  \
        }                                    \
    } while (0)

#define GRF_LAUNCH_CHECK() GRF_HIP(hipGetLastError())

// ---- device buffers ---------------------------------------------------------
// Memory a caller lends for the duration of one call: while an Arena is
// installed on the calling thread (ArenaScope), DevBuf::reserve carves
// 256-byte aligned ranges from it instead of calling hipMalloc, and throws
// GRF_EINVAL when the arena is exhausted.
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0;
    const char *owner = "";  // named in the error when the arena is exhausted
};
Arena *current_arena();
struct ArenaScope {
    Arena *prev;
    explicit ArenaScope(Arena *a);
    ~ArenaScope();
    ArenaScope(const ArenaScope &) = delete;
    ArenaScope &operator=(const ArenaScope &) = delete;
};

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    bool borrowed = false;  // carved from an Arena: never freed here
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    void reserve(size_t n);  // grow-only; contents are not preserved
    void release();
    template <class T>
    T *as() const { return static_cast<T *>(ptr); }
};

template <class T>
void upload(DevBuf &b, const std::vector<T> &v, hipStream_t s) {
    b.reserve(v.size() * sizeof(T) + 16);
    if (!v.empty()) GRF_HIP(hipMemcpyAsync(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// ---- mesh as seen by kernels (plain device pointers, passed by value) ------
// vertex capacity of the on-chip PCG size classes (a graph goes to the first
// class that holds it)
constexpr int kPcgClasses = 6;
constexpr int32_t kPcgCap[kPcgClasses] = {64, 256, 1024, 4096, 10176, 20352};
// launch shape of each class: TPB threads, K vertices per thread (TPB K >= cap),
// thread t owning the graph-local vertices t + TPB i
constexpr int kChipTpb[kPcgClasses] = {64, 64, 128, 512, 1024, 1024};
constexpr int kChipK[kPcgClasses] = {1, 4, 8, 8, 10, 20};

struct MeshView {
    int32_t V, E;
    int32_t max_deg;      // largest vertex degree (edge ends)
    int64_t NI, N;        // interior DOFs, all DOFs
    const int64_t *off;   // [E+1] first interior DOF of each edge
    const int32_t *m;     // [E] interior DOF count
    const int32_t *eu;    // [E] tail vertex
    const int32_t *ev;    // [E] head vertex
    const double *he;     // [E] local mesh size
    const double *kap2;   // [E] kappa^2 of the edge's graph (per call)
    const int64_t *vptr;  // [V+1] CSR over edge ends
    const int32_t *adj_e; // [2E] edge of the end
    const int32_t *adj_o; // [2E] vertex at the other end
    const int8_t *adj_s;  // [2E] 0 = tail end (u_e), 1 = head end (v_e)
    const double *msqrt;  // [N] sqrt of the lumped mass diagonal
    // graphs of a batch (one graph: ng = 1): vertices gv0[g] .. gv0[g+1]-1 and edges
    // ge0[g] .. ge0[g+1]-1; segs[4g..4g+3] = (local DOFs, local interior DOFs, first
    // interior row, first vertex row) of graph g in this mesh's DOF order
    int32_t ng;
    const int32_t *gv0, *ge0;
    const int64_t *segs;
    int32_t maxVg, maxEg;  // largest graph of the batch (host-side dispatch)
    int32_t consistent;    // shifted systems with the consistent mass matrix (GRF_MASS_CONSISTENT_SYS)
    int32_t cnoise;        // consistent-mass noise (GRF_NOISE_CONSISTENT)
    int64_t maxNg;
    // 64-DOF tiles of the batch's graphs: graph g's tiles are tile0[g] .. tile0[g+1]-1
    const int64_t *tile0;  // [ng+1]
    int64_t ntiles;
    // first four edge ends of every vertex (column-major [4][V]: the other vertex, or the
    // vertex itself past its degree; eend: 2 edge + side, or -1 past the degree) and the degree
    const int32_t *ell, *eend, *deg;
    // graphs ordered by PCG size class (kPcgCap), largest first within a class:
    // class c is gord[cls_off[c] .. cls_off[c+1]-1]; class kPcgClasses holds the
    // graphs too large for every on-chip class
    const int32_t *gord;
    int32_t cls_off[kPcgClasses + 2];
    // graph-local ids of the first four edge ends of every vertex ([V], 16 bits
    // each, the vertex itself past its degree; graphs of an on-chip class only)
    const uint2 *ell16;
    // per graph and wavefront of its class shape: bit i set if item i of some
    // lane of the wavefront has degree > 4 ([ng][16])
    const uint32_t *ovfm;
    // vertex PCG row order: the graphs beyond every on-chip class keep their operator
    // rows (dh, coef, diag of S^, P^, Q^) in a Cuthill-McKee order of their vertices,
    // every other graph in vertex order.  prow[u]: row of vertex u; pvtx[r]: vertex of
    // row r; pell[j][r] ([4][V]): graph-local row of the j-th ELL neighbour of row r's
    // vertex (its own past the degree); padj[k] ([2E]): graph-local row of adj_o[k]
    const int32_t *prow, *pvtx, *pell, *padj;
    // edge-end slots past the first four (degree > 4) of the graphs of an on-chip class,
    // for products that spread them over a whole workgroup: each such vertex's slots are
    // cut into pieces of at most 64, the pieces packed into chunks of 64 entries (a piece
    // never crosses a chunk; unused entries have piece -1).  Graph g's entries are
    // ovent[ovent0[g] .. ovent0[g+1]-1], (CSR slot k, graph-local piece, graph-local row
    // of the vertex, graph-local neighbour), its pieces number ovnp[g]; ovpc[u] = (first
    // piece, end) of vertex u, (0, 0) for a vertex of degree <= 4.
    const int4 *ovent;
    const int32_t *ovent0, *ovnp;
    const int2 *ovpc;
};

}  // namespace grf

// ---- the opaque handle ---------------------------------------------------------
struct grf_graph {
    int device = 0;
    uint64_t serial = 0;  // unique per created handle (batch cache key)
    int64_t V = 0, E = 0, NI = 0, N = 0;
    double h = 0;
    uint32_t flags = 0;
    std::vector<int64_t> eu, ev, off;
    std::vector<int32_t> m;
    std::vector<double> len, he, ml;
    std::vector<int64_t> vptr;
    std::vector<int32_t> adj_e, adj_o;
    std::vector<int8_t> adj_s;
    // device copies
    grf::DevBuf d_off, d_m, d_eu, d_ev, d_he, d_kap2, d_vptr, d_adj_e, d_adj_o, d_adj_s, d_msqrt;
    // graphs of a batch (a single graph is a batch of one)
    std::vector<int32_t> gv0, ge0;
    std::vector<int64_t> segs;
    int32_t max_deg = 0, maxVg = 0, maxEg = 0;
    int64_t maxNg = 0;
    std::vector<int64_t> tile0;  // [ng+1] first 64-DOF tile of every graph
    grf::DevBuf d_gv0, d_ge0, d_segs, d_ell, d_eend, d_deg, d_tile0;
    std::vector<int32_t> gord;
    int32_t cls_off[grf::kPcgClasses + 2] = {};
    grf::DevBuf d_gord, d_ell16, d_ovfm, d_prow, d_pvtx, d_pell, d_padj;
    grf::DevBuf d_ovent, d_ovent0, d_ovnp, d_ovpc;
    double kap2_loaded = -1.0;
    // workspace, grown on demand
    struct Work;
    Work *work = nullptr;
    grf::MeshView view() const;
};

namespace grf {

// host-side mesh construction shared by single and batched graphs
void build_mesh(grf_graph &g, int64_t V, int64_t E, const int64_t *edges, const double *lengths, double h,
                uint32_t flags);
// Host arrays bound for device buffers, copied by flush(): a mesh is prepared
// completely on the host before its first HIP call.
struct Uploads {
    struct Item {
        DevBuf *b;
        std::shared_ptr<const void> hold;  // keeps the host array alive until the copy is done
        const void *data;
        size_t bytes;
    };
    std::vector<Item> items;
    template <class T>
    void add(DevBuf &b, std::vector<T> v) {  // by value: callers move arrays they no longer need
        auto h = std::make_shared<std::vector<T>>(std::move(v));
        items.push_back(Item{&b, h, h->data(), h->size() * sizeof(T)});
    }
    void flush(hipStream_t s) {
        for (Item &it : items) {
            it.b->reserve(it.bytes + 16);
            if (it.bytes) GRF_HIP(hipMemcpyAsync(it.b->ptr, it.data, it.bytes, hipMemcpyHostToDevice, s));
        }
    }
};
void prepare_mesh(grf_graph &g, Uploads &up);                 // host: every derived array of the mesh
void finish_upload(grf_graph &g, Uploads &up, hipStream_t s); // device: the copies, then a sync
void upload_mesh(grf_graph &g, hipStream_t s);                // both

// quadrature schedule (host, FP64)
struct Shifts {
    double k = 0;
    int32_t kminus = 0, kplus = 0;
    std::vector<double> cI, cL;
};
Shifts make_shifts(double beta, double step, double h, const grf_opts &o);

grf_opts resolve_opts(const grf_opts *o);

// drops cached batches that contain the graph with this serial (batch.hip)
void batch_forget(uint64_t serial);

// Optional per-kernel timing with HIP events on the launch stream.
struct KTimer {
    struct Rec {
        int id;
        hipEvent_t a, b;
    };
    bool on = false;
    hipStream_t st = nullptr;
    std::vector<Rec> recs;
    KTimer(bool enabled, hipStream_t s) : on(enabled), st(s) {}
    KTimer(const KTimer &) = delete;
    ~KTimer();
    void begin(int id);
    void end();
    // after the stream is synchronised: add elapsed times to stats
    void collect(grf_stats *stats);
};

}  // namespace grf
