// Entry point grf_sample_noalloc: grf_sample for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// Every workspace buffer of the call (noise and accumulator in the sample
// layout, per-shift coefficients, block operand tables, vertex systems, PCG
// vectors and operators, iteration counts) is carved from `scratch`, a
// file-scope device array of kScratchBytes, instead of being allocated.  The
// loader places one copy of the array on every device the library runs on and
// keeps it until the process ends.  Its address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current; the
// kernels receive that address like any other buffer.  Every call on a device
// shares its copy and finds the previous call's contents there: the path
// clears what it needs itself (the accumulator rows, every written output), and
// two calls that overlap on one device race on it.
#include <algorithm>
#include <mutex>

#include "work.h"

namespace grf {
namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;  // 128 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scr_mu;
void *g_scr_ptr[kMaxDevices] = {};

// device address of this device's copy of scratch (the host-side name is only a stand-in)
void *scratch_address(int dev) {
    GRF_REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d beyond the %d devices the scratch table holds", dev,
                kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scr_mu);
    if (!g_scr_ptr[dev]) {
        void *p = nullptr;
        GRF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        GRF_REQUIRE(p != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
        g_scr_ptr[dev] = p;
    }
    return g_scr_ptr[dev];
}

// Swaps a graph's workspace for a call-local one and restores it on every exit path.
struct WorkSwap {
    grf_graph &g;
    grf_graph::Work *saved;
    grf_graph::Work local;
    explicit WorkSwap(grf_graph &gr) : g(gr), saved(gr.work) { g.work = &local; }
    ~WorkSwap() { g.work = saved; }
};

}  // namespace
}  // namespace grf

using namespace grf;

extern "C" {

int grf_sample_noalloc(grf_graph *g, double kappa, double beta, double quad_step, int64_t n_samples,
                       uint64_t seed, double *out, const grf_opts *opts) {
    try {
        GRF_REQUIRE(g, "graph is NULL");
        grf_opts o = resolve_opts(opts);
        GRF_REQUIRE(o.precond != GRF_PRECOND_LEARNED,
                    "grf_sample_noalloc: the learned preconditioner keeps its own workspace; use Jacobi or NN");
        o.timing = 0;  // per-kernel events would be created in the call
        int dev = -1;
        GRF_HIP(hipGetDevice(&dev));
        GRF_REQUIRE(dev == g->device, "grf_sample_noalloc: device %d is current, the graph lives on device %d", dev,
                    g->device);
        Arena arena;
        arena.base = static_cast<char *>(scratch_address(dev));
        arena.size = kScratchBytes;
        arena.owner = "grf_sample_noalloc";
        WorkSwap ws(*g);
        ArenaScope scope(&arena);
        return sample_impl(g, kappa, beta, quad_step, n_samples, seed, nullptr, out, &o);
    } catch (const ::grf::Error &err) {
        return err.code;
    } catch (const std::bad_alloc &) {
        ::grf::set_error("host allocation failed");
        return GRF_ENOMEM;
    } catch (...) {
        ::grf::set_error("unexpected internal error");
        return GRF_EDEVICE;
    }
}

}  // extern "C"
