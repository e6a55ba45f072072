// Allocation-free relaxation sweeps (phmg_relax_apply_noalloc), for callers
// that cannot allocate device memory while they run: code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc.
//
// The sweep of eq. "eq:ASM" needs three work buffers besides the caller's b
// and x: the residual r (n doubles), the Chebyshev direction d (n) and the
// staged patch results Y (sum of the patch sizes).  phmg_relax_apply takes
// them from the context; this variant takes them from one file-scope device
// array of kScratchDoubles doubles (32 MiB), which every GPU the library runs
// on holds until the process ends.  Its device address differs per GPU and
// is resolved once per device with hipGetSymbolAddress, with that device
// current, when a hierarchy is created there (host code never passes the
// array's name to a kernel: on the host that name is not a device address).
//
// Every call on one GPU shares that GPU's array and leaves its last contents
// behind.  No buffer needs to start at zero (each is written before it is
// read inside the call), but calls that overlap in time on one GPU -- on two
// streams, or from two threads -- race on the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "host_util.h"
#include "phmg_internal.h"

namespace {

constexpr int64_t kScratchDoubles = PHMG_NOALLOC_MAX_DOUBLES;   // 32 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mutex;
double* g_scratch[kMaxDevices] = {};                    // device address of `scratch` per device

// offsets of r, d and Y inside the array, each aligned to 256 bytes
int64_t align32(int64_t n) { return (n + 31) / 32 * 32; }

}  // namespace

void phmg::noalloc_init_current_device() {
    int dev = 0;
    hipcheck(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) fail(PHMG_EINVAL, "device id " + std::to_string(dev) + " out of range");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_scratch[dev]) return;
    void* p = nullptr;
    hipcheck(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) fail(PHMG_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch[dev] = static_cast<double*>(p);
}

extern "C" {

phmg_status phmg_relax_apply_noalloc(phmg_ctx ctx, int level, const double* b, double* x, int nu) {
    using namespace phmg;
    return guarded([&]() -> phmg_status {
        if (!ctx || !b || !x) fail(PHMG_EINVAL, "null argument");
        if (level < 0 || level >= (int)ctx->L.size() - 1)
            fail(PHMG_EINVAL, "level out of range (coarsest has no patches)");
        if (nu < 0) fail(PHMG_EINVAL, "nu < 0");
        const Level& L = ctx->L[level];
        const int64_t need = 2 * align32(L.n) + align32(L.sum_m);
        if (need > kScratchDoubles)
            fail(PHMG_EINVAL, lvl(level) + "needs " + std::to_string(need) +
                                  " doubles of work space (2 n + sum m), more than the " +
                                  std::to_string(kScratchDoubles) + " of the allocation-free array");
        if (!L.ready) fail(PHMG_ESTATE, lvl(level) + "relax_setup has not been run");
        double* base = nullptr;
        {
            std::lock_guard<std::mutex> lock(g_mutex);
            if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch[ctx->device];
        }
        if (!base) fail(PHMG_ESTATE, "the allocation-free array was not resolved on this context's device");
        double* r = base;
        double* d = base + align32(L.n);
        double* Y = base + 2 * align32(L.n);
        relax_level(ctx, level, b, x, nu, false, false, r, d, Y, false);
        hipcheck(hipGetLastError(), "kernel launch");
        return PHMG_OK;
    });
}

}  // extern "C"
