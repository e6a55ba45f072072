// Host-side helpers shared by the library's translation units: error
// reporting across the C ABI, device allocation owned by a context, and the
// per-kernel HIP-event profiler.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "phmg_internal.h"

namespace phmg {

// message of the last failed call on this thread (phmg_last_error)
inline thread_local std::string g_last_error;

struct Error : std::runtime_error {
    phmg_status code;
    Error(phmg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(phmg_status c, const std::string& m) { throw Error(c, m); }

inline void hipcheck(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(PHMG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
T* dalloc(phmg_ctx ctx, int64_t count) {
    if (count <= 0) count = 1;
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(T) * (size_t)count) != hipSuccess) {
        (void)hipGetLastError();
        fail(PHMG_ENOMEM, "hipMalloc of " + std::to_string(sizeof(T) * (size_t)count) + " bytes failed");
    }
    ctx->allocs.push_back(p);
    return static_cast<T*>(p);
}

inline void dfree(phmg_ctx ctx, void* p) {
    if (!p) return;
    auto it = std::find(ctx->allocs.begin(), ctx->allocs.end(), p);
    if (it != ctx->allocs.end()) ctx->allocs.erase(it);
    (void)hipFree(p);
}

template <typename T>
T* upload(phmg_ctx ctx, const T* h, int64_t count) {
    T* d = dalloc<T>(ctx, count);
    if (count > 0) hipcheck(hipMemcpy(d, h, sizeof(T) * (size_t)count, hipMemcpyHostToDevice), "hipMemcpy H2D");
    return d;
}

inline std::string lvl(int l) { return "level " + std::to_string(l) + ": "; }

// Exceptions never cross the C ABI: every entry point runs its body here.
template <typename F>
phmg_status guarded(F&& f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return PHMG_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return PHMG_EINVAL;
    }
}

// RAII pair of HIP events around the launches of one kernel class on one
// level, recorded only when that class is enabled in the profile mask.
struct Timed {
    phmg_ctx ctx;
    int id, level;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEvent_t take() {
        auto& pool = ctx->prof.pool;
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        hipcheck(hipEventCreate(&e), "hipEventCreate");
        return e;
    }
    hipStream_t stream;
    Timed(phmg_ctx c, int k, int l, hipStream_t s = nullptr) : ctx(c), id(k), level(l), stream(s ? s : c->stream) {
        if (!(ctx->prof.mask & (1u << k))) return;
        e0 = take();
        e1 = take();
        hipcheck(hipEventRecord(e0, stream), "hipEventRecord");
    }
    ~Timed() {
        if (!e0) return;
        (void)hipEventRecord(e1, stream);
        ctx->prof.pending.push_back({id, level, e0, e1});
    }
};

inline void require_ready(phmg_ctx ctx) {
    for (size_t l = 0; l < ctx->L.size(); ++l)
        if (!ctx->L[l].ready) fail(PHMG_ESTATE, lvl((int)l) + "relax_setup has not been run");
}

inline void drain_profile(phmg_ctx ctx) {
    if (ctx->prof.pending.empty()) return;
    hipcheck(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    for (auto& it : ctx->prof.pending) {
        float ms = 0.f;
        hipcheck(hipEventElapsedTime(&ms, it.e0, it.e1), "hipEventElapsedTime");
        const int l = std::min(std::max(it.level, 0), PHMG_MAX_LEVELS - 1);
        ctx->prof.ms[it.kernel][l] += ms;
        ctx->prof.count[it.kernel][l] += 1;
        ctx->prof.pool.push_back(it.e0);
        ctx->prof.pool.push_back(it.e1);
    }
    ctx->prof.pending.clear();
}

}  // namespace phmg
