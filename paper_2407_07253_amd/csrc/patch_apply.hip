// gfx950 batched patch solve of the additive Schwarz sweep (Section 3.4,
// eq. "eq:ASM"): y_i = K_i^{-1} r[S_i] for every Vanka-star patch, streaming the
// explicit patch inverses stored by the set-up.  This is the dominant kernel of
// the solve phase (HBM-bound: every factor word is read once per sweep).
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "phmg_internal.h"

namespace phmg {
namespace {

// ---------------------------------------------------------------------------
// Batched patch solve: y_i = K_i^{-1} r[S_i].  One workgroup per patch; the
// gathered residual sits in LDS.  Each wavefront streams the columns j = w,
// w+4, w+8, ... of the stored inverse (column-major, leading dimension ld =
// m rounded up to V), every lane owning V consecutive rows of up to NRT row
// tiles, so a wave-load is always 64 x 8 bytes and four columns are in flight
// per wave.  The four per-wave partial sums are combined in LDS once per
// group of NRT row tiles.
// ---------------------------------------------------------------------------
template <typename T, int V>
struct FactorLoad;
template <>
struct FactorLoad<double, 1> {
    __device__ static inline void load(const double* p, double (&a)[1]) { a[0] = *p; }
};
template <>
struct FactorLoad<float, 2> {
    __device__ static inline void load(const float* p, float (&a)[2]) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        a[0] = v.x;
        a[1] = v.y;
    }
};
template <>
struct FactorLoad<__hip_bfloat16, 4> {
    __device__ static inline void load(const __hip_bfloat16* p, float (&a)[4]) {
        const uint2 v = *reinterpret_cast<const uint2*>(p);
        a[0] = __uint_as_float(v.x << 16);
        a[1] = __uint_as_float(v.x & 0xffff0000u);
        a[2] = __uint_as_float(v.y << 16);
        a[3] = __uint_as_float(v.y & 0xffff0000u);
    }
};

// Stream one patch: Y[i] = sum_j B[i, j] s_r[j] for the patch's m rows (the
// gathered right-hand side s_r in LDS, B column-major with leading dimension ld).
template <typename T, typename Acc, int V, int NRT, int U>
__device__ inline void stream_patch(const T* __restrict__ A, int m, int ld, const Acc* s_r,
                                    Acc (&s_red)[NRT][kBlock / kWave][kWave * V], double* __restrict__ Yp) {
    constexpr int NW = kBlock / kWave;
    constexpr int TILE = kWave * V;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int r0 = 0; r0 < m; r0 += NRT * TILE) {
        Acc acc[NRT][V];
#pragma unroll
        for (int q = 0; q < NRT; ++q)
#pragma unroll
            for (int v = 0; v < V; ++v) acc[q][v] = 0;
        int j = wave;
        for (; j + (U - 1) * NW < m; j += U * NW) {
            Acc a[U][NRT][V];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const T* col = A + (int64_t)(j + u * NW) * ld + r0 + lane * V;
#pragma unroll
                for (int q = 0; q < NRT; ++q) {
                    if (r0 + q * TILE + lane * V < m) FactorLoad<T, V>::load(col + q * TILE, a[u][q]);
                    else
#pragma unroll
                        for (int v = 0; v < V; ++v) a[u][q][v] = 0;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const Acc rj = s_r[j + u * NW];
#pragma unroll
                for (int q = 0; q < NRT; ++q)
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[q][v] += a[u][q][v] * rj;
            }
        }
        for (; j < m; j += NW) {
            const T* col = A + (int64_t)j * ld + r0 + lane * V;
            const Acc rj = s_r[j];
#pragma unroll
            for (int q = 0; q < NRT; ++q) {
                if (r0 + q * TILE + lane * V < m) {
                    Acc a[V];
                    FactorLoad<T, V>::load(col + q * TILE, a);
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[q][v] += a[v] * rj;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NRT; ++q)
#pragma unroll
            for (int v = 0; v < V; ++v) s_red[q][wave][lane * V + v] = acc[q][v];
        __syncthreads();
        for (int t = threadIdx.x; t < NRT * TILE; t += kBlock) {
            const int i = r0 + t;
            if (i < m) {
                const int q = t / TILE, e = t % TILE;
                Yp[i] = (double)((s_red[q][0][e] + s_red[q][1][e]) + (s_red[q][2][e] + s_red[q][3][e]));
            }
        }
        __syncthreads();
    }
}

// One workgroup per patch.
template <typename T, typename Acc, int V, int NRT, int U>
__global__ __launch_bounds__(kBlock) void patch_apply_kernel(const int32_t* __restrict__ order,
                                                             const int64_t* __restrict__ pptr,
                                                             const int32_t* __restrict__ pdofs,
                                                             const int64_t* __restrict__ foff,
                                                             const T* __restrict__ F, const double* __restrict__ r,
                                                             double* __restrict__ Y) {
    extern __shared__ double s_buf[];
    Acc* s_r = reinterpret_cast<Acc*>(s_buf);
    __shared__ Acc s_red[NRT][kBlock / kWave][kWave * V];
    const int p = order[blockIdx.x];
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    const int ld = (m + V - 1) / V * V;
    for (int t = threadIdx.x; t < m; t += kBlock) s_r[t] = (Acc)r[pdofs[base + t]];
    __syncthreads();
    stream_patch<T, Acc, V, NRT, U>(F + foff[p], m, ld, s_r, s_red, Y + base);
}

// Persistent form: a grid sized to the resident workgroups; workgroup b takes
// the patches order[b], order[b + G], ... (largest first, so every workgroup
// gets a similar mix of sizes).  The gather of the next patch's right-hand
// side is issued into registers before the current patch is streamed (its
// latency hides behind the stream) and lands in the second LDS buffer.
template <typename T, typename Acc, int V, int NRT, int U, int R>
__global__ __launch_bounds__(kBlock) void patch_apply_persist_kernel(int npatch, const int32_t* __restrict__ order,
                                                                     const int64_t* __restrict__ pptr,
                                                                     const int32_t* __restrict__ pdofs,
                                                                     const int64_t* __restrict__ foff,
                                                                     const T* __restrict__ F,
                                                                     const double* __restrict__ r,
                                                                     double* __restrict__ Y, int ldbuf) {
    extern __shared__ double s_buf[];
    Acc* s_buf0 = reinterpret_cast<Acc*>(s_buf);
    Acc* s_buf1 = s_buf0 + ldbuf;
    __shared__ Acc s_red[NRT][kBlock / kWave][kWave * V];
    int idx = blockIdx.x;
    if (idx >= npatch) return;
    int p = order[idx];
    int64_t base = pptr[p];
    int m = (int)(pptr[p + 1] - base);
    for (int t = threadIdx.x; t < m; t += kBlock) s_buf0[t] = (Acc)r[pdofs[base + t]];
    __syncthreads();
    int cur = 0;
    for (;;) {
        const int nidx = idx + (int)gridDim.x;
        int pn = -1, mn = 0;
        int64_t basen = 0;
        Acc pre[R];
        if (nidx < npatch) {
            pn = order[nidx];
            basen = pptr[pn];
            mn = (int)(pptr[pn + 1] - basen);
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int t = threadIdx.x + u * kBlock;
                pre[u] = t < mn ? (Acc)r[pdofs[basen + t]] : (Acc)0;
            }
        }
        const int ld = (m + V - 1) / V * V;
        stream_patch<T, Acc, V, NRT, U>(F + foff[p], m, ld, cur ? s_buf1 : s_buf0, s_red, Y + base);
        if (pn < 0) break;
        Acc* s_next = cur ? s_buf0 : s_buf1;
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int t = threadIdx.x + u * kBlock;
            if (t < mn) s_next[t] = pre[u];
        }
        __syncthreads();
        idx = nidx;
        p = pn;
        base = basen;
        m = mn;
        cur ^= 1;
    }
}

}  // namespace

// Kernel shapes the set-up autotuner chooses from, per precision:
// (row tiles held per pass NRT, columns in flight per wave U), one workgroup
// per patch or persistent.
namespace {
template <typename T, typename Acc, int V, int NRT, int U>
void launch_apply_shape(hipStream_t s, const Level& L, const int64_t* off, const double* r) {
    hipLaunchKernelGGL((patch_apply_kernel<T, Acc, V, NRT, U>), dim3(L.npatch), dim3(kBlock), sizeof(Acc) * L.max_m, s,
                       L.order, L.pptr, L.pdofs_perm, off, (const T*)L.factors, r, L.Y);
}

template <typename T, typename Acc, int V, int NRT, int U, int R>
void launch_persist_r(hipStream_t s, const Level& L, const int64_t* off, const double* r) {
    const int ldbuf = (L.max_m + 1) & ~1;
    const size_t lds = 2 * sizeof(Acc) * (size_t)ldbuf;
    auto kernel = patch_apply_persist_kernel<T, Acc, V, NRT, U, R>;
    static int resident = 0;                          // workgroups resident on the whole GPU
    if (resident == 0) {
        int per_cu = 0, ncu = 0, dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kernel, kBlock, lds);
        resident = std::max(1, per_cu) * std::max(1, ncu);
    }
    const int grid = std::min(L.npatch, resident);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), lds, s, L.npatch, L.order, L.pptr, L.pdofs_perm, off,
                       (const T*)L.factors, r, L.Y, ldbuf);
}

template <typename T, typename Acc, int V, int NRT, int U>
void launch_persist_shape(hipStream_t s, const Level& L, const int64_t* off, const double* r) {
    const int R = (L.max_m + kBlock - 1) / kBlock;
    if (R <= 1) launch_persist_r<T, Acc, V, NRT, U, 1>(s, L, off, r);
    else if (R <= 2) launch_persist_r<T, Acc, V, NRT, U, 2>(s, L, off, r);
    else launch_persist_r<T, Acc, V, NRT, U, 4>(s, L, off, r);
}
}  // namespace

int apply_variant_count(int prec) { return prec == PHMG_PREC_F64 ? 9 : 6; }

void launch_patch_apply(hipStream_t s, const Level& L, const double* r) {
    if (L.npatch <= 0) return;
    const int v = L.apply_variant;
    if (L.prec == PHMG_PREC_F32) {
        switch (v) {
            case 1: launch_apply_shape<float, float, 2, 1, 8>(s, L, L.fofflp, r); break;
            case 2: launch_apply_shape<float, float, 2, 2, 2>(s, L, L.fofflp, r); break;
            case 3: launch_apply_shape<float, float, 2, 1, 4>(s, L, L.fofflp, r); break;
            case 4: launch_persist_shape<float, float, 2, 2, 4>(s, L, L.fofflp, r); break;
            case 5: launch_persist_shape<float, float, 2, 1, 8>(s, L, L.fofflp, r); break;
            default: launch_apply_shape<float, float, 2, 2, 4>(s, L, L.fofflp, r);
        }
    } else if (L.prec == PHMG_PREC_BF16) {
        switch (v) {
            case 1: launch_apply_shape<__hip_bfloat16, float, 4, 1, 8>(s, L, L.fofflp, r); break;
            case 2: launch_apply_shape<__hip_bfloat16, float, 4, 1, 2>(s, L, L.fofflp, r); break;
            case 3: launch_apply_shape<__hip_bfloat16, float, 4, 2, 4>(s, L, L.fofflp, r); break;
            case 4: launch_persist_shape<__hip_bfloat16, float, 4, 1, 4>(s, L, L.fofflp, r); break;
            case 5: launch_persist_shape<__hip_bfloat16, float, 4, 1, 8>(s, L, L.fofflp, r); break;
            default: launch_apply_shape<__hip_bfloat16, float, 4, 1, 4>(s, L, L.fofflp, r);
        }
    } else {
        switch (v) {
            case 1: launch_apply_shape<double, double, 1, 3, 4>(s, L, L.foff, r); break;
            case 2: launch_apply_shape<double, double, 1, 2, 4>(s, L, L.foff, r); break;
            case 3: launch_apply_shape<double, double, 1, 4, 2>(s, L, L.foff, r); break;
            case 4: launch_apply_shape<double, double, 1, 1, 8>(s, L, L.foff, r); break;
            case 5: launch_apply_shape<double, double, 1, 3, 2>(s, L, L.foff, r); break;
            case 6: launch_persist_shape<double, double, 1, 4, 4>(s, L, L.foff, r); break;
            case 7: launch_persist_shape<double, double, 1, 3, 4>(s, L, L.foff, r); break;
            case 8: launch_persist_shape<double, double, 1, 2, 4>(s, L, L.foff, r); break;
            default: launch_apply_shape<double, double, 1, 4, 4>(s, L, L.foff, r);
        }
    }
}

}  // namespace phmg
