// gfx950 batched patch solve of the additive Schwarz sweep (Section 3.4,
// eq. "eq:ASM"): y_i = K_i^{-1} r[S_i] for every Vanka-star patch, streaming the
// explicit patch inverses stored by the set-up.  This is the dominant kernel of
// the solve phase (HBM-bound: every factor word is read once per sweep).
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

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

template <typename T, typename Acc, int V, int NRT, int U>
__global__ __launch_bounds__(kBlock) void patch_apply_kernel(const int32_t* __restrict__ order,
                                                             const int64_t* __restrict__ pptr,
                                                             const int32_t* __restrict__ pdofs,
                                                             const int64_t* __restrict__ foff,
                                                             const T* __restrict__ F, const double* __restrict__ r,
                                                             double* __restrict__ Y) {
    constexpr int NW = kBlock / kWave;
    constexpr int TILE = kWave * V;
    extern __shared__ double s_buf[];
    Acc* s_r = reinterpret_cast<Acc*>(s_buf);
    __shared__ Acc s_red[NRT][NW][TILE];
    const int p = order[blockIdx.x];
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    const int ld = (m + V - 1) / V * V;
    for (int t = threadIdx.x; t < m; t += kBlock) s_r[t] = (Acc)r[pdofs[base + t]];
    __syncthreads();
    const T* A = F + foff[p];
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
                Y[base + i] = (double)((s_red[q][0][e] + s_red[q][1][e]) + (s_red[q][2][e] + s_red[q][3][e]));
            }
        }
        __syncthreads();
    }
}

}  // namespace

// Kernel shapes the set-up autotuner chooses from, per precision:
// (row tiles held per pass NRT, columns in flight per wave U).
namespace {
template <typename T, typename Acc, int V, int NRT, int U>
void launch_apply_shape(hipStream_t s, const Level& L, const int64_t* off, const double* r) {
    hipLaunchKernelGGL((patch_apply_kernel<T, Acc, V, NRT, U>), dim3(L.npatch), dim3(kBlock), sizeof(Acc) * L.max_m, s,
                       L.order, L.pptr, L.pdofs_perm, off, (const T*)L.factors, r, L.Y);
}
}  // namespace

int apply_variant_count(int prec) { return prec == PHMG_PREC_F64 ? 6 : 4; }

void launch_patch_apply(hipStream_t s, const Level& L, const double* r) {
    if (L.npatch <= 0) return;
    const int v = L.apply_variant;
    if (L.prec == PHMG_PREC_F32) {
        switch (v) {
            case 1: launch_apply_shape<float, float, 2, 1, 8>(s, L, L.fofflp, r); break;
            case 2: launch_apply_shape<float, float, 2, 2, 2>(s, L, L.fofflp, r); break;
            case 3: launch_apply_shape<float, float, 2, 1, 4>(s, L, L.fofflp, r); break;
            default: launch_apply_shape<float, float, 2, 2, 4>(s, L, L.fofflp, r);
        }
    } else if (L.prec == PHMG_PREC_BF16) {
        switch (v) {
            case 1: launch_apply_shape<__hip_bfloat16, float, 4, 1, 8>(s, L, L.fofflp, r); break;
            case 2: launch_apply_shape<__hip_bfloat16, float, 4, 1, 2>(s, L, L.fofflp, r); break;
            case 3: launch_apply_shape<__hip_bfloat16, float, 4, 2, 4>(s, L, L.fofflp, r); break;
            default: launch_apply_shape<__hip_bfloat16, float, 4, 1, 4>(s, L, L.fofflp, r);
        }
    } else {
        switch (v) {
            case 1: launch_apply_shape<double, double, 1, 3, 4>(s, L, L.foff, r); break;
            case 2: launch_apply_shape<double, double, 1, 2, 4>(s, L, L.foff, r); break;
            case 3: launch_apply_shape<double, double, 1, 4, 2>(s, L, L.foff, r); break;
            case 4: launch_apply_shape<double, double, 1, 1, 8>(s, L, L.foff, r); break;
            case 5: launch_apply_shape<double, double, 1, 3, 2>(s, L, L.foff, r); break;
            default: launch_apply_shape<double, double, 1, 4, 4>(s, L, L.foff, r);
        }
    }
}

}  // namespace phmg
