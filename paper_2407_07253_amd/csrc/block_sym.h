// Block patch solve on the symmetric strip layout (templates; each precision is
// instantiated in a translation unit of its own, block_sym_<prec>.hip, so the
// unrolled kernels compile in parallel).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "mfma.h"
#include "phmg_internal.h"

namespace phmg {
namespace blocksym {

// ---------------------------------------------------------------------------
// Block patch solve on the symmetric strip layout (the layout of the
// single-system solve on symmetric levels): Y_i = S_i G_i, one workgroup of
// four waves per patch.  The stored part of S_i is cut into 16 x 16 tiles
// (s, t), t <= s, numbered in strip-major order; tile u belongs to wave u % 4.
// A tile is loaded once (lane l: row l % 16, columns 4 kk + l / 16 of the tile,
// one element per MFMA operand) and feeds
//   * the row product  Y[strip s] += L(s, t) G[block t]   (4 MFMAs), and
//   * the transposed product  Y[block t] += L(s, t)^T G[strip s]  (4 MFMAs) on
//     the tile transposed through a 16 x 17 LDS buffer of the wave.
// With L the stored entries (S = L + L^T, phmg_internal.h) a diagonal tile
// holds L_ss and takes both products into block s.  Every wave keeps an
// accumulator tile for each of the NB 16-row blocks of Y in registers (its tile
// list is fixed at compile time, so every accumulator index is a constant); the
// four partial results are then added in wave order through LDS.  PD tiles of a wave are loaded ahead of the one being
// multiplied; PD does not change the arithmetic, so all shapes give the same
// bits.  G (16 NB x 16) sits in LDS.
// ---------------------------------------------------------------------------
template <bool ST>
__device__ inline double sym_ld(const double* p) { return ST ? __builtin_nontemporal_load(p) : *p; }
template <bool ST>
__device__ inline float sym_ld(const float* p) { return ST ? __builtin_nontemporal_load(p) : *p; }
template <bool ST>
__device__ inline float sym_ld(const __hip_bfloat16* p) {
    const uint16_t* q = reinterpret_cast<const uint16_t*>(p);
    const uint16_t v = ST ? __builtin_nontemporal_load(q) : *q;
    return __uint_as_float((uint32_t)v << 16);
}

__host__ __device__ constexpr int tile_strip(int i) {
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= i) ++s;
    return s;
}
__host__ __device__ constexpr int tile_col(int i) { return i - tile_strip(i) * (tile_strip(i) + 1) / 2; }

// tile (s, t) of a patch with m DoFs: lane (li, lk) gets the stored entry L(16 s + li, 16 t + 4 kk + lk)
// (S = L + L^T, see phmg_internal.h), zero where nothing is stored (padding rows of the last strip,
// columns past the diagonal block, rows above a diagonal column's stored row groups)
template <typename T, typename Acc, bool ST>
__device__ inline void sym_tile_load(const T* A, int m, int s, int t, int li, int lk, Acc (&a)[4]) {
    constexpr int VP = factor_pad<T>();
    const int r0 = s * kStrip, h = min(kStrip, m - r0), hp = (h + VP - 1) / VP * VP;
    const T* S = A + sym_strip_offset(s, VP);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int c = 4 * kk + lk;                      // column inside the tile
        int64_t off;
        bool ok = li < hp;
        if (t < s) {
            off = (int64_t)(t * kStrip + c) * hp + li;
        } else {
            constexpr int PG = sym_pack(VP);
            const int gc = c / PG * PG;
            ok = ok && c < h && li >= gc;
            off = (int64_t)hp * r0 + sym_diag_offset(min(c, h - 1), hp, PG) + (max(li, gc) - gc);
        }
        a[kk] = ok ? (Acc)sym_ld<ST>(S + off) : (Acc)0;
    }
}

// the first PD tiles of wave W (tile numbers W, W + 4, ...)
template <typename T, typename Acc, int NB, int PD, bool ST, int W>
__device__ inline void sym_wave_prologue(Acc (&buf)[PD][4], const T* A, int m, int ns, int li, int lk) {
    constexpr int NTILE = NB * (NB + 1) / 2;
#pragma unroll
    for (int k = 0; k < PD; ++k) {
        const int i = W + 4 * k;
        if (i < NTILE && tile_strip(i) < ns) sym_tile_load<T, Acc, ST>(A, m, tile_strip(i), tile_col(i), li, lk, buf[k]);
    }
}

// the tiles of wave W, PD of them loaded ahead of the one being multiplied
template <typename T, typename Acc, int NB, int PD, bool ST, int W>
__device__ inline void sym_wave_tiles(typename Mfma<Acc>::acc_t (&acc)[NB], Acc (&buf)[PD][4], const T* A, int m,
                                      int ns, int li, int lk, const Acc* s_g, Acc* s_t) {
    constexpr int NTILE = NB * (NB + 1) / 2;
    constexpr int TLD = kStrip + 1;
#pragma clang loop unroll(full)
    for (int s = 0; s < NB; ++s) {
#pragma clang loop unroll(full)
        for (int t = 0; t <= s; ++t) {
            const int i = s * (s + 1) / 2 + t;
            if (i % 4 == W) {
                const int k = (i - W) / 4;
                if (s < ns) {
                    Acc a[4], gr[4];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        a[kk] = buf[k % PD][kk];
                        gr[kk] = s_g[(t * kStrip + 4 * kk + lk) * kBS + li];
                    }
                    // L(s, t) G_t into block s and L(s, t)^T G_s into block t (for a diagonal tile
                    // both go to block s: the diagonal block is L_ss + L_ss^T)
                    Acc* tb = s_t + (k & 1) * kStrip * TLD;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) tb[(4 * kk + lk) * TLD + li] = a[kk];
                    __builtin_amdgcn_wave_barrier();
                    Acc at[4], gc[4];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        at[kk] = tb[li * TLD + 4 * kk + lk];
                        gc[kk] = s_g[(s * kStrip + 4 * kk + lk) * kBS + li];
                    }
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        acc[s] = Mfma<Acc>::step(a[kk], gr[kk], acc[s]);
                        acc[t] = Mfma<Acc>::step(at[kk], gc[kk], acc[t]);
                    }
                }
                const int i2 = i + 4 * PD;
                if (i2 < NTILE && tile_strip(i2) < ns)
                    sym_tile_load<T, Acc, ST>(A, m, tile_strip(i2), tile_col(i2), li, lk, buf[k % PD]);
            }
        }
    }
}

template <typename T, typename Acc, int NB, int PD, bool ST>
__global__ __launch_bounds__(kBlock) void block_apply_sym_kernel(const int32_t* __restrict__ order,
                                                                 const int64_t* __restrict__ pptr,
                                                                 const int32_t* __restrict__ pdofs,
                                                                 const int64_t* __restrict__ foff,
                                                                 const T* __restrict__ F, const double* __restrict__ X,
                                                                 double* __restrict__ Y,
                                                                 const double* __restrict__ gw) {
    typedef typename Mfma<Acc>::acc_t acc_t;
    constexpr int TLD = kStrip + 1;
    constexpr int RPP = kBlock / kBS;                                  // rows of G per pass of the workgroup
    extern __shared__ double s_buf[];
    Acc* s_g = reinterpret_cast<Acc*>(s_buf);                          // G: 16 NB rows x kBS columns
    const int p = order[blockIdx.x];
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    const int ns = (m + kStrip - 1) / kStrip;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int li = lane & 15, lk = lane >> 4;
    Acc* s_t = s_g + NB * kStrip * kBS + wave * 2 * kStrip * TLD;     // this wave's transpose buffers
    const T* A = F + foff[p];
    // the wave's first tiles are in flight during the gather, which they do not need
    Acc buf[PD][4];
    switch (wave) {
        case 0: sym_wave_prologue<T, Acc, NB, PD, ST, 0>(buf, A, m, ns, li, lk); break;
        case 1: sym_wave_prologue<T, Acc, NB, PD, ST, 1>(buf, A, m, ns, li, lk); break;
        case 2: sym_wave_prologue<T, Acc, NB, PD, ST, 2>(buf, A, m, ns, li, lk); break;
        default: sym_wave_prologue<T, Acc, NB, PD, ST, 3>(buf, A, m, ns, li, lk); break;
    }
    // G = X[S_i, :] (times the DoF weights W_i in the adjoint sweep), all loads issued before the stores
    {
        const int c = threadIdx.x % kBS, r = threadIdx.x / kBS;
        int idx[NB];
        double v[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int l = r + RPP * b;
            idx[b] = l < m ? pdofs[base + l] : -1;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int l = r + RPP * b;
            v[b] = idx[b] >= 0 ? X[(int64_t)idx[b] * kBS + c] : 0.0;
            if (gw && idx[b] >= 0) v[b] *= gw[base + l];
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int l = r + RPP * b;
            if (l < ns * kStrip) s_g[l * kBS + c] = (Acc)v[b];
        }
    }
    __syncthreads();
    acc_t acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = acc_t{0, 0, 0, 0};
    switch (wave) {
        case 0: sym_wave_tiles<T, Acc, NB, PD, ST, 0>(acc, buf, A, m, ns, li, lk, s_g, s_t); break;
        case 1: sym_wave_tiles<T, Acc, NB, PD, ST, 1>(acc, buf, A, m, ns, li, lk, s_g, s_t); break;
        case 2: sym_wave_tiles<T, Acc, NB, PD, ST, 2>(acc, buf, A, m, ns, li, lk, s_g, s_t); break;
        default: sym_wave_tiles<T, Acc, NB, PD, ST, 3>(acc, buf, A, m, ns, li, lk, s_g, s_t); break;
    }
    // partial results added in wave order into the G buffer (no longer read)
    __syncthreads();
    double* s_y = reinterpret_cast<double*>(s_buf);                  // 16 NB x kBS doubles
    for (int w = 0; w < kBlock / kWave; ++w) {
        if (wave == w) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (b < ns) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = b * kStrip + Mfma<Acc>::row(lane, e);
                        double* dst = s_y + row * kBS + li;
                        *dst = (w == 0 ? 0.0 : *dst) + (double)acc[b][e];
                    }
                }
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < m * kBS; e += kBlock) Y[base * kBS + e] = s_y[e];
}

template <typename T, typename Acc, int NB, int PD>
void launch_block_sym_shape(hipStream_t s, const Level& L, const double* X, const double* gw) {
    // G and the four waves' transpose buffers, then (reused) the f64 sum of the four partial results
    const size_t lds = std::max(sizeof(Acc) * ((size_t)NB * kStrip * kBS + 8 * (size_t)kStrip * (kStrip + 1)),
                                sizeof(double) * (size_t)NB * kStrip * kBS);
    auto kernel = streams_factors(L, true) ? block_apply_sym_kernel<T, Acc, NB, PD, true>
                                           : block_apply_sym_kernel<T, Acc, NB, PD, false>;
    hipLaunchKernelGGL(kernel, dim3(L.npatch), dim3(kBlock), lds, s, L.order, L.pptr, L.pdofs, L.fofflp,
                       (const T*)L.factors, X, L.Yb, gw);
}

template <typename T, typename Acc, int NB>
void launch_block_sym_nb(hipStream_t s, const Level& L, const double* X, const double* gw) {
    switch (L.block_variant) {
        case 1: launch_block_sym_shape<T, Acc, NB, 2>(s, L, X, gw); break;
        case 2: launch_block_sym_shape<T, Acc, NB, 3>(s, L, X, gw); break;
        case 3: launch_block_sym_shape<T, Acc, NB, 4>(s, L, X, gw); break;
        default: launch_block_sym_shape<T, Acc, NB, 1>(s, L, X, gw);
    }
}

template <typename T, typename Acc>
void launch(hipStream_t s, const Level& L, const double* X, const double* gw) {
    switch (block_sym_blocks(L)) {
        case 4: launch_block_sym_nb<T, Acc, 4>(s, L, X, gw); break;
        case 9: launch_block_sym_nb<T, Acc, 9>(s, L, X, gw); break;
        default: launch_block_sym_nb<T, Acc, 14>(s, L, X, gw);
    }
}

}  // namespace blocksym
}  // namespace phmg
