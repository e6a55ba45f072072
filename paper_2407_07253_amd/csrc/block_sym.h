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
// one element per MFMA operand; bfloat16 tiles in 8-byte loads, see SymTile) and feeds
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

constexpr int kTld = kStrip + 1;                  // leading dimension of the transpose buffers

// A tile in flight and its two MFMA operand layouts.  Generic form: the tile is
// loaded in the A-operand layout (one element per lane per MFMA) and only the
// transposed operand goes through the wave's LDS buffer tb (T[c][q] at c kTld + q).
template <typename T, typename Acc>
struct SymTile {
    Acc v[4];
    template <bool ST>
    __device__ inline void load(const T* A, int m, int s, int t, int li, int lk, int /*lane*/) {
        sym_tile_load<T, Acc, ST>(A, m, s, t, li, lk, v);
    }
    // (t < s: an off-diagonal tile; the generic form loads every tile the same way)
    __device__ inline void zero() {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) v[kk] = (Acc)0;
    }
    __device__ inline void operands(Acc* tb, int li, int lk, int /*lane*/, bool /*offdiag*/, Acc (&a)[4],
                                    Acc (&at)[4]) const {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            a[kk] = v[kk];
            tb[(4 * kk + lk) * kTld + li] = v[kk];
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) at[kk] = tb[li * kTld + 4 * kk + lk];
    }
};

// bfloat16 tiles (whole stored diagonal blocks, column-major with leading dimension hp, a multiple
// of 8): lane l loads rows 4 (l % 4) .. + 3 of tile column l / 4 in one 8-byte load, and both operand
// layouts are read back from the LDS buffer -- one load instruction per tile instead of four.
template <>
struct SymTile<__hip_bfloat16, float> {
    uint32_t lo = 0, hi = 0;
    template <bool ST>
    __device__ inline void load(const __hip_bfloat16* A, int m, int s, int t, int /*li*/, int /*lk*/, int lane) {
        const int r0 = s * kStrip, h = min(kStrip, m - r0), hp = (h + 7) / 8 * 8, wc = t < s ? kStrip : h;
        const int c = lane / 4, q0 = 4 * (lane % 4);
        lo = 0;
        hi = 0;
        if (q0 < hp && c < wc) {
            typedef uint32_t u2 __attribute__((ext_vector_type(2)));
            const u2* q = reinterpret_cast<const u2*>(A + sym_strip_offset(s, 8) + (int64_t)(t * kStrip + c) * hp + q0);
            const u2 v = ST ? __builtin_nontemporal_load(q) : *q;
            lo = v.x;
            hi = v.y;
        }
    }
    __device__ inline void zero() {
        lo = 0;
        hi = 0;
    }
    __device__ inline void operands(float* tb, int li, int lk, int lane, bool /*offdiag*/, float (&a)[4],
                                    float (&at)[4]) const {
        const int c = lane / 4, q0 = 4 * (lane % 4);
        tb[c * kTld + q0] = __uint_as_float(lo << 16);
        tb[c * kTld + q0 + 1] = __uint_as_float(lo & 0xffff0000u);
        tb[c * kTld + q0 + 2] = __uint_as_float(hi << 16);
        tb[c * kTld + q0 + 3] = __uint_as_float(hi & 0xffff0000u);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            a[kk] = tb[(4 * kk + lk) * kTld + li];
            at[kk] = tb[li * kTld + 4 * kk + lk];
        }
    }
};

// float32 tiles: an off-diagonal tile (column-major, leading dimension hp, a multiple of 4) comes in
// one 16-byte load per lane (rows 4 (l % 4) .. + 3 of tile column l / 4) and both operand layouts are
// read back from LDS; a diagonal tile (packed row groups) takes the generic element loads.
template <>
struct SymTile<float, float> {
    float v[4];
    template <bool ST>
    __device__ inline void load(const float* A, int m, int s, int t, int li, int lk, int lane) {
        if (t < s) {
            const int r0 = s * kStrip, h = min(kStrip, m - r0), hp = (h + 3) / 4 * 4;
            const int c = lane / 4, q0 = 4 * (lane % 4);
            zero();
            if (q0 < hp) {
                typedef float f4v __attribute__((ext_vector_type(4)));
                const f4v* q = reinterpret_cast<const f4v*>(A + sym_strip_offset(s, 4) + (int64_t)(t * kStrip + c) * hp + q0);
                const f4v x = ST ? __builtin_nontemporal_load(q) : *q;
                v[0] = x.x;
                v[1] = x.y;
                v[2] = x.z;
                v[3] = x.w;
            }
        } else {
            sym_tile_load<float, float, ST>(A, m, s, t, li, lk, v);
        }
    }
    __device__ inline void zero() {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) v[kk] = 0.0f;
    }
    __device__ inline void operands(float* tb, int li, int lk, int lane, bool offdiag, float (&a)[4],
                                    float (&at)[4]) const {
        if (offdiag) {
            const int c = lane / 4, q0 = 4 * (lane % 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) tb[c * kTld + q0 + i] = v[i];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                a[kk] = tb[(4 * kk + lk) * kTld + li];
                at[kk] = tb[li * kTld + 4 * kk + lk];
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                a[kk] = v[kk];
                tb[(4 * kk + lk) * kTld + li] = v[kk];
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) at[kk] = tb[li * kTld + 4 * kk + lk];
        }
    }
};

// the first PD tiles of wave W (tile numbers W, W + 4, ...)
template <typename T, typename Acc, int NB, int PD, bool ST, int W>
__device__ inline void sym_wave_prologue(SymTile<T, Acc> (&buf)[PD], const T* A, int m, int ns, int li, int lk,
                                         int lane) {
    constexpr int NTILE = NB * (NB + 1) / 2;
#pragma unroll
    for (int k = 0; k < PD; ++k) {
        const int i = W + 4 * k;
        if (i < NTILE && tile_strip(i) < ns) buf[k].template load<ST>(A, m, tile_strip(i), tile_col(i), li, lk, lane);
        else buf[k].zero();
    }
}

// the tiles of wave W, PD of them loaded ahead of the one being multiplied
template <typename T, typename Acc, int NB, int PD, bool ST, int W>
__device__ inline void sym_wave_tiles(typename Mfma<Acc>::acc_t (&acc)[NB], SymTile<T, Acc> (&buf)[PD], const T* A,
                                      int m, int ns, int li, int lk, int lane, const Acc* s_g, Acc* s_t) {
    constexpr int NTILE = NB * (NB + 1) / 2;
#pragma clang loop unroll(full)
    for (int s = 0; s < NB; ++s) {
#pragma clang loop unroll(full)
        for (int t = 0; t <= s; ++t) {
            const int i = s * (s + 1) / 2 + t;
            if (i % 4 == W) {
                const int k = (i - W) / 4;
                if (s < ns) {
                    // L(s, t) G_t into block s and L(s, t)^T G_s into block t (for a diagonal tile
                    // both go to block s: the diagonal block is L_ss + L_ss^T)
                    // the G operands first: their LDS reads overlap the transpose round trip
                    Acc a[4], at[4], gr[4], gc[4];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        gr[kk] = s_g[(t * kStrip + 4 * kk + lk) * kBS + li];
                        gc[kk] = s_g[(s * kStrip + 4 * kk + lk) * kBS + li];
                    }
                    buf[k % PD].operands(s_t + (k & 1) * kStrip * kTld, li, lk, lane, t < s, a, at);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        acc[s] = Mfma<Acc>::step(a[kk], gr[kk], acc[s]);
                        acc[t] = Mfma<Acc>::step(at[kk], gc[kk], acc[t]);
                    }
                }
                const int i2 = i + 4 * PD;
                if (i2 < NTILE && tile_strip(i2) < ns)
                    buf[k % PD].template load<ST>(A, m, tile_strip(i2), tile_col(i2), li, lk, lane);
            }
        }
    }
}

template <typename T, typename Acc, int NB, int PD, bool ST>
__global__ __launch_bounds__(kBlock) void block_apply_sym_kernel(const int64_t* __restrict__ pinfo,
                                                                 const int32_t* __restrict__ pdofs,
                                                                 const T* __restrict__ F, const double* __restrict__ X,
                                                                 double* __restrict__ Y,
                                                                 const double* __restrict__ gw) {
    typedef typename Mfma<Acc>::acc_t acc_t;
    constexpr int RPP = kBlock / kBS;                                  // rows of G per pass of the workgroup
    extern __shared__ double s_buf[];
    Acc* s_g = reinterpret_cast<Acc*>(s_buf);                          // G: 16 NB rows x kBS columns
    // the patch at this launch position (first slot, factor offset, size) in one read
    const int64_t* info = pinfo + 4 * (int64_t)blockIdx.x;
    const int64_t base = info[0];
    const int m = (int)info[2];
    const int ns = (m + kStrip - 1) / kStrip;
    const int lane = threadIdx.x & (kWave - 1), wave = wave_id();
    const int li = lane & 15, lk = lane >> 4;
    Acc* s_t = s_g + NB * kStrip * kBS + wave * 2 * kStrip * kTld;    // this wave's transpose buffers
    const T* A = F + info[1];
    // the wave's first tiles are in flight during the gather, which they do not need
    SymTile<T, Acc> buf[PD];
    switch (wave) {
        case 0: sym_wave_prologue<T, Acc, NB, PD, ST, 0>(buf, A, m, ns, li, lk, lane); break;
        case 1: sym_wave_prologue<T, Acc, NB, PD, ST, 1>(buf, A, m, ns, li, lk, lane); break;
        case 2: sym_wave_prologue<T, Acc, NB, PD, ST, 2>(buf, A, m, ns, li, lk, lane); break;
        default: sym_wave_prologue<T, Acc, NB, PD, ST, 3>(buf, A, m, ns, li, lk, lane); break;
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
        case 0: sym_wave_tiles<T, Acc, NB, PD, ST, 0>(acc, buf, A, m, ns, li, lk, lane, s_g, s_t); break;
        case 1: sym_wave_tiles<T, Acc, NB, PD, ST, 1>(acc, buf, A, m, ns, li, lk, lane, s_g, s_t); break;
        case 2: sym_wave_tiles<T, Acc, NB, PD, ST, 2>(acc, buf, A, m, ns, li, lk, lane, s_g, s_t); break;
        default: sym_wave_tiles<T, Acc, NB, PD, ST, 3>(acc, buf, A, m, ns, li, lk, lane, s_g, s_t); break;
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
    hipLaunchKernelGGL(kernel, dim3(L.npatch), dim3(kBlock), lds, s, L.pinfo, L.pdofs, (const T*)L.factors, X,
                       L.Yb, gw);
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
