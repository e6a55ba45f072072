// gfx950 kernels of the multi-right-hand-side (block) path: up to kBS = 16
// systems K x_c = b_c relaxed, cycled and solved together.
//
// Block vectors are stored interleaved, X[i * kBS + c] for DoF i and
// right-hand side c, so the kBS values of one DoF are one 128-byte line: every
// CSR entry and every patch DoF gathers a full line.
//
//  * spmm_kernel,         Y = alpha K X + beta Z (residuals, transfers): 16
//    spmm_quad_kernel     lanes per row, or 2 / 4 lanes of 8 / 4 columns each
//  * block_apply_kernel   Y_i = K_i^{-1} X[S_i, :] for every patch as a dense
//                         m x m by m x 16 product on MFMA (f64 16x16x4 for
//                         float64 factors, f32 16x16x4 with float32
//                         accumulation for float32 / bfloat16 factors); each
//                         factor word is read once per sweep for all 16 systems
//  * block_scatter_kernel the weighted DoF-centric sum of eq. "eq:ASM"
//  * block FGMRES kernels classical Gram-Schmidt passes per column
//
// Columns never mix: column c of every result depends on column c of the
// inputs only, in a fixed summation order, so results are reproducible.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "mfma.h"
#include "phmg_internal.h"

namespace phmg {
namespace {

inline int grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (1 << 20)) g = 1 << 20;
    return (int)g;
}

// ---------------------------------------------------------------------------
// Y = alpha K X + beta Z (Z may be null or alias Y).  kBS * GN lanes per row:
// lane (c, g) sums the entries g, g + GN, ... of the row for column c; the GN
// partial sums are combined with shuffles.  XM: XCD-contiguous row ranges
// (as in the single-vector SpMV; the grid is then a multiple of 8).
// ---------------------------------------------------------------------------
__device__ inline int64_t logical_block(bool xm) {
    if (!xm) return blockIdx.x;
    const int64_t per = gridDim.x / 8;
    return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

template <int GN, bool XM>
__global__ __launch_bounds__(kBlock) void spmm_kernel(int32_t nrows, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const double* __restrict__ val,
                                                      const double* __restrict__ X, double alpha, const double* Z,
                                                      double beta, double* Y) {
    constexpr int LPR = kBS * GN;
    const int c = threadIdx.x & (kBS - 1);
    const int g = (threadIdx.x / kBS) & (GN - 1);
    const int64_t sub = (logical_block(XM) * blockDim.x + threadIdx.x) / LPR;
    const int64_t nsub = ((int64_t)gridDim.x * blockDim.x) / LPR;
    for (int64_t row = sub; row < nrows; row += nsub) {
        const int beg = rowptr[row], end = rowptr[row + 1];
        double s = 0.0;
        if (GN == 1) {
            // the 16 lanes of the row load 16 indices at once and broadcast them, so
            // the 16 gathers of a chunk are independent loads; entries are still
            // added in row order
            for (int k0 = beg; k0 < end; k0 += kBS) {
                const int cnt = min(kBS, end - k0);
                int ck = 0;
                double vk = 0.0;
                if (c < cnt) {
                    ck = col[k0 + c];
                    vk = val[k0 + c];
                }
#pragma unroll
                for (int t = 0; t < kBS; ++t) {
                    const int cc = __shfl(ck, t, kBS);
                    const double vv = __shfl(vk, t, kBS);
                    if (t < cnt) s += vv * X[(int64_t)cc * kBS + c];
                }
            }
        } else {
            for (int k = beg + g; k < end; k += GN) s += val[k] * X[(int64_t)col[k] * kBS + c];
        }
#pragma unroll
        for (int off = LPR / 2; off >= kBS; off >>= 1) s += __shfl_xor(s, off, LPR);
        if (g == 0) {
            double out = alpha * s;
            if (Z) out += beta * Z[row * kBS + c];
            Y[row * kBS + c] = out;
        }
    }
}

// ---------------------------------------------------------------------------
// Y = alpha K X + beta Z with LPR = 4 (or 2) lanes per row and 16 / LPR columns
// of X per lane (64 / LPR rows per wave; a row of X is read in 32-byte pieces).
// The lanes of a row load 4 LPR entries at once (entry k0 + LPR j + l in lane l)
// and pass them round with quad DPP broadcasts (no LDS); each column sums the
// row's entries in row order, as spmm_kernel<1, false> does, so the bits are
// that kernel's.
// ---------------------------------------------------------------------------
template <int LPR, int T>
__device__ inline int row_bcast(int x) {
    // lane T of each group of LPR lanes inside a quad, to the whole group
    constexpr int C = LPR == 4 ? (T | T << 2 | T << 4 | T << 6) : (T | T << 2 | (T + 2) << 4 | (T + 2) << 6);
    return __builtin_amdgcn_update_dpp(0, x, C, 0xF, 0xF, false);
}
template <int LPR, int T>
__device__ inline double row_bcast_d(double x) {
    const int lo = row_bcast<LPR, T>(__double2loint(x)), hi = row_bcast<LPR, T>(__double2hiint(x));
    return __hiloint2double(hi, lo);
}
typedef double dq4 __attribute__((ext_vector_type(4)));

template <int LPR, bool XM>
__global__ __launch_bounds__(kBlock) void spmm_quad_kernel(int32_t nrows, const int32_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           const double* __restrict__ X, double alpha, const double* Z,
                                                           double beta, double* Y) {
    static_assert(LPR == 2 || LPR == 4, "lanes per row");
    constexpr int CPL = kBS / LPR, NQ = CPL / 4, CH = 4 * LPR;   // columns per lane, 32-byte pieces, chunk
    const int l = threadIdx.x & (LPR - 1);         // columns CPL l .. CPL l + CPL - 1
    const int64_t sub = (logical_block(XM) * blockDim.x + threadIdx.x) / LPR;
    const int64_t nsub = ((int64_t)gridDim.x * blockDim.x) / LPR;
    for (int64_t row = sub; row < nrows; row += nsub) {
        const int beg = rowptr[row], end = rowptr[row + 1];
        dq4 s[NQ];
#pragma unroll
        for (int h = 0; h < NQ; ++h) s[h] = dq4{0.0, 0.0, 0.0, 0.0};
        for (int k0 = beg; k0 < end; k0 += CH) {
            const int cnt = min(CH, end - k0);
            int ck[4];
            double vk[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = LPR * j + l;
                ck[j] = k < cnt ? col[k0 + k] : 0;
                vk[j] = k < cnt ? val[k0 + k] : 0.0;
            }
            auto step = [&](int cc, double vv) {
                const double* xr = X + (int64_t)cc * kBS + CPL * l;
#pragma unroll
                for (int h = 0; h < NQ; ++h) {
                    const dq4 x = *reinterpret_cast<const dq4*>(xr + 4 * h);
#pragma unroll
                    for (int e = 0; e < 4; ++e) s[h][e] += vv * x[e];
                }
            };
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (LPR * j + 0 < cnt) step(row_bcast<LPR, 0>(ck[j]), row_bcast_d<LPR, 0>(vk[j]));
                if (LPR * j + 1 < cnt) step(row_bcast<LPR, 1>(ck[j]), row_bcast_d<LPR, 1>(vk[j]));
                if constexpr (LPR == 4) {
                    if (LPR * j + 2 < cnt) step(row_bcast<LPR, 2>(ck[j]), row_bcast_d<LPR, 2>(vk[j]));
                    if (LPR * j + 3 < cnt) step(row_bcast<LPR, 3>(ck[j]), row_bcast_d<LPR, 3>(vk[j]));
                }
            }
        }
#pragma unroll
        for (int h = 0; h < NQ; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t o = row * kBS + CPL * l + 4 * h + e;
                double out = alpha * s[h][e];
                if (Z) out += beta * Z[o];
                Y[o] = out;
            }
    }
}

// ---------------------------------------------------------------------------
// Block patch solve.  One workgroup per patch (launch order: decreasing m).
// The gathered right-hand sides G = X[P S_i, :] (m x 16, rows padded with
// zeros to a multiple of 4) sit in LDS.  The stored inverse B_i (column-major,
// leading dimension ld = m rounded up to factor_pad) is streamed once: in one k-step of
// 4 columns, lane l loads V consecutive rows of column k0 + l/16 (an 8-byte
// load for every precision) and feeds V MFMAs, MFMA v taking the rows
// r0 + V*i + v (i = l % 16) as its 16-row A tile; the B operand is G[k0 + l/16]
// [l % 16].  A wave owns NT such 16V-row groups per pass; passes are dealt to
// the four waves round-robin.  The result rows go to the staging array Y
// (sum m x 16) for the scatter.
// ---------------------------------------------------------------------------
template <typename T, int V>
struct BlockLoad;
typedef float st_f2 __attribute__((ext_vector_type(2)));
typedef uint32_t st_u2 __attribute__((ext_vector_type(2)));
template <>
struct BlockLoad<double, 1> {
    template <bool ST>
    __device__ static inline void load(const double* p, double (&a)[1]) {
        a[0] = ST ? __builtin_nontemporal_load(p) : *p;
    }
};
template <>
struct BlockLoad<float, 2> {
    template <bool ST>
    __device__ static inline void load(const float* p, float (&a)[2]) {
        const st_f2* q = reinterpret_cast<const st_f2*>(p);
        const st_f2 v = ST ? __builtin_nontemporal_load(q) : *q;
        a[0] = v.x;
        a[1] = v.y;
    }
};
template <>
struct BlockLoad<__hip_bfloat16, 4> {
    template <bool ST>
    __device__ static inline void load(const __hip_bfloat16* p, float (&a)[4]) {
        const st_u2* q = reinterpret_cast<const st_u2*>(p);
        const st_u2 v = ST ? __builtin_nontemporal_load(q) : *q;
        a[0] = __uint_as_float(v.x << 16);
        a[1] = __uint_as_float(v.x & 0xffff0000u);
        a[2] = __uint_as_float(v.y << 16);
        a[3] = __uint_as_float(v.y & 0xffff0000u);
    }
};

template <typename T, typename Acc, int V, int NT, int U, bool ST>
__global__ __launch_bounds__(kBlock) void block_apply_kernel(const int32_t* __restrict__ order,
                                                             const int64_t* __restrict__ pptr,
                                                             const int32_t* __restrict__ pdofs,
                                                             const int64_t* __restrict__ foff,
                                                             const T* __restrict__ F, const double* __restrict__ X,
                                                             double* __restrict__ Y,
                                                             const double* __restrict__ gw,
                                                             const int32_t* __restrict__ pidx) {
    typedef typename Mfma<Acc>::acc_t acc_t;
    constexpr int NW = kBlock / kWave;
    constexpr int GROUP = 16 * V;                 // rows of one row group
    constexpr int PASS = GROUP * NT;              // rows of one pass of a wave
    extern __shared__ double s_buf[];
    Acc* s_g = reinterpret_cast<Acc*>(s_buf);
    const int p = order[blockIdx.x];
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    const int mpad = (m + 3) & ~3;
    const int ld = (m + factor_pad<T>() - 1) / factor_pad<T>() * factor_pad<T>();
    // gw (adjoint sweep): the weight of the gathered DoF, W_i before the solve
    for (int t = threadIdx.x; t < mpad * kBS; t += kBlock) {
        const int l = t / kBS, c = t % kBS;
        double v = 0.0;
        if (l < m) {
            v = X[(int64_t)pdofs[base + l] * kBS + c];
            if (gw) v *= gw[base + pidx[base + l]];
        }
        s_g[t] = (Acc)v;
    }
    __syncthreads();
    const T* A = F + foff[p];
    const int lane = threadIdx.x & (kWave - 1), wave = wave_id();
    const int li = lane & 15, lk = lane >> 4;
    const int npass = (m + PASS - 1) / PASS;
    for (int pass = wave; pass < npass; pass += NW) {
        const int r0 = pass * PASS;
        acc_t acc[NT][V];
#pragma unroll
        for (int q = 0; q < NT; ++q)
#pragma unroll
            for (int v = 0; v < V; ++v) acc[q][v] = acc_t{0, 0, 0, 0};
        bool rowok[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) rowok[q] = r0 + q * GROUP + li * V < m;
        int k0 = 0;
        for (; k0 + 4 * (U - 1) < mpad; k0 += 4 * U) {
            Acc a[U][NT][V];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = k0 + 4 * u + lk;
                const T* colp = A + (int64_t)k * ld + r0 + li * V;
#pragma unroll
                for (int q = 0; q < NT; ++q) {
                    if (rowok[q] && k < m) BlockLoad<T, V>::template load<ST>(colp + q * GROUP, a[u][q]);
                    else
#pragma unroll
                        for (int v = 0; v < V; ++v) a[u][q][v] = 0;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const Acc b = s_g[(k0 + 4 * u + lk) * kBS + li];
#pragma unroll
                for (int q = 0; q < NT; ++q)
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[q][v] = Mfma<Acc>::step(a[u][q][v], b, acc[q][v]);
            }
        }
        for (; k0 < mpad; k0 += 4) {
            const int k = k0 + lk;
            const T* colp = A + (int64_t)k * ld + r0 + li * V;
            const Acc b = s_g[k * kBS + li];
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                Acc a[V];
                if (rowok[q] && k < m) BlockLoad<T, V>::template load<ST>(colp + q * GROUP, a);
                else
#pragma unroll
                    for (int v = 0; v < V; ++v) a[v] = 0;
#pragma unroll
                for (int v = 0; v < V; ++v) acc[q][v] = Mfma<Acc>::step(a[v], b, acc[q][v]);
            }
        }
#pragma unroll
        for (int q = 0; q < NT; ++q)
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = r0 + q * GROUP + Mfma<Acc>::row(lane, e) * V + v;
                    if (row < m) Y[(base + row) * kBS + li] = (double)acc[q][v][e];
                }
    }
}

// ---------------------------------------------------------------------------
// s = sum_{slots t of DoF j, ascending patch id} w_t Y[t, c] (or wd_j times the
// unweighted sum, one weight per DoF);  dn = a s + c' d;
// X = (x_zero ? 0 : X) + dn;  d = dn when storing.  One lane per (DoF, column).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void block_scatter_kernel(int32_t n, const int32_t* __restrict__ sptr,
                                                               const int32_t* __restrict__ sslot,
                                                               const double* __restrict__ w,
                                                               const double* __restrict__ wd,
                                                               const double* __restrict__ Y, double a, double cd,
                                                               double* __restrict__ d, double* __restrict__ x,
                                                               int flags) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t j = t / kBS;
    const int c = (int)(t % kBS);
    if (j >= n) return;
    const double wj = wd ? wd[j] : 1.0;
    double s = 0.0;
    const int end = sptr[j + 1];
    // four slots in flight, summed in ascending slot order (a missing slot adds +0)
    for (int t = sptr[j]; t < end; t += 4) {
        int q[4];
        double y[4], wq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = t + u < end ? sslot[t + u] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            y[u] = q[u] >= 0 ? Y[(int64_t)q[u] * kBS + c] : 0.0;
            wq[u] = w && q[u] >= 0 ? w[q[u]] : 1.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s += w ? wq[u] * y[u] : y[u];
    }
    if (wd) s *= wj;
    double dn = a * s;
    if (flags & 2) dn = cd * d[t] + dn;
    x[t] = (flags & 1) ? dn : x[t] + dn;
    if (flags & 4) d[t] = dn;
}

// X[i, c] = sum_{j < n} Ainv_rm[i * nb + j] B[j, c]: one wavefront per row,
// lane (c, q) sums j = q, q + 4, ...
__global__ __launch_bounds__(kBlock) void block_coarse_solve_kernel(int32_t n, int32_t nb,
                                                                    const double* __restrict__ Ainv,
                                                                    const double* __restrict__ B,
                                                                    double* __restrict__ X) {
    const int lane = threadIdx.x & (kWave - 1);
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (row >= n) return;
    const int c = lane & (kBS - 1), q = lane / kBS;
    const double* a = Ainv + (int64_t)row * nb;
    double s = 0.0;
    for (int j = q; j < n; j += kWave / kBS) s += a[j] * B[(int64_t)j * kBS + c];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (q == 0) X[(int64_t)row * kBS + c] = s;
}

// ---------------------------------------------------------------------------
// Gram-Schmidt passes over the block Krylov basis V_0..V_{ncol-1} (each n x 16,
// stride ldv), over the rows with per-thread accumulators:
//   MODE 0: h_j = V_j^T w                      (per column)
//   MODE 1: w <- w - sum_j V_j h_j, then h'_j = V_j^T w (h' into the partials)
//   MODE 2: w <- w - sum_j V_j h_j, then ||w||^2
// The products are formed in chunks of kGsChunk basis vectors, one pass over the
// rows per chunk (the first pass also updates w; later passes re-read it), so a
// thread keeps kGsChunk accumulators instead of one per basis vector: with few
// registers the fixed grid of kBlockGsBlocks workgroups stays resident at 8
// waves per SIMD and keeps enough loads in flight.  Partials per workgroup:
// partial[(j * kBS + c) * gridDim.x + block].
// ---------------------------------------------------------------------------
constexpr int kMaxBasis = 32;
constexpr int kGsChunk = 8;

template <int MODE>
__global__ __launch_bounds__(kBlock) void block_gs_kernel(int64_t n, int ncol, const double* __restrict__ V,
                                                          int64_t ldv, double* __restrict__ w,
                                                          const double* __restrict__ h,
                                                          double* __restrict__ partial) {
    __shared__ double sh[kGsChunk][kBlock / kWave][kBS];
    __shared__ double s_h[kMaxBasis][kBS];
    const int c = threadIdx.x & (kBS - 1);
    const int lane = threadIdx.x & (kWave - 1), wave = wave_id();
    if (MODE != 0) {
        for (int t = threadIdx.x; t < kMaxBasis * kBS; t += kBlock) {
            const int j = t / kBS;
            s_h[j][t % kBS] = j < ncol ? h[t] : 0.0;
        }
        __syncthreads();
    }
    const int64_t rows_per_grid = ((int64_t)gridDim.x * kBlock) / kBS;
    const int64_t i0 = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kBS;
    const int nchunk = MODE == 2 ? 1 : (ncol + kGsChunk - 1) / kGsChunk;
    for (int ch = 0; ch < nchunk; ++ch) {
        double dot[kGsChunk];
#pragma unroll
        for (int q = 0; q < kGsChunk; ++q) dot[q] = 0.0;
        for (int64_t i = i0; i < n; i += rows_per_grid) {
            const int64_t e = i * kBS + c;
            double wi = w[e];
            if (MODE != 0 && ch == 0) {
                double s = 0.0;
#pragma unroll 8
                for (int j = 0; j < ncol; ++j) s += V[j * ldv + e] * s_h[j][c];
                wi -= s;
                w[e] = wi;
            }
            if (MODE == 2) {
                dot[0] += wi * wi;
            } else {
#pragma unroll
                for (int q = 0; q < kGsChunk; ++q) {
                    const int j = ch * kGsChunk + q;
                    if (j < ncol) dot[q] += V[j * ldv + e] * wi;
                }
            }
        }
        const int nq = MODE == 2 ? 1 : min(kGsChunk, ncol - ch * kGsChunk);
#pragma unroll
        for (int q = 0; q < kGsChunk; ++q) {
            if (q < nq) {
                double v = dot[q];
                v += __shfl_xor(v, 16);
                v += __shfl_xor(v, 32);
                if (lane < kBS) sh[q][wave][lane] = v;
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < nq * kBS; t += kBlock) {
            const int q = t / kBS, cc = t % kBS;
            const int64_t slot = (int64_t)((ch * kGsChunk + q) * kBS + cc);
            partial[slot * gridDim.x + blockIdx.x] = (sh[q][0][cc] + sh[q][1][cc]) + (sh[q][2][cc] + sh[q][3][cc]);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void block_reduce_kernel(int nparts, const double* __restrict__ partial,
                                                              double* __restrict__ out) {
    __shared__ double sh[kBlock / kWave];
    const int t = blockIdx.x;
    double s = 0.0;
    for (int q = threadIdx.x; q < nparts; q += kBlock) s += partial[(int64_t)t * nparts + q];
    for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
    const int lane = threadIdx.x & (kWave - 1), wave = wave_id();
    if (lane == 0) sh[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[t] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// X[i, c] += sum_{j < ncol} Z_j[i, c] y[j * kBS + c]
__global__ __launch_bounds__(kBlock) void block_gemv_add_kernel(int64_t n, int ncol, const double* __restrict__ Z,
                                                                int64_t ldz, const double* __restrict__ y,
                                                                double* __restrict__ X) {
    const int64_t total = n * kBS;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % kBS);
        double s = 0.0;
        for (int j = 0; j < ncol; ++j) s += Z[j * ldz + e] * y[j * kBS + c];
        X[e] += s;
    }
}

// D[i, c] = act_c ? S[i, c] / den_c : 0   (cs = {den[kBS], act[kBS]})
__global__ __launch_bounds__(kBlock) void block_scale_kernel(int64_t n, const double* __restrict__ S,
                                                             const double* __restrict__ cs, double* __restrict__ D) {
    const int64_t total = n * kBS;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % kBS);
        D[e] = cs[kBS + c] != 0.0 ? S[e] / cs[c] : 0.0;
    }
}

// interleave nrhs right-hand-side-major vectors (src[c * n + i]) into a block
// (dst[i * kBS + c]), zero columns beyond nrhs; and back
__global__ __launch_bounds__(kBlock) void interleave_kernel(int64_t n, int nrhs, const double* __restrict__ src,
                                                            double* __restrict__ dst) {
    const int64_t total = n * kBS;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / kBS;
        const int c = (int)(e % kBS);
        dst[e] = c < nrhs ? src[(int64_t)c * n + i] : 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void deinterleave_kernel(int64_t n, int nrhs, const double* __restrict__ src,
                                                              double* __restrict__ dst) {
    const int64_t total = n * nrhs;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / n);
        const int64_t i = e % n;
        dst[e] = src[i * kBS + c];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_spmm(hipStream_t s, const DevCsr& A, const double* X, double alpha, const double* Z, double beta,
                 double* Y) {
    if (A.nrows <= 0) return;
    if (A.bquad) {
        // bquad lanes per row (2 or 4), 16 / bquad columns of X per lane
        int grid = grid_for((int64_t)A.nrows * A.bquad, kBlock);
        if (A.bxcd) grid = (grid + 7) / 8 * 8;
        auto go = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, A.nrows, A.rowptr, A.col, A.val, X, alpha, Z,
                               beta, Y);
        };
        if (A.bquad == 2) {
            if (A.bxcd) go(spmm_quad_kernel<2, true>);
            else go(spmm_quad_kernel<2, false>);
        } else {
            if (A.bxcd) go(spmm_quad_kernel<4, true>);
            else go(spmm_quad_kernel<4, false>);
        }
        return;
    }
    const int gn = A.bgroup == 2 || A.bgroup == 4 ? A.bgroup : 1;
    int grid = grid_for((int64_t)A.nrows * kBS * gn, kBlock);
    if (A.bxcd) grid = (grid + 7) / 8 * 8;
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, A.nrows, A.rowptr, A.col, A.val, X, alpha, Z,
                           beta, Y);
    };
    switch (gn * 2 + (A.bxcd ? 1 : 0)) {
        case 2: go(spmm_kernel<1, false>); break;
        case 3: go(spmm_kernel<1, true>); break;
        case 4: go(spmm_kernel<2, false>); break;
        case 5: go(spmm_kernel<2, true>); break;
        case 8: go(spmm_kernel<4, false>); break;
        default: go(spmm_kernel<4, true>); break;
    }
}

namespace {
template <typename T, typename Acc, int V, int NT, int U>
void launch_block_shape(hipStream_t s, const Level& L, const void* factors, const int64_t* off, const double* X,
                        const double* gw) {
    const size_t lds = sizeof(Acc) * (size_t)((L.max_m + 3) & ~3) * kBS;
    // the block path streams the general layout (the general copy on symmetric levels)
    auto kernel = streams_factors(L, false) ? block_apply_kernel<T, Acc, V, NT, U, true>
                                            : block_apply_kernel<T, Acc, V, NT, U, false>;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kernel, dim3(L.npatch), dim3(kBlock), lds, s, L.order, L.pptr, L.pdofs_perm, off,
                       (const T*)factors, X, L.Yb, gw, L.pidx);
}

}  // namespace

int block_sym_blocks(const Level& L) {
    if (!L.sym || L.npatch == 0) return 0;
    const int64_t nb = (L.max_m + kStrip - 1) / kStrip;
    return nb <= 4 ? 4 : (nb <= 9 ? 9 : (nb <= 14 ? 14 : 0));
}

int block_variant_count(const Level& /*L*/) { return 4; }

void launch_block_apply(hipStream_t s, const Level& L, const double* X, bool transpose) {
    if (L.npatch <= 0) return;
    // adjoint sweep on a symmetric level: K_i^{-T} = K_i^{-1} up to the level's
    // rounding asymmetry, applied to the weighted gather
    const double* gw = transpose ? L.pweight : nullptr;
    if (block_sym_blocks(L) > 0) {
        if (L.prec == PHMG_PREC_F32) launch_block_sym_f32(s, L, X, gw);
        else if (L.prec == PHMG_PREC_BF16) launch_block_sym_bf16(s, L, X, gw);
        else launch_block_sym_f64(s, L, X, gw);
        return;
    }
    // symmetric levels with patches above 14 strips keep a general copy for the block path
    const void* factors = L.sym ? L.bfactors : L.factors;
    const int64_t* off = L.sym ? L.bfoff : L.fofflp;
    const int v = L.block_variant;
    if (L.prec == PHMG_PREC_F32) {
        switch (v) {
            case 1: launch_block_shape<float, float, 2, 2, 2>(s, L, factors, off, X, gw); break;
            case 2: launch_block_shape<float, float, 2, 1, 8>(s, L, factors, off, X, gw); break;
            case 3: launch_block_shape<float, float, 2, 2, 4>(s, L, factors, off, X, gw); break;
            default: launch_block_shape<float, float, 2, 1, 4>(s, L, factors, off, X, gw);
        }
    } else if (L.prec == PHMG_PREC_BF16) {
        switch (v) {
            case 1: launch_block_shape<__hip_bfloat16, float, 4, 1, 2>(s, L, factors, off, X, gw); break;
            case 2: launch_block_shape<__hip_bfloat16, float, 4, 1, 8>(s, L, factors, off, X, gw); break;
            case 3: launch_block_shape<__hip_bfloat16, float, 4, 2, 2>(s, L, factors, off, X, gw); break;
            default: launch_block_shape<__hip_bfloat16, float, 4, 1, 4>(s, L, factors, off, X, gw);
        }
    } else {
        switch (v) {
            case 1: launch_block_shape<double, double, 1, 2, 4>(s, L, factors, off, X, gw); break;
            case 2: launch_block_shape<double, double, 1, 1, 8>(s, L, factors, off, X, gw); break;
            case 3: launch_block_shape<double, double, 1, 4, 2>(s, L, factors, off, X, gw); break;
            default: launch_block_shape<double, double, 1, 1, 4>(s, L, factors, off, X, gw);
        }
    }
}

void launch_block_scatter(hipStream_t s, const Level& L, double a, double c, double* d, bool store_d, double* X,
                          bool x_zero, bool transpose) {
    if (L.n <= 0) return;
    const int flags = (x_zero ? 1 : 0) | (c != 0.0 ? 2 : 0) | (store_d ? 4 : 0);
    const double* w = transpose || L.wdof ? nullptr : L.pweight;
    const double* wd = transpose ? nullptr : L.wdof;
    hipLaunchKernelGGL(block_scatter_kernel, dim3(grid_for((int64_t)L.n * kBS, kBlock)), dim3(kBlock), 0, s, L.n,
                       L.sptr, L.sslot, w, wd, L.Yb, a, c, d, X, flags);
}

void launch_block_coarse_solve(hipStream_t s, const Level& L, const double* B, double* X, bool transpose) {
    // transposed: the column-major inverse read row by row is the transposed inverse
    hipLaunchKernelGGL(block_coarse_solve_kernel, dim3(grid_for((int64_t)L.n * kWave, kBlock)), dim3(kBlock), 0, s,
                       L.n, L.nb, transpose ? L.cdense : L.cinv, B, X);
}

void launch_block_gs(hipStream_t s, int mode, int64_t n, int ncol, const double* V, int64_t ldv, double* w,
                     const double* h, double* partial, double* out) {
    const int nout = mode == 2 ? 1 : ncol;
    if (mode == 0)
        hipLaunchKernelGGL(block_gs_kernel<0>, dim3(kBlockGsBlocks), dim3(kBlock), 0, s, n, ncol, V, ldv, w, h, partial);
    else if (mode == 1)
        hipLaunchKernelGGL(block_gs_kernel<1>, dim3(kBlockGsBlocks), dim3(kBlock), 0, s, n, ncol, V, ldv, w, h, partial);
    else
        hipLaunchKernelGGL(block_gs_kernel<2>, dim3(kBlockGsBlocks), dim3(kBlock), 0, s, n, ncol, V, ldv, w, h, partial);
    hipLaunchKernelGGL(block_reduce_kernel, dim3(nout * kBS), dim3(kBlock), 0, s, kBlockGsBlocks, partial, out);
}

int block_gs_max_basis() { return kMaxBasis; }

void launch_block_gemv_add(hipStream_t s, int64_t n, int ncol, const double* Z, int64_t ldz, const double* y,
                           double* X) {
    hipLaunchKernelGGL(block_gemv_add_kernel, dim3(std::min(grid_for(n * kBS, kBlock), 8192)), dim3(kBlock), 0, s, n,
                       ncol, Z, ldz, y, X);
}

void launch_block_scale(hipStream_t s, int64_t n, const double* S, const double* cs, double* D) {
    hipLaunchKernelGGL(block_scale_kernel, dim3(std::min(grid_for(n * kBS, kBlock), 8192)), dim3(kBlock), 0, s, n, S,
                       cs, D);
}

void launch_interleave(hipStream_t s, int64_t n, int nrhs, const double* src, double* dst) {
    hipLaunchKernelGGL(interleave_kernel, dim3(std::min(grid_for(n * kBS, kBlock), 8192)), dim3(kBlock), 0, s, n,
                       nrhs, src, dst);
}

void launch_deinterleave(hipStream_t s, int64_t n, int nrhs, const double* src, double* dst) {
    if (nrhs <= 0 || n <= 0) return;
    hipLaunchKernelGGL(deinterleave_kernel, dim3(std::min(grid_for(n * nrhs, kBlock), 8192)), dim3(kBlock), 0, s, n,
                       nrhs, src, dst);
}

}  // namespace phmg
