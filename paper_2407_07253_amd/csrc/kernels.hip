// gfx950 kernels of the Vanka-star / phMG / FGMRES hot path.
//
//  * spmv_kernel       residual r = b - K x and the transfer products (Section 3.1, 3.4)
//  * extract_kernel    K_i = K[S_i, S_i] for every patch (Section 3.4)
//  * gj_kernel         in-place inversion of every patch matrix by blocked
//                      Gauss-Jordan elimination with partial pivoting; the
//                      rank-16 updates run on MFMA f64 16x16x4 tiles
//  * patch_apply       y_i = K_i^{-1} r[S_i] streaming the stored inverses
//  * scatter_kernel    x += omega sum_i R_i^T W_i y_i, DoF-centric, fixed
//                      ascending patch order (eq. "eq:ASM")
//  * coarse kernels    dense bordered coarse matrix, its inverse, solves
//  * FGMRES kernels    deterministic multi-dot products and updates
//
// Every reduction has a fixed shape (no floating-point atomics), so results are
// bitwise reproducible from run to run.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "phmg_internal.h"

namespace phmg {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

inline int grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (1 << 20)) g = 1 << 20;
    return (int)g;
}

__global__ __launch_bounds__(kBlock) void fill_kernel(int64_t n, double* __restrict__ x, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ __launch_bounds__(kBlock) void fill_i32_kernel(int64_t n, int32_t* __restrict__ x, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ __launch_bounds__(kBlock) void copy_kernel(int64_t n, const double* __restrict__ s, double* __restrict__ d) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

// ---------------------------------------------------------------------------
// CSR SpMV, G lanes per row: y = alpha * A x + beta * z  (z may alias y)
// ---------------------------------------------------------------------------
template <int G>
__global__ __launch_bounds__(kBlock) void spmv_kernel(int32_t nrows, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const double* __restrict__ val,
                                                      const double* __restrict__ x, double alpha, const double* z,
                                                      double beta, double* y) {
    const int lane = threadIdx.x & (G - 1);
    const int64_t sub = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
    const int64_t nsub = ((int64_t)gridDim.x * blockDim.x) / G;
    for (int64_t row = sub; row < nrows; row += nsub) {
        const int beg = rowptr[row], end = rowptr[row + 1];
        double s = 0.0;
        for (int k = beg + lane; k < end; k += G) s += val[k] * x[col[k]];
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
        if (lane == 0) {
            double out = alpha * s;
            if (z) out += beta * z[row];
            y[row] = out;
        }
    }
}

// ---------------------------------------------------------------------------
// Patch extraction: one workgroup per patch; column-major m x m output.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void extract_kernel(const int64_t* __restrict__ pptr,
                                                         const int32_t* __restrict__ pdofs,
                                                         const int64_t* __restrict__ foff,
                                                         const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val, double* __restrict__ out) {
    extern __shared__ int32_t s_dofs[];
    const int p = blockIdx.x;
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    double* A = out + foff[p];
    for (int t = threadIdx.x; t < m; t += blockDim.x) s_dofs[t] = pdofs[base + t];
    const int64_t mm = (int64_t)m * m;
    for (int64_t e = threadIdx.x; e < mm; e += blockDim.x) A[e] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int a = wave; a < m; a += kBlock / kWave) {
        const int g = s_dofs[a];
        const int end = rowptr[g + 1];
        for (int k = rowptr[g] + lane; k < end; k += kWave) {
            const int c = col[k];
            int lo = 0, hi = m;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_dofs[mid] < c) lo = mid + 1; else hi = mid;
            }
            if (lo < m && s_dofs[lo] == c) A[a + (int64_t)lo * m] = val[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan inversion with partial pivoting, in place, one
// workgroup per matrix.  Column-major m x m at F + foff[p].
//
// Panels of 16 columns are eliminated in LDS (pivot = largest |entry| on or
// below the diagonal of the current column, ties to the lowest row, exactly
// the pivot sequence of LU with partial pivoting).  The panel's row swaps are
// then applied to the other columns and those columns receive the rank-16
// update  A[:, R] += (Q - E) A_old[k0:k0+16, R]  on MFMA f64 16x16x4 tiles,
// where Q is the eliminated panel and E the identity rows of the panel.  The
// pivoting is undone at the end by column swaps in reverse order.
//
// MFMA f64 16x16x4 lane layout (lane l, accumulator element v):
//   A operand A[l % 16][l / 16], B operand B[l / 16][l % 16],
//   C/D element D[l / 16 + 4 v][l % 16].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void gj_kernel(const int64_t* __restrict__ pptr,
                                                    const int64_t* __restrict__ foff,
                                                    const int32_t* __restrict__ order, double* __restrict__ F,
                                                    int ldq, int* __restrict__ status) {
    extern __shared__ double smem[];
    double* Q = smem;                        // ldq x kPanel, column-major
    double* fcol = Q + (int64_t)ldq * kPanel;  // ldq
    int* piv = (int*)(fcol + ldq);           // ldq
    __shared__ double s_val[kBlock / kWave];
    __shared__ int s_idx[kBlock / kWave];
    __shared__ double s_tol;
    __shared__ int s_fail;

    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int p = order ? order[blockIdx.x] : (int)blockIdx.x;
    const int m = (int)(pptr[p + 1] - pptr[p]);
    double* A = F + foff[p];

    // ||A||_inf = max_i sum_j |A_ij|
    double rs = 0.0;
    for (int i = tid; i < m; i += kBlock) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += fabs(A[i + (int64_t)j * m]);
        rs = fmax(rs, s);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) rs = fmax(rs, __shfl_xor(rs, off));
    if (lane == 0) s_val[wave] = rs;
    __syncthreads();
    if (tid == 0) {
        double mx = 0.0;
        for (int q = 0; q < kBlock / kWave; ++q) mx = fmax(mx, s_val[q]);
        s_tol = 1e-14 * mx;
        s_fail = 0;
    }
    __syncthreads();
    const double tol = s_tol;

    for (int k0 = 0; k0 < m; k0 += kPanel) {
        const int w = min(kPanel, m - k0);
        for (int e = tid; e < m * w; e += kBlock) {
            const int i = e % m, c = e / m;
            Q[i + c * ldq] = A[i + (int64_t)(k0 + c) * m];
        }
        __syncthreads();
        for (int c = 0; c < w; ++c) {
            const int k = k0 + c;
            double bv = -1.0;
            int bi = INT_MAX;
            for (int i = k + tid; i < m; i += kBlock) {
                const double v = fabs(Q[i + c * ldq]);
                if (v > bv) { bv = v; bi = i; }
            }
            for (int off = kWave / 2; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int oi = __shfl_xor(bi, off);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if (lane == 0) { s_val[wave] = bv; s_idx[wave] = bi; }
            __syncthreads();
            if (tid == 0) {
                for (int q = 1; q < kBlock / kWave; ++q) {
                    if (s_val[q] > bv || (s_val[q] == bv && s_idx[q] < bi)) { bv = s_val[q]; bi = s_idx[q]; }
                }
                if (bi >= m || !(bv > tol)) s_fail = 1;
                piv[k] = bi < m ? bi : k;
            }
            __syncthreads();
            if (s_fail) {
                if (tid == 0) atomicMin(status, p);
                return;
            }
            const int pr = piv[k];
            if (pr != k && tid < w) {
                const double t = Q[k + tid * ldq];
                Q[k + tid * ldq] = Q[pr + tid * ldq];
                Q[pr + tid * ldq] = t;
            }
            __syncthreads();
            const double d = 1.0 / Q[k + c * ldq];
            for (int i = tid; i < m; i += kBlock) fcol[i] = Q[i + c * ldq];
            __syncthreads();
            if (tid < w) Q[k + tid * ldq] = (tid == c) ? d : Q[k + tid * ldq] * d;
            __syncthreads();
            for (int e = tid; e < m * w; e += kBlock) {
                const int i = e % m, cc = e / m;
                if (i == k) continue;
                const double f = fcol[i];
                if (cc == c) Q[i + c * ldq] = -f * d;
                else Q[i + cc * ldq] -= f * Q[k + cc * ldq];
            }
            __syncthreads();
        }
        // row swaps of this panel in every other column
        for (int j = tid; j < m; j += kBlock) {
            if (j >= k0 && j < k0 + w) continue;
            double* cj = A + (int64_t)j * m;
            for (int c = 0; c < w; ++c) {
                const int pr = piv[k0 + c];
                if (pr != k0 + c) {
                    const double t = cj[k0 + c];
                    cj[k0 + c] = cj[pr];
                    cj[pr] = t;
                }
            }
        }
        __syncthreads();
        // rank-w update of the other columns on MFMA f64 16x16x4
        {
            const int nb16 = (m + 15) / 16;
            const int li = lane & 15, lk = lane >> 4;
            for (int jb = wave; jb < nb16; jb += kBlock / kWave) {
                const int j = jb * 16 + li;
                const bool jv = (j < m) && (j < k0 || j >= k0 + w);
                double bop[4];
#pragma unroll
                for (int kt = 0; kt < 4; ++kt) {
                    const int kk = kt * 4 + lk;
                    bop[kt] = (jv && kk < w) ? A[(k0 + kk) + (int64_t)j * m] : 0.0;
                }
                for (int ib = 0; ib < nb16; ++ib) {
                    d4 acc;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = ib * 16 + lk + 4 * v;
                        acc[v] = (jv && i < m) ? A[i + (int64_t)j * m] : 0.0;
                    }
#pragma unroll
                    for (int kt = 0; kt < 4; ++kt) {
                        const int i = ib * 16 + li, kk = kt * 4 + lk;
                        double aop = 0.0;
                        if (i < m && kk < w) {
                            aop = Q[i + kk * ldq];
                            if (i == k0 + kk) aop -= 1.0;
                        }
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[kt], acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = ib * 16 + lk + 4 * v;
                        if (jv && i < m) A[i + (int64_t)j * m] = acc[v];
                    }
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < m * w; e += kBlock) {
            const int i = e % m, c = e / m;
            A[i + (int64_t)(k0 + c) * m] = Q[i + c * ldq];
        }
        __syncthreads();
    }
    for (int k = m - 1; k >= 0; --k) {
        const int pr = piv[k];
        if (pr != k) {
            for (int i = tid; i < m; i += kBlock) {
                const double t = A[i + (int64_t)k * m];
                A[i + (int64_t)k * m] = A[i + (int64_t)pr * m];
                A[i + (int64_t)pr * m] = t;
            }
        }
        __syncthreads();
    }
}

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

// f64 set-up result (column-major, ld = m) -> reduced-precision factors with
// ld = m rounded up to V (padding rows are zero); one workgroup per patch.
template <typename T, int V>
__global__ __launch_bounds__(kBlock) void convert_patch_kernel(const int64_t* __restrict__ pptr,
                                                               const int64_t* __restrict__ foff64,
                                                               const int64_t* __restrict__ fofflp,
                                                               const double* __restrict__ src, T* __restrict__ dst) {
    const int p = blockIdx.x;
    const int m = (int)(pptr[p + 1] - pptr[p]);
    const int ld = (m + V - 1) / V * V;
    const double* a = src + foff64[p];
    T* b = dst + fofflp[p];
    const int64_t total = (int64_t)ld * m;
    for (int64_t e = threadIdx.x; e < total; e += kBlock) {
        const int i = (int)(e % ld), j = (int)(e / ld);
        const double v = i < m ? a[i + (int64_t)j * m] : 0.0;
        if constexpr (sizeof(T) == 4) b[e] = (T)v;
        else b[e] = __float2bfloat16((float)v);
    }
}

// ---------------------------------------------------------------------------
// Dense Gauss-Jordan inversion of one large matrix (the coarsest level) over
// the whole GPU: per panel of w columns, gj_panel_kernel (one workgroup,
// panel in LDS) eliminates the panel with partial pivoting and writes it
// back with its pivots; gj_update_kernel (one wavefront per 16-column block)
// applies the panel's row swaps to its columns and the rank-w update on MFMA
// f64 16x16x4 tiles.  gj_unscramble_kernel undoes the pivoting (column swaps
// in reverse order), one thread per row.  Column-major N x N.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void gj_panel_kernel(double* __restrict__ A, int N, int k0, int w,
                                                          int* __restrict__ piv, int* __restrict__ status,
                                                          const double* __restrict__ tolp) {
    extern __shared__ double smem[];
    double* Q = smem;               // N x w
    double* fcol = Q + (int64_t)N * w;
    __shared__ double s_val[kBlock / kWave];
    __shared__ int s_idx[kBlock / kWave];
    __shared__ int s_fail;
    __shared__ int s_piv[kPanel];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const double tol = tolp[0];
    if (status[0] != INT32_MAX) return;            // an earlier panel failed
    for (int e = tid; e < N * w; e += kBlock) {
        const int i = e % N, c = e / N;
        Q[i + (int64_t)c * N] = A[i + (int64_t)(k0 + c) * N];
    }
    if (tid == 0) s_fail = 0;
    __syncthreads();
    for (int c = 0; c < w; ++c) {
        const int k = k0 + c;
        double bv = -1.0;
        int bi = INT_MAX;
        for (int i = k + tid; i < N; i += kBlock) {
            const double v = fabs(Q[i + (int64_t)c * N]);
            if (v > bv) { bv = v; bi = i; }
        }
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off);
            const int oi = __shfl_xor(bi, off);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { s_val[wave] = bv; s_idx[wave] = bi; }
        __syncthreads();
        if (tid == 0) {
            for (int q = 1; q < kBlock / kWave; ++q)
                if (s_val[q] > bv || (s_val[q] == bv && s_idx[q] < bi)) { bv = s_val[q]; bi = s_idx[q]; }
            if (bi >= N || !(bv > tol)) s_fail = 1;
            s_piv[c] = bi < N ? bi : k;
        }
        __syncthreads();
        if (s_fail) {
            if (tid == 0) atomicMin(status, 0);
            return;
        }
        const int pr = s_piv[c];
        if (pr != k && tid < w) {
            const double t = Q[k + (int64_t)tid * N];
            Q[k + (int64_t)tid * N] = Q[pr + (int64_t)tid * N];
            Q[pr + (int64_t)tid * N] = t;
        }
        __syncthreads();
        const double d = 1.0 / Q[k + (int64_t)c * N];
        for (int i = tid; i < N; i += kBlock) fcol[i] = Q[i + (int64_t)c * N];
        __syncthreads();
        if (tid < w) Q[k + (int64_t)tid * N] = (tid == c) ? d : Q[k + (int64_t)tid * N] * d;
        __syncthreads();
        for (int e = tid; e < N * w; e += kBlock) {
            const int i = e % N, cc = e / N;
            if (i == k) continue;
            const double f = fcol[i];
            if (cc == c) Q[i + (int64_t)c * N] = -f * d;
            else Q[i + (int64_t)cc * N] -= f * Q[k + (int64_t)cc * N];
        }
        __syncthreads();
    }
    for (int e = tid; e < N * w; e += kBlock) {
        const int i = e % N, c = e / N;
        A[i + (int64_t)(k0 + c) * N] = Q[i + (int64_t)c * N];
    }
    if (tid < w) piv[k0 + tid] = s_piv[tid];
}

// one wavefront per 16-column block outside the panel
__global__ __launch_bounds__(kBlock) void gj_update_kernel(double* __restrict__ A, int N, int k0, int w,
                                                           const int* __restrict__ piv,
                                                           const int* __restrict__ status) {
    if (status[0] != INT32_MAX) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int jb = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int nb16 = (N + 15) / 16;
    if (jb >= nb16) return;
    const int li = lane & 15, lk = lane >> 4;
    const int j = jb * 16 + li;
    const bool jv = (j < N) && (j < k0 || j >= k0 + w);
    if (jv) {
        double* cj = A + (int64_t)j * N;
        for (int c = 0; c < w; ++c) {
            const int pr = piv[k0 + c];
            if (pr != k0 + c && lk == 0) {
                const double t = cj[k0 + c];
                cj[k0 + c] = cj[pr];
                cj[pr] = t;
            }
        }
    }
    // the swaps (lane lk == 0 of each column) must be visible to the other lanes of the wave
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    __threadfence_block();
    double bop[4];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
        const int kk = kt * 4 + lk;
        bop[kt] = (jv && kk < w) ? A[(k0 + kk) + (int64_t)j * N] : 0.0;
    }
    const bool any = __any(jv ? 1 : 0);
    if (!any) return;
    for (int ib = 0; ib < nb16; ++ib) {
        d4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = ib * 16 + lk + 4 * v;
            acc[v] = (jv && i < N) ? A[i + (int64_t)j * N] : 0.0;
        }
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            const int i = ib * 16 + li, kk = kt * 4 + lk;
            double aop = 0.0;
            if (i < N && kk < w) {
                aop = A[i + (int64_t)(k0 + kk) * N];
                if (i == k0 + kk) aop -= 1.0;
            }
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[kt], acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = ib * 16 + lk + 4 * v;
            if (jv && i < N) A[i + (int64_t)j * N] = acc[v];
        }
    }
}

__global__ __launch_bounds__(kBlock) void gj_unscramble_kernel(double* __restrict__ A, int N,
                                                               const int* __restrict__ piv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int k = N - 1; k >= 0; --k) {
        const int pr = piv[k];
        if (pr != k) {
            const double t = A[i + (int64_t)k * N];
            A[i + (int64_t)k * N] = A[i + (int64_t)pr * N];
            A[i + (int64_t)pr * N] = t;
        }
    }
}

// tol = 1e-14 * max_i sum_j |A_ij| (column-major N x N), one block
__global__ __launch_bounds__(kBlock) void inf_norm_tol_kernel(const double* __restrict__ A, int N,
                                                              double* __restrict__ tol) {
    __shared__ double sh[kBlock / kWave];
    double rs = 0.0;
    for (int i = threadIdx.x; i < N; i += kBlock) {
        double s = 0.0;
        for (int j = 0; j < N; ++j) s += fabs(A[i + (int64_t)j * N]);
        rs = fmax(rs, s);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) rs = fmax(rs, __shfl_xor(rs, off));
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = rs;
    __syncthreads();
    if (threadIdx.x == 0) tol[0] = 1e-14 * fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// s_j = sum_{slots t of DoF j, ascending patch id} w_t Y[t];  dn = a s_j + c d_j;
// x_j = (x_zero ? 0 : x_j) + dn;  d_j = dn when storing (Chebyshev direction).
// Richardson is a = omega, c = 0.
__global__ __launch_bounds__(kBlock) void scatter_kernel(int32_t n, const int32_t* __restrict__ sptr,
                                                         const int32_t* __restrict__ sslot,
                                                         const double* __restrict__ w, const double* __restrict__ Y,
                                                         double a, double c, double* __restrict__ d,
                                                         double* __restrict__ x, int flags) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    const int end = sptr[j + 1];
    if (w) {
        for (int t = sptr[j]; t < end; ++t) {
            const int q = sslot[t];
            s += w[q] * Y[q];
        }
    } else {
        for (int t = sptr[j]; t < end; ++t) s += Y[sslot[t]];
    }
    double dn = a * s;
    if (flags & 2) dn = c * d[j] + dn;
    x[j] = (flags & 1) ? dn : x[j] + dn;
    if (flags & 4) d[j] = dn;
}

__global__ __launch_bounds__(kBlock) void power_start_kernel(int64_t n, double* __restrict__ v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = 1.0 + 0.5 * sin((double)i);
}

__global__ __launch_bounds__(kBlock) void scale_by_devnorm_kernel(int64_t n, const double* __restrict__ s,
                                                                  const double* __restrict__ norm2,
                                                                  double* __restrict__ d) {
    const double q = sqrt(norm2[0]);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i] / q;
}

// ---------------------------------------------------------------------------
// Coarse level
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void coarse_build_kernel(int32_t n, int32_t nb, const int32_t* __restrict__ rowptr,
                                                              const int32_t* __restrict__ col,
                                                              const double* __restrict__ val,
                                                              const double* __restrict__ z, double* __restrict__ D) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) D[i + (int64_t)col[k] * nb] = val[k];
    if (nb > n) {
        D[i + (int64_t)n * nb] = z[i];
        D[n + (int64_t)i * nb] = z[i];
    }
}

__global__ __launch_bounds__(kBlock) void transpose_kernel(int32_t n, const double* __restrict__ s,
                                                           double* __restrict__ d) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int i = (int)(e / n), j = (int)(e % n);
    d[e] = s[i + (int64_t)j * n];       // d row-major (i, j) = s column-major (i, j)
}

// x[i] = sum_{j < n} Ainv_rm[i * nb + j] b[j]   (one wavefront per row)
__global__ __launch_bounds__(kBlock) void coarse_solve_kernel(int32_t n, int32_t nb, const double* __restrict__ Ainv,
                                                              const double* __restrict__ b, double* __restrict__ x) {
    const int lane = threadIdx.x & (kWave - 1);
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (row >= n) return;
    const double* a = Ainv + (int64_t)row * nb;
    double s = 0.0;
    for (int j = lane; j < n; j += kWave) s += a[j] * b[j];
    for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) x[row] = s;
}

// ---------------------------------------------------------------------------
// FGMRES helpers (fixed reduction shapes)
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double* sh) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(kBlock) void multidot_partial_kernel(int64_t n, int ncol, const double* __restrict__ V,
                                                                  int64_t ldv, const double* __restrict__ w,
                                                                  double* __restrict__ partial) {
    __shared__ double sh[kBlock / kWave];
    for (int c = 0; c < ncol; ++c) {
        const double* v = V + (int64_t)c * ldv;
        double s = 0.0;
        for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
            s += v[i] * w[i];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) partial[(int64_t)c * gridDim.x + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kBlock) void reduce_cols_kernel(int nparts, const double* __restrict__ partial,
                                                             double* __restrict__ out) {
    __shared__ double sh[kBlock / kWave];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int q = threadIdx.x; q < nparts; q += kBlock) s += partial[(int64_t)c * nparts + q];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[c] = s;
}

__global__ __launch_bounds__(kBlock) void gemv_sub_kernel(int64_t n, int ncol, const double* __restrict__ V,
                                                          int64_t ldv, const double* __restrict__ h,
                                                          double* __restrict__ w) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < ncol; ++c) s += V[i + (int64_t)c * ldv] * h[c];
        w[i] -= s;
    }
}

__global__ __launch_bounds__(kBlock) void gemv_add_kernel(int64_t n, int ncol, const double* __restrict__ Z,
                                                          int64_t ldz, const double* __restrict__ y,
                                                          double* __restrict__ x) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < ncol; ++c) s += Z[i + (int64_t)c * ldz] * y[c];
        x[i] += s;
    }
}

__global__ __launch_bounds__(kBlock) void scale_copy_kernel(int64_t n, const double* __restrict__ s, double q,
                                                            double* __restrict__ d) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i] / q;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_fill(hipStream_t s, int64_t n, double* x, double v) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, x, v);
}

void launch_fill_i32(hipStream_t s, int64_t n, int32_t* x, int32_t v) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, x, v);
}

void launch_copy(hipStream_t s, int64_t n, const double* src, double* dst) {
    if (n <= 0) return;
    hipLaunchKernelGGL(copy_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, src, dst);
}

void launch_spmv(hipStream_t s, const DevCsr& A, const double* x, double alpha, const double* z, double beta,
                 double* y) {
    if (A.nrows <= 0) return;
    const int grid = grid_for((int64_t)A.nrows * A.group, kBlock);
    switch (A.group) {
#define PHMG_SPMV_CASE(G)                                                                                      \
    case G:                                                                                                    \
        hipLaunchKernelGGL(spmv_kernel<G>, dim3(grid), dim3(kBlock), 0, s, A.nrows, A.rowptr, A.col, A.val, x, \
                           alpha, z, beta, y);                                                                 \
        break;
        PHMG_SPMV_CASE(2)
        PHMG_SPMV_CASE(4)
        PHMG_SPMV_CASE(8)
        PHMG_SPMV_CASE(16)
        PHMG_SPMV_CASE(32)
        PHMG_SPMV_CASE(64)
#undef PHMG_SPMV_CASE
        default:
            hipLaunchKernelGGL(spmv_kernel<8>, dim3(grid_for((int64_t)A.nrows * 8, kBlock)), dim3(kBlock), 0, s,
                               A.nrows, A.rowptr, A.col, A.val, x, alpha, z, beta, y);
    }
}

void launch_extract(hipStream_t s, const Level& L, double* out) {
    if (L.npatch <= 0) return;
    hipLaunchKernelGGL(extract_kernel, dim3(L.npatch), dim3(kBlock), sizeof(int32_t) * L.max_m, s, L.pptr, L.pdofs,
                       L.foff, L.K.rowptr, L.K.col, L.K.val, out);
}

size_t gj_lds_bytes(int ldq) { return sizeof(double) * ((size_t)ldq * kPanel + ldq) + sizeof(int) * ldq; }

void launch_gj_invert(hipStream_t s, int npatch, const int64_t* pptr, const int64_t* foff, const int32_t* order,
                      double* A, int max_m, int* status) {
    if (npatch <= 0) return;
    const size_t lds = gj_lds_bytes(max_m);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)gj_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(gj_kernel, dim3(npatch), dim3(kBlock), lds, s, pptr, foff, order, A, max_m, status);
}

// Kernel shapes the set-up autotuner chooses from, per precision:
// (row tiles held per pass NRT, columns in flight per wave U).
namespace {
template <typename T, typename Acc, int V, int NRT, int U>
void launch_apply_shape(hipStream_t s, const Level& L, const int64_t* off, const double* r) {
    hipLaunchKernelGGL((patch_apply_kernel<T, Acc, V, NRT, U>), dim3(L.npatch), dim3(kBlock), sizeof(Acc) * L.max_m, s,
                       L.order, L.pptr, L.pdofs, off, (const T*)L.factors, r, L.Y);
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

void launch_convert_patches(hipStream_t s, const Level& L, const double* src, void* dst) {
    if (L.npatch <= 0) return;
    if (L.prec == PHMG_PREC_F32)
        hipLaunchKernelGGL((convert_patch_kernel<float, 2>), dim3(L.npatch), dim3(kBlock), 0, s, L.pptr, L.foff,
                           L.fofflp, src, (float*)dst);
    else if (L.prec == PHMG_PREC_BF16)
        hipLaunchKernelGGL((convert_patch_kernel<__hip_bfloat16, 4>), dim3(L.npatch), dim3(kBlock), 0, s, L.pptr,
                           L.foff, L.fofflp, src, (__hip_bfloat16*)dst);
}

void launch_scatter(hipStream_t s, const Level& L, double a, double c, double* d, bool store_d, double* x,
                    bool x_zero) {
    if (L.n <= 0) return;
    const int flags = (x_zero ? 1 : 0) | (c != 0.0 ? 2 : 0) | (store_d ? 4 : 0);
    hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(L.n, kBlock)), dim3(kBlock), 0, s, L.n, L.sptr, L.sslot,
                       L.pweight, L.Y, a, c, d, x, flags);
}

void launch_power_start(hipStream_t s, int64_t n, double* v) {
    hipLaunchKernelGGL(power_start_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, v);
}

void launch_scale_by_devnorm(hipStream_t s, int64_t n, const double* src, const double* norm2, double* dst) {
    hipLaunchKernelGGL(scale_by_devnorm_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n,
                       src, norm2, dst);
}

int coarse_panel_width(int N) {
    // the panel (N x w doubles) and one column must fit in LDS (<= 150 KiB)
    for (int w = kPanel; w >= 1; w /= 2)
        if ((size_t)N * (w + 1) * sizeof(double) <= 150 * 1024) return w;
    return 0;
}

void launch_dense_gj(hipStream_t s, double* A, int N, int* piv, int* status, double* tol) {
    const int w0 = coarse_panel_width(N);
    hipLaunchKernelGGL(inf_norm_tol_kernel, dim3(1), dim3(kBlock), 0, s, A, N, tol);
    const size_t lds = (size_t)N * (w0 + 1) * sizeof(double);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)gj_panel_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int nb16 = (N + 15) / 16;
    const int grid_upd = (nb16 * kWave + kBlock - 1) / kBlock;
    for (int k0 = 0; k0 < N; k0 += w0) {
        const int w = std::min(w0, N - k0);
        hipLaunchKernelGGL(gj_panel_kernel, dim3(1), dim3(kBlock), lds, s, A, N, k0, w, piv, status, tol);
        hipLaunchKernelGGL(gj_update_kernel, dim3(grid_upd), dim3(kBlock), 0, s, A, N, k0, w, piv, status);
    }
    hipLaunchKernelGGL(gj_unscramble_kernel, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, s, A, N, piv);
}

void launch_coarse_build(hipStream_t s, const Level& L, double* dense) {
    launch_fill(s, (int64_t)L.nb * L.nb, dense, 0.0);
    hipLaunchKernelGGL(coarse_build_kernel, dim3(grid_for(L.n, kBlock)), dim3(kBlock), 0, s, L.n, L.nb, L.K.rowptr,
                       L.K.col, L.K.val, L.cnull, dense);
}

void launch_transpose(hipStream_t s, int n, const double* src, double* dst) {
    hipLaunchKernelGGL(transpose_kernel, dim3(grid_for((int64_t)n * n, kBlock)), dim3(kBlock), 0, s, n, src, dst);
}

void launch_coarse_solve(hipStream_t s, const Level& L, const double* b, double* x) {
    hipLaunchKernelGGL(coarse_solve_kernel, dim3(grid_for((int64_t)L.n * kWave, kBlock)), dim3(kBlock), 0, s, L.n,
                       L.nb, L.cinv, b, x);
}

void launch_multidot(hipStream_t s, int64_t n, int ncol, const double* V, int64_t ldv, const double* w,
                     double* partial, double* out, bool /*accumulate*/) {
    hipLaunchKernelGGL(multidot_partial_kernel, dim3(kRedBlocks), dim3(kBlock), 0, s, n, ncol, V, ldv, w, partial);
    hipLaunchKernelGGL(reduce_cols_kernel, dim3(ncol), dim3(kBlock), 0, s, kRedBlocks, partial, out);
}

void launch_gemv_sub(hipStream_t s, int64_t n, int ncol, const double* V, int64_t ldv, const double* h, double* w) {
    hipLaunchKernelGGL(gemv_sub_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, ncol, V,
                       ldv, h, w);
}

void launch_gemv_add(hipStream_t s, int64_t n, int ncol, const double* Z, int64_t ldz, const double* y, double* x) {
    hipLaunchKernelGGL(gemv_add_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, ncol, Z,
                       ldz, y, x);
}

void launch_scale_copy(hipStream_t s, int64_t n, const double* src, double denom, double* dst) {
    hipLaunchKernelGGL(scale_copy_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, src,
                       denom, dst);
}

}  // namespace phmg
