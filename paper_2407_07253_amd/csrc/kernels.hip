// gfx950 kernels of the Vanka-star / phMG / FGMRES hot path.
//
//  * spmv_kernel       residual r = b - K x and the transfer products (Section 3.1, 3.4)
//  * extract_kernel    K_i = K[S_i, S_i] for every patch (Section 3.4)
//  * gj_kernel         in-place inversion of every patch matrix by blocked
//                      Gauss-Jordan elimination with partial pivoting; the
//                      rank-16 updates run on MFMA f64 16x16x4 tiles
//                      (gj_wide_kernel: 24-column panels for 257-384 DoFs)
//  * patch_apply       y_i = K_i^{-1} r[S_i]: in patch_apply.hip
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
// CSR SpMV, G lanes per row: y = alpha * A x + beta * z  (z may alias y).
// With XM the workgroups are renumbered so that each of the 8 XCDs (which
// receive workgroups round-robin) sweeps one contiguous eighth of the rows:
// neighbouring rows gather neighbouring x entries, so the gathers of one XCD
// stay in its own L2.  The grid is a multiple of 8 in that case.
// ---------------------------------------------------------------------------
__device__ inline int64_t logical_block(bool xm) {
    if (!xm) return blockIdx.x;
    const int64_t per = gridDim.x / 8;
    return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

template <int G, bool XM, int UNR = 4>
__global__ __launch_bounds__(kBlock) void spmv_kernel(int32_t nrows, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const double* __restrict__ val,
                                                      const double* __restrict__ x, double alpha, const double* z,
                                                      double beta, double* y) {
    const int lane = threadIdx.x & (G - 1);
    const int64_t sub = (logical_block(XM) * blockDim.x + threadIdx.x) / G;
    const int64_t nsub = ((int64_t)gridDim.x * blockDim.x) / G;
    for (int64_t row = sub; row < nrows; row += nsub) {
        const int beg = rowptr[row], end = rowptr[row + 1];
        double s = 0.0;
        // UNR entries per lane in flight (all indices first, then all gathers,
        // predicated at the row end); each lane still adds its entries
        // k = beg + lane, + G, + 2G, ... in order (a missing entry adds +0)
        for (int k = beg + lane; k < end; k += UNR * G) {
            int c[UNR];
            double v[UNR], xv[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const bool ok = k + u * G < end;
                c[u] = ok ? col[k + u * G] : 0;
                v[u] = ok ? val[k + u * G] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) xv[u] = k + u * G < end ? x[c[u]] : 0.0;
#pragma unroll
            for (int u = 0; u < UNR; ++u) s += v[u] * xv[u];
        }
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
// CSR SpMV with G lanes per row and 4 consecutive entries per lane: the row's
// range is widened down to a multiple of 4, so lane l's entries k0 + 4 (l + G j)
// .. + 3 come in one 16-byte index load and two 16-byte value loads (the
// arrays carry 4 padding entries; entries outside the row add +0).  Each lane
// adds its entries in order, then the G partial sums are combined.
// ---------------------------------------------------------------------------
template <int G>
__global__ __launch_bounds__(kBlock) void spmv_vec_kernel(int32_t nrows, const int32_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ col,
                                                          const double* __restrict__ val,
                                                          const double* __restrict__ x, double alpha, const double* z,
                                                          double beta, double* y) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const int lane = threadIdx.x & (G - 1);
    const int64_t sub = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t nsub = ((int64_t)gridDim.x * blockDim.x) / G;
    for (int64_t row = sub; row < nrows; row += nsub) {
        const int beg = rowptr[row], end = rowptr[row + 1];
        double s = 0.0;
        for (int k = (beg & ~3) + 4 * lane; k < end; k += 4 * G) {
            const i4 c = *reinterpret_cast<const i4*>(col + k);
            const dv2 va = *reinterpret_cast<const dv2*>(val + k);
            const dv2 vb = *reinterpret_cast<const dv2*>(val + k + 2);
            const double v[4] = {va.x, va.y, vb.x, vb.y};
            double xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = k + u >= beg && k + u < end ? x[c[u]] : 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u) s += (k + u >= beg && k + u < end ? v[u] : 0.0) * xv[u];
        }
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
// y = A1 x1 - A2 x2 (same rows), G lanes per row: the restricted residual
// R b - (R K) x of the cycle in one pass over the coarse rows.  Each row's two
// sums are formed as in spmv_kernel and subtracted at the end.
// ---------------------------------------------------------------------------
template <int G>
__global__ __launch_bounds__(kBlock) void spmv_diff_kernel(int32_t nrows, const int32_t* __restrict__ rp1,
                                                           const int32_t* __restrict__ c1,
                                                           const double* __restrict__ v1,
                                                           const double* __restrict__ x1,
                                                           const int32_t* __restrict__ rp2,
                                                           const int32_t* __restrict__ c2,
                                                           const double* __restrict__ v2,
                                                           const double* __restrict__ x2, double* __restrict__ y) {
    const int lane = threadIdx.x & (G - 1);
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (row >= nrows) return;
    // the row's entries of both matrices as one index range [0, n1 + n2), so the
    // loads of both are in flight together; lane-strided within each matrix
    const int b1 = rp1[row], n1 = rp1[row + 1] - b1;
    const int b2 = rp2[row], n2 = rp2[row + 1] - b2;
    double s1 = 0.0, s2 = 0.0;
    for (int t = lane; t < n1 + n2; t += 4 * G) {
        int c[4];
        double v[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = t + u * G;
            c[u] = 0;
            v[u] = 0.0;
            if (k < n1) {
                c[u] = c1[b1 + k];
                v[u] = v1[b1 + k];
            } else if (k < n1 + n2) {
                c[u] = c2[b2 + k - n1];
                v[u] = v2[b2 + k - n1];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = t + u * G;
            xv[u] = k < n1 ? x1[c[u]] : (k < n1 + n2 ? x2[c[u]] : 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (t + u * G < n1) s1 += v[u] * xv[u];
            else s2 += v[u] * xv[u];
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off, G);
        s2 += __shfl_xor(s2, off, G);
    }
    if (lane == 0) y[row] = s1 - s2;
}

// ---------------------------------------------------------------------------
// Row-block SpMV: y = alpha * A x + beta * z (z may alias y).  The rows are cut
// at create into blocks of at most kRbRows rows and kRbNnz nonzeros; one
// workgroup per block multiplies all of the block's nonzeros with their x
// entries into LDS (each thread kRbNnz / 256 consecutive-stride entries, all
// loads in flight, col / val read fully coalesced), then 8 lanes per row add
// the row's products (lane-strided, then a fixed xor tree).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void rowblock_spmv_kernel(const int32_t* __restrict__ rblk,
                                                               const int32_t* __restrict__ rowptr,
                                                               const int32_t* __restrict__ col,
                                                               const double* __restrict__ val,
                                                               const double* __restrict__ x, double alpha,
                                                               const double* z, double beta, double* y) {
    constexpr int PER = kRbNnz / kBlock;
    constexpr int G = kBlock / kRbRows;
    __shared__ double s_p[kRbNnz];
    const int r0 = rblk[blockIdx.x], r1 = rblk[blockIdx.x + 1];
    const int k0 = rowptr[r0], nk = rowptr[r1] - k0;
    {
        int c[PER];
        double v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int k = threadIdx.x + u * kBlock;
            c[u] = k < nk ? col[k0 + k] : 0;
            v[u] = k < nk ? val[k0 + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int k = threadIdx.x + u * kBlock;
            if (k < nk) s_p[k] = v[u] * x[c[u]];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x % G, r = r0 + (int)threadIdx.x / G;
    double s = 0.0;
    int beg = 0, end = 0;
    if (r < r1) {
        beg = rowptr[r] - k0;
        end = rowptr[r + 1] - k0;
    }
    for (int k = beg + lane; k < end; k += G) s += s_p[k];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
    if (r < r1 && lane == 0) {
        double out = alpha * s;
        if (z) out += beta * z[r];
        y[r] = out;
    }
}

// ---------------------------------------------------------------------------
// Patch extraction: one workgroup per patch; column-major m x m output.  The
// patch rows are assembled kExtractRows at a time in an LDS tile (row a of the
// patch matrix = row pdofs[a] of K restricted to the patch DoFs, positions
// found by binary search in the sorted DoF list; 16 lanes per row, so the 16
// rows of a tile are searched at once), and each tile is written out column by
// column, kExtractRows consecutive entries of a column per store run: every
// output byte is written once, with no separate zero fill.
// ---------------------------------------------------------------------------
constexpr int kExtractRows = 16;

__global__ __launch_bounds__(kBlock) void extract_kernel(const int64_t* __restrict__ pptr,
                                                         const int32_t* __restrict__ pdofs,
                                                         const int64_t* __restrict__ foff,
                                                         const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val, double* __restrict__ out,
                                                         double* __restrict__ ptol) {
    extern __shared__ double s_tile[];                  // kExtractRows x m (column-major), then m DoF ids
    __shared__ double s_max[kBlock / kWave];
    const int p = blockIdx.x;
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    int32_t* s_dofs = reinterpret_cast<int32_t*>(s_tile + (int64_t)kExtractRows * m);
    double* A = out + foff[p];
    for (int t = threadIdx.x; t < m; t += blockDim.x) s_dofs[t] = pdofs[base + t];
    const int lane = threadIdx.x & (kWave - 1), wave = wave_id();
    double rmax = 0.0;
    for (int a0 = 0; a0 < m; a0 += kExtractRows) {
        const int h = min(kExtractRows, m - a0);
        for (int e = threadIdx.x; e < kExtractRows * m; e += blockDim.x) s_tile[e] = 0.0;
        __syncthreads();
        // 16 lanes per row, four rows per wave: a tile's rows are all in flight at once
        for (int q = 4 * wave + (lane >> 4); q < h; q += 4 * (kBlock / kWave)) {
            const int g = s_dofs[a0 + q];
            const int end = rowptr[g + 1];
            double rsum = 0.0;
            // four entries per lane at a time: their column and value loads are all issued
            // before the searches (same entries, same order of the row sum)
            for (int k0 = rowptr[g] + (lane & 15); k0 < end; k0 += 4 * 16) {
                int cs[4];
                double vs[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = k0 + 16 * u;
                    cs[u] = k < end ? col[k] : -1;
                    vs[u] = k < end ? val[k] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = cs[u];
                    if (c < 0) continue;
                    int lo = 0, hi = m;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (s_dofs[mid] < c) lo = mid + 1; else hi = mid;
                    }
                    if (lo < m && s_dofs[lo] == c) {
                        s_tile[q + kExtractRows * lo] = vs[u];
                        rsum += fabs(vs[u]);
                    }
                }
            }
            for (int off = 8; off > 0; off >>= 1) rsum += __shfl_xor(rsum, off, 16);
            rmax = fmax(rmax, rsum);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kExtractRows * m; e += blockDim.x) {
            const int q = e % kExtractRows, j = e / kExtractRows;
            if (q < h) A[(a0 + q) + (int64_t)j * m] = s_tile[e];
        }
        __syncthreads();
    }
    rmax = fmax(rmax, __shfl_xor(rmax, 16));
    rmax = fmax(rmax, __shfl_xor(rmax, 32));
    if (lane == 0) s_max[wave] = rmax;
    __syncthreads();
    if (threadIdx.x == 0)
        ptol[p] = 1e-14 * fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3]));
}

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan inversion with partial pivoting, in place, one
// workgroup per patch matrix (column-major m x m at F + foff[p]).
//
// Panels of 16 columns are eliminated in LDS.  Pivoting is tracked through
// logical row positions, so no panel row moves: the pivot is the largest
// |entry| among rows at logical position >= k, ties to the lowest logical
// position -- the pivot sequence of LU with partial pivoting.  A step costs two
// barriers (publish the per-wave candidates; publish a copy of the pivot row).
// The panel's row swaps are applied to the other columns, which then receive
// the rank-16 update A[:, R] += (Q - E) A_old[k0:k0+16, R] on MFMA f64
// 16x16x4 tiles (formed transposed so the accumulator tiles map to whole
// column segments), Q being the eliminated panel in logical row order and E the
// identity rows of the panel; the panel goes back to A in logical order.
//
// The column interchanges that would turn the result into K_i^{-1} are not
// performed: what is stored is B = (P K_i)^{-1}, and K_i^{-1} r = B (P r).  The
// kernel writes the permuted DoF list pdofs_perm[t] = pdofs[idx[t]] (idx =
// identity with the swaps applied in order), so the patch solve gathers P r
// at no extra cost, and idx itself (pidx): the transposed solve
// K_i^{-T} v = P^T B^T v puts entry t of B^T v at local position idx[t].  The singularity threshold 1e-14 ||K_i||_inf comes from
// the extraction kernel.
//
// MFMA f64 16x16x4 lane layout (lane l, accumulator element v):
//   A operand A[l % 16][l / 16], B operand B[l / 16][l % 16],
//   C/D element D[l / 16 + 4 v][l % 16].
// ---------------------------------------------------------------------------
// kGjTiles: 16 x 16 accumulator tiles of a column block updated together.  One
// keeps the register count, and so the number of resident waves, highest
// (measured faster than two or four on the 64..210-DoF patches of the P4/P3
// level); patches above 256 DoFs (two or more rows per thread) take four, whose
// loads in flight shorten the update's per-tile latency chain (on 362-DoF
// patches 51.6 -> 47.9 ms for 4,221 of them; gj_wide_kernel now takes 257-384).
template <int R, int kGjTiles>
__global__ __launch_bounds__(kBlock) void gj_kernel(const int64_t* __restrict__ pptr,
                                                    const int64_t* __restrict__ foff,
                                                    const int32_t* __restrict__ order, double* __restrict__ F,
                                                    const double* __restrict__ ptol,
                                                    const int32_t* __restrict__ pdofs,
                                                    int32_t* __restrict__ pdofs_perm,
                                                    int32_t* __restrict__ pidx, int ldq,
                                                    int* __restrict__ status) {
    constexpr int W = kPanel, NWV = kBlock / kWave;
    __shared__ double s_cv[2][NWV];
    __shared__ int s_ci[2][NWV];
    __shared__ int s_cp[2][NWV];
    __shared__ int s_phys_at[2];
    __shared__ int s_piv_panel[W];
    __shared__ double s_prow[2][W];
    extern __shared__ double smem[];
    double* Q = smem;                                  // ldq x W, physical rows
    int* s_phys = (int*)(Q + (int64_t)ldq * W);        // logical -> physical (m)
    int* piv = s_phys + ldq;                           // pivots of the whole patch (m)

    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id();
    const int p = order ? order[blockIdx.x] : (int)blockIdx.x;
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    double* A = F + foff[p];
    const double tol = ptol[p];

    for (int k0 = 0; k0 < m; k0 += W) {
        const int w = min(W, m - k0);
        for (int c = 0; c < w; ++c)
            for (int i = tid; i < m; i += kBlock) Q[i + c * ldq] = A[i + (int64_t)(k0 + c) * m];
        int lpos[R];
#pragma unroll
        for (int q = 0; q < R; ++q) lpos[q] = tid + q * kBlock;
        for (int i = tid; i < m; i += kBlock) s_phys[i] = i;
        __syncthreads();
        for (int c = 0; c < w; ++c) {
            const int k = k0 + c, buf = c & 1;
            double bv = -1.0;
            int bl = INT_MAX, bp = -1;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int r = tid + q * kBlock;
                if (r < m && lpos[q] >= k) {
                    const double a = fabs(Q[r + c * ldq]);
                    if (a > bv || (a == bv && lpos[q] < bl)) { bv = a; bl = lpos[q]; bp = r; }
                }
            }
            for (int off = kWave / 2; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int ol = __shfl_xor(bl, off), op = __shfl_xor(bp, off);
                if (ov > bv || (ov == bv && ol < bl)) { bv = ov; bl = ol; bp = op; }
            }
            if (lane == 0) { s_cv[buf][wave] = bv; s_ci[buf][wave] = bl; s_cp[buf][wave] = bp; }
            if (tid == 0) s_phys_at[buf] = s_phys[k];
            __syncthreads();                                          // barrier A
            bv = s_cv[buf][0]; bl = s_ci[buf][0]; bp = s_cp[buf][0];
            for (int q = 1; q < NWV; ++q) {
                const double ov = s_cv[buf][q];
                const int ol = s_ci[buf][q];
                if (ov > bv || (ov == bv && ol < bl)) { bv = ov; bl = ol; bp = s_cp[buf][q]; }
            }
            if (bp < 0 || !(bv > tol)) {                              // uniform decision
                if (tid == 0) atomicMin(status, p);
                return;
            }
            const int rk = s_phys_at[buf];
            if (tid < w) s_prow[buf][tid] = Q[bp + tid * ldq];
            if (tid == 0) {
                s_piv_panel[c] = bl;
                s_phys[bl] = rk;
                s_phys[k] = bp;
            }
            __syncthreads();                                          // barrier B
            const double d = 1.0 / s_prow[buf][c];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int r = tid + q * kBlock;
                if (r >= m) continue;
                if (r == bp) {
                    for (int cc = 0; cc < w; ++cc) Q[r + cc * ldq] = (cc == c) ? d : s_prow[buf][cc] * d;
                    lpos[q] = k;
                } else {
                    const double f = Q[r + c * ldq];
                    for (int cc = 0; cc < w; ++cc)
                        Q[r + cc * ldq] = (cc == c) ? -f * d : Q[r + cc * ldq] - f * (s_prow[buf][cc] * d);
                    if (r == rk) lpos[q] = bl;
                }
            }
        }
        if (tid < w) piv[k0 + tid] = s_piv_panel[tid];
        __syncthreads();
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
        // rank-w update of the other columns on MFMA f64 16x16x4, computed transposed:
        // A[I, J]^T += A_old[k0:k0+16, J]^T (Q - E)[I, :]^T, so that the accumulator
        // element v of lane l is A[i0 + l % 16][j0 + l / 16 + 4 v] and each load or
        // store of the wave covers four 128-byte column segments
        {
            const int nb16 = (m + 15) / 16;
            const int li = lane & 15, lk = lane >> 4;
            for (int jb = wave; jb < nb16; jb += NWV) {
                const int j = jb * 16 + li;
                const bool jv = (j < m) && (j < k0 || j >= k0 + w);
                if (!__any(jv ? 1 : 0)) continue;
                double bop[4];
#pragma unroll
                for (int kt = 0; kt < 4; ++kt) {
                    const int kk = kt * 4 + lk;
                    bop[kt] = (jv && kk < w) ? A[(k0 + kk) + (int64_t)j * m] : 0.0;
                }
                bool cv[4];                                   // columns of the accumulator elements
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int jc = jb * 16 + lk + 4 * v;
                    cv[v] = jc < m && (jc < k0 || jc >= k0 + w);
                }
                for (int ib = 0; ib < nb16; ib += kGjTiles) {
                    d4 acc[kGjTiles];
                    double aop[kGjTiles][4];
#pragma unroll
                    for (int h = 0; h < kGjTiles; ++h) {
                        const int i = (ib + h) * 16 + li;
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            acc[h][v] = (cv[v] && i < m) ? A[i + (int64_t)(jb * 16 + lk + 4 * v) * m] : 0.0;
#pragma unroll
                        for (int kt = 0; kt < 4; ++kt) {
                            const int kk = kt * 4 + lk;
                            double a = 0.0;
                            if (i < m && kk < w) {
                                a = Q[s_phys[i] + kk * ldq];
                                if (i == k0 + kk) a -= 1.0;
                            }
                            aop[h][kt] = a;
                        }
                    }
#pragma unroll
                    for (int h = 0; h < kGjTiles; ++h)
#pragma unroll
                        for (int kt = 0; kt < 4; ++kt)
                            acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(bop[kt], aop[h][kt], acc[h], 0, 0, 0);
#pragma unroll
                    for (int h = 0; h < kGjTiles; ++h) {
                        const int i = (ib + h) * 16 + li;
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (cv[v] && i < m) A[i + (int64_t)(jb * 16 + lk + 4 * v) * m] = acc[h][v];
                    }
                }
            }
        }
        // the eliminated panel goes back in logical order
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + q * kBlock;
            if (r >= m) continue;
            for (int c = 0; c < w; ++c) A[lpos[q] + (int64_t)(k0 + c) * m] = Q[r + c * ldq];
        }
        __syncthreads();
    }
    // P r gather list: idx = identity with the row swaps applied in order
    if (tid == 0) {
        for (int t = 0; t < m; ++t) s_phys[t] = t;
        for (int k = 0; k < m; ++k) {
            const int pr = piv[k];
            if (pr != k) {
                const int t = s_phys[k];
                s_phys[k] = s_phys[pr];
                s_phys[pr] = t;
            }
        }
    }
    __syncthreads();
    for (int t = tid; t < m; t += kBlock) {
        pdofs_perm[base + t] = pdofs[base + s_phys[t]];
        pidx[base + t] = s_phys[t];
    }
}

// ---------------------------------------------------------------------------
// The same inversion for patches of kWideMinM + 1 .. kWideMaxM DoFs (the
// Scott-Vogelius vertex patches), where gj_kernel moves every patch matrix
// (about 1 MB) through memory once per 16-column panel.  Here:
//  * 24-column panels (two thirds of the passes over the matrix), eliminated in
//    LDS by a 512-thread workgroup with one row per thread; two workgroups fit a
//    CU, so one's panel elimination overlaps the other's update (32-column
//    panels leave room for one workgroup per CU and were slower, as were 384-
//    and 640-thread workgroups);
//  * rows are never moved during the elimination: the logical -> physical row
//    map and each row's logical position persist across panels, the update
//    addresses the panel rows through the map, and one pass at the end puts
//    the rows of every column in logical order (instead of one pass of row
//    swaps per panel);
//  * the update's units (a column block with columns outside the panel, TG row
//    tiles) are dealt to the waves; since one unit may write rows that another
//    still reads as its B operand (the panel rows of its columns), those rows
//    are first copied into the panel's own columns, free until the panel is
//    written back.
// Same pivot rule (largest |entry| among logical positions >= k, ties to the
// lowest position), same stored B = (P K_i)^{-1}, pivot and DoF lists.
// ---------------------------------------------------------------------------
constexpr int kWidePanel = 24, kWideThreads = 512, kWideMinM = 256, kWideMaxM = 384;

__global__ __launch_bounds__(kWideThreads) void gj_wide_kernel(const int64_t* __restrict__ pptr,
                                                               const int64_t* __restrict__ foff,
                                                               const int32_t* __restrict__ order,
                                                               double* __restrict__ F,
                                                               const double* __restrict__ ptol,
                                                               const int32_t* __restrict__ pdofs,
                                                               int32_t* __restrict__ pdofs_perm,
                                                               int32_t* __restrict__ pidx, int ldq,
                                                               int* __restrict__ status) {
    constexpr int W = kWidePanel, NWV = kWideThreads / kWave, KT = W / 4, TG = 2;
    constexpr int NR = NWV <= 4 ? 4 : (NWV <= 8 ? 8 : 16);       // lanes of the candidate reduction
    static_assert(NWV <= NR && NR <= kWave, "candidate reduction over the first NR lanes");
    static_assert(kWideMaxM <= kWideThreads, "one row per thread");
    __shared__ double s_cv[2][NWV];
    __shared__ int s_ci[2][NWV];
    __shared__ int s_cp[2][NWV];
    __shared__ int s_phys_at[2];
    __shared__ double s_prow[2][W];
    extern __shared__ double smem[];
    double* Q = smem;                                  // ldq x W, physical rows
    int* s_phys = (int*)(Q + (int64_t)ldq * W);        // logical -> physical (m), kept across panels

    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id();
    const int p = order ? order[blockIdx.x] : (int)blockIdx.x;
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    double* A = F + foff[p];
    const double tol = ptol[p];
    const int r = tid;                                 // this thread's physical row (m <= kWideThreads)
    int lpos = r;                                      // its logical position
    if (r < m) s_phys[r] = r;
    const int nb16 = (m + 15) / 16, li = lane & 15, lk = lane >> 4;

    for (int k0 = 0; k0 < m; k0 += W) {
        const int w = min(W, m - k0);
        if (r < m)
            for (int c = 0; c < w; ++c) Q[r + c * ldq] = A[r + (int64_t)(k0 + c) * m];
        __syncthreads();
        for (int c = 0; c < w; ++c) {
            const int k = k0 + c, buf = c & 1;
            double bv = -1.0;
            int bl = INT_MAX, bp = -1;
            if (r < m && lpos >= k) {
                bv = fabs(Q[r + c * ldq]);
                bl = lpos;
                bp = r;
            }
            for (int off = kWave / 2; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int ol = __shfl_xor(bl, off), op = __shfl_xor(bp, off);
                if (ov > bv || (ov == bv && ol < bl)) { bv = ov; bl = ol; bp = op; }
            }
            if (lane == 0) { s_cv[buf][wave] = bv; s_ci[buf][wave] = bl; s_cp[buf][wave] = bp; }
            if (tid == 0) s_phys_at[buf] = s_phys[k];
            __syncthreads();                                          // barrier A
            // the waves' candidates, reduced over the first NR lanes of every wave
            // (logical positions are distinct, so the winner does not depend on the order)
            bv = lane < NWV ? s_cv[buf][lane] : -1.0;
            bl = lane < NWV ? s_ci[buf][lane] : INT_MAX;
            bp = lane < NWV ? s_cp[buf][lane] : -1;
            for (int off = NR / 2; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int ol = __shfl_xor(bl, off), op = __shfl_xor(bp, off);
                if (ov > bv || (ov == bv && ol < bl)) { bv = ov; bl = ol; bp = op; }
            }
            bv = __shfl(bv, 0);
            bl = __shfl(bl, 0);
            bp = __shfl(bp, 0);
            if (bp < 0 || !(bv > tol)) {                              // uniform decision
                if (tid == 0) atomicMin(status, p);
                return;
            }
            const int rk = s_phys_at[buf];
            if (tid < w) s_prow[buf][tid] = Q[bp + tid * ldq];
            if (tid == 0) {
                s_phys[bl] = rk;
                s_phys[k] = bp;
            }
            __syncthreads();                                          // barrier B
            const double d = 1.0 / s_prow[buf][c];
            if (r < m) {
                if (r == bp) {
                    for (int cc = 0; cc < w; ++cc) Q[r + cc * ldq] = (cc == c) ? d : s_prow[buf][cc] * d;
                    lpos = k;
                } else {
                    const double f = Q[r + c * ldq];
                    for (int cc = 0; cc < w; ++cc)
                        Q[r + cc * ldq] = (cc == c) ? -f * d : Q[r + cc * ldq] - f * (s_prow[buf][cc] * d);
                    if (r == rk) lpos = bl;
                }
            }
        }
        // rank-w update of the other columns, transposed as in gj_kernel: A[i, J] +=
        // sum_kk ((Q - E)[i, kk]) A[phys(k0 + kk), J], i physical, E(i, kk) = [i == phys(k0 + kk)].
        // First the B operand rows A(phys(k0 + kk), j) of every other column j go into the
        // panel's own columns (Q holds the panel until it is written back), as element
        // A[j + (k0 + kk) m]: the units then read them coalesced, and no unit can overwrite
        // them while another still needs them.
        if (r < m && (r < k0 || r >= k0 + w))
            for (int kk = 0; kk < w; ++kk) A[r + (int64_t)(k0 + kk) * m] = A[s_phys[k0 + kk] + (int64_t)r * m];
        int pk[KT];
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            const int kk = kt * 4 + lk;
            pk[kt] = kk < w ? s_phys[k0 + kk] : -1;
        }
        __syncthreads();
        {
            // column blocks with at least one column outside the panel; a block the panel
            // covers in part keeps its other columns (per-column masks)
            const int pb_lo = (k0 + 15) / 16, pb_hi = (k0 + w) / 16;   // blocks inside the panel
            const int nfull = (k0 + w == m) ? nb16 - pb_lo : max(0, pb_hi - pb_lo);
            const int nig = (nb16 + TG - 1) / TG, nunits = (nb16 - nfull) * nig;
            for (int u = wave; u < nunits; u += NWV) {
                const int jbx = u / nig, ig = u - jbx * nig;
                const int jb = jbx < pb_lo ? jbx : jbx + nfull, j = jb * 16 + li;
                const bool jv = j < m && (j < k0 || j >= k0 + w);
                double bop[KT];
#pragma unroll
                for (int kt = 0; kt < KT; ++kt)
                    bop[kt] = (jv && pk[kt] >= 0) ? A[j + (int64_t)(k0 + kt * 4 + lk) * m] : 0.0;
                bool cv[4];                            // columns of the accumulator elements
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int jc = jb * 16 + lk + 4 * v;
                    cv[v] = jc < m && (jc < k0 || jc >= k0 + w);
                }
                d4 acc[TG];
#pragma unroll
                for (int h = 0; h < TG; ++h) {
                    const int i = (ig * TG + h) * 16 + li;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        acc[h][v] = (cv[v] && i < m) ? A[i + (int64_t)(jb * 16 + lk + 4 * v) * m] : 0.0;
                }
#pragma unroll
                for (int h = 0; h < TG; ++h) {
                    const int i = (ig * TG + h) * 16 + li;
#pragma unroll
                    for (int kt = 0; kt < KT; ++kt) {
                        double a = 0.0;
                        if (i < m && pk[kt] >= 0) {
                            a = Q[i + (kt * 4 + lk) * ldq];
                            if (i == pk[kt]) a -= 1.0;
                        }
                        acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(bop[kt], a, acc[h], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int h = 0; h < TG; ++h) {
                    const int i = (ig * TG + h) * 16 + li;
                    if (i >= m) continue;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (cv[v]) A[i + (int64_t)(jb * 16 + lk + 4 * v) * m] = acc[h][v];
                }
            }
        }
        __syncthreads();                               // the copied operand rows are read
        // the eliminated panel goes back in physical row order
        if (r < m)
            for (int c = 0; c < w; ++c) A[r + (int64_t)(k0 + c) * m] = Q[r + c * ldq];
        __syncthreads();
    }
    // rows in logical order: B(l, j) = A(phys(l), j), W columns at a time through Q
    for (int j0 = 0; j0 < m; j0 += W) {
        const int w = min(W, m - j0);
        if (r < m)
            for (int c = 0; c < w; ++c) Q[r + c * ldq] = A[r + (int64_t)(j0 + c) * m];
        __syncthreads();
        if (r < m) {
            const int pr = s_phys[r];
            for (int c = 0; c < w; ++c) A[r + (int64_t)(j0 + c) * m] = Q[pr + c * ldq];
        }
        __syncthreads();
    }
    // P r gather list: the logical -> physical map is the identity with the row swaps applied in order
    if (r < m) {
        pdofs_perm[base + r] = pdofs[base + s_phys[r]];
        pidx[base + r] = s_phys[r];
    }
}

// ---------------------------------------------------------------------------
// The same blocked Gauss-Jordan inversion for levels of small patches
// (m <= kGjLdsMax): the whole m x m matrix sits in the workgroup's LDS, so it
// is read from global memory once and written back once, instead of once per
// 16-column panel.  Wave 0 eliminates each panel alone (its rows, RW per
// lane, held in registers: no barriers inside the panel) and writes it back
// in logical row order; then all waves apply the panel's row swaps to the
// other columns and the rank-16 update on MFMA f64 16x16x4 tiles, as in
// gj_kernel.  Same pivots (largest |entry| among logical positions >= k, ties
// to the lowest position), same stored B = (P K_i)^{-1} and pivot lists.
// Up to 141 DoFs would fit the 160 KB of LDS, but one wave eliminating 141
// rows, with one workgroup per CU, measured 3x slower than gj_kernel on the
// 141-DoF patches; with one row per lane (m <= 64) it is 1.7-2x faster.
// ---------------------------------------------------------------------------
constexpr int kGjLdsMax = 64;

template <int RW>
__global__ __launch_bounds__(kBlock) void gj_lds_kernel(const int64_t* __restrict__ pptr,
                                                        const int64_t* __restrict__ foff,
                                                        const int32_t* __restrict__ order, double* __restrict__ F,
                                                        const double* __restrict__ ptol,
                                                        const int32_t* __restrict__ pdofs,
                                                        int32_t* __restrict__ pdofs_perm,
                                                        int32_t* __restrict__ pidx, int ldq,
                                                        int* __restrict__ status) {
    constexpr int W = kPanel, NWV = kBlock / kWave;
    extern __shared__ double smem[];
    __shared__ int s_fail;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id();
    const int p = order[blockIdx.x];
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    double* G = F + foff[p];
    double* A = smem;                                      // m x m, column-major, ld m
    int* piv = reinterpret_cast<int*>(smem + (int64_t)ldq * ldq);   // pivots of the whole patch (m)
    int* perm = piv + ldq;                                           // gather list (m)
    const double tol = ptol[p];
    const int mm = m * m;
    for (int e = tid; e < mm; e += kBlock) A[e] = G[e];
    if (tid == 0) s_fail = 0;
    __syncthreads();

    for (int k0 = 0; k0 < m; k0 += W) {
        const int w = min(W, m - k0);
        if (wave == 0) {
            // rows lane, lane + 64, ... of the panel; at the panel's start every row
            // sits at its logical position
            double v[RW][W];
            int lpos[RW];
#pragma unroll
            for (int q = 0; q < RW; ++q) {
                const int r = lane + q * kWave;
                lpos[q] = r;
#pragma unroll
                for (int c = 0; c < W; ++c) v[q][c] = (r < m && c < w) ? A[r + (k0 + c) * m] : 0.0;
            }
            bool fail = false;
            for (int c = 0; c < w; ++c) {
                const int k = k0 + c;
                double bv = -1.0;
                int bl = INT_MAX, bo = -1;                        // value, logical position, owner (lane * RW + q)
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    const int r = lane + q * kWave;
                    double a = 0.0;
#pragma unroll
                    for (int cc = 0; cc < W; ++cc)
                        if (cc == c) a = fabs(v[q][cc]);
                    if (r < m && lpos[q] >= k && (a > bv || (a == bv && lpos[q] < bl))) {
                        bv = a;
                        bl = lpos[q];
                        bo = lane * RW + q;
                    }
                }
                for (int off = kWave / 2; off > 0; off >>= 1) {
                    const double ov = __shfl_xor(bv, off);
                    const int ol = __shfl_xor(bl, off), oo = __shfl_xor(bo, off);
                    if (ov > bv || (ov == bv && ol < bl)) {
                        bv = ov;
                        bl = ol;
                        bo = oo;
                    }
                }
                if (bo < 0 || !(bv > tol)) {                      // uniform over the wave
                    fail = true;
                    break;
                }
                const int ol = bo / RW, oq = bo % RW;
                double prow[W];
#pragma unroll
                for (int cc = 0; cc < W; ++cc) {
                    double mine = 0.0;
#pragma unroll
                    for (int q = 0; q < RW; ++q)
                        if (q == oq) mine = v[q][cc];
                    prow[cc] = __shfl(mine, ol);
                }
                double pc = 0.0;
#pragma unroll
                for (int cc = 0; cc < W; ++cc)
                    if (cc == c) pc = prow[cc];
                const double d = 1.0 / pc;
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    const int r = lane + q * kWave;
                    if (r >= m) continue;
                    if (lane * RW + q == bo) {
#pragma unroll
                        for (int cc = 0; cc < W; ++cc) v[q][cc] = (cc == c) ? d : prow[cc] * d;
                        lpos[q] = k;
                    } else {
                        double f = 0.0;
#pragma unroll
                        for (int cc = 0; cc < W; ++cc)
                            if (cc == c) f = v[q][cc];
#pragma unroll
                        for (int cc = 0; cc < W; ++cc) v[q][cc] = (cc == c) ? -f * d : v[q][cc] - f * (prow[cc] * d);
                        if (lpos[q] == k) lpos[q] = bl;              // the row at position k moves to bl
                    }
                }
                if (lane == 0) piv[k] = bl;
            }
            if (fail) {
                if (lane == 0) {
                    s_fail = 1;
                    atomicMin(status, p);
                }
            } else {
                // the eliminated panel goes back in logical order (rows are in registers)
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    const int r = lane + q * kWave;
                    if (r >= m) continue;
#pragma unroll
                    for (int c = 0; c < W; ++c)
                        if (c < w) A[lpos[q] + (k0 + c) * m] = v[q][c];
                }
            }
        }
        __syncthreads();
        if (s_fail) return;                                       // uniform: every wave leaves here
        // row swaps of this panel in every other column
        for (int j = tid; j < m; j += kBlock) {
            if (j >= k0 && j < k0 + w) continue;
            double* cj = A + j * m;
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
        // rank-w update of the other columns on MFMA f64 16x16x4, formed transposed as
        // in gj_kernel; (Q - E) is read from the panel columns, now in logical order
        {
            const int nb16 = (m + 15) / 16;
            const int li = lane & 15, lk = lane >> 4;
            for (int jb = wave; jb < nb16; jb += NWV) {
                const int j = jb * 16 + li;
                const bool jv = (j < m) && (j < k0 || j >= k0 + w);
                if (!__any(jv ? 1 : 0)) continue;
                double bop[4];
#pragma unroll
                for (int kt = 0; kt < 4; ++kt) {
                    const int kk = kt * 4 + lk;
                    bop[kt] = (jv && kk < w) ? A[(k0 + kk) + j * m] : 0.0;
                }
                bool cv[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int jc = jb * 16 + lk + 4 * v;
                    cv[v] = jc < m && (jc < k0 || jc >= k0 + w);
                }
                for (int ib = 0; ib < nb16; ++ib) {
                    const int i = ib * 16 + li;
                    d4 acc;
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[v] = (cv[v] && i < m) ? A[i + (jb * 16 + lk + 4 * v) * m] : 0.0;
                    double aop[4];
#pragma unroll
                    for (int kt = 0; kt < 4; ++kt) {
                        const int kk = kt * 4 + lk;
                        double a = 0.0;
                        if (i < m && kk < w) {
                            a = A[i + (k0 + kk) * m];
                            if (i == k0 + kk) a -= 1.0;
                        }
                        aop[kt] = a;
                    }
#pragma unroll
                    for (int kt = 0; kt < 4; ++kt)
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bop[kt], aop[kt], acc, 0, 0, 0);
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (cv[v] && i < m) A[i + (jb * 16 + lk + 4 * v) * m] = acc[v];
                }
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < mm; e += kBlock) G[e] = A[e];
    // P r gather list: idx = identity with the row swaps applied in order
    if (tid == 0) {
        for (int t = 0; t < m; ++t) perm[t] = t;
        for (int k = 0; k < m; ++k) {
            const int pr = piv[k];
            if (pr != k) {
                const int t = perm[k];
                perm[k] = perm[pr];
                perm[pr] = t;
            }
        }
    }
    __syncthreads();
    for (int t = tid; t < m; t += kBlock) {
        pdofs_perm[base + t] = pdofs[base + perm[t]];
        pidx[base + t] = perm[t];
    }
}

// f64 set-up result (column-major, ld = m) -> reduced-precision factors with
// ld = m rounded up to V = factor_pad<T>() (padding rows are zero); one
// workgroup per patch.
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
        if constexpr (sizeof(T) == 8) b[e] = v;
        else if constexpr (sizeof(T) == 4) b[e] = (T)v;
        else b[e] = __float2bfloat16((float)v);
    }
}

// f64 set-up result B = (P K_i)^{-1} (column-major, ld = m) -> the symmetric
// strip layout (phmg_internal.h) of S_i = (K_i^{-1} + K_i^{-T}) / 2 in precision T.  Column t of
// B is column idx[t] of K_i^{-1} (idx = pidx), so K_i^{-1}(i, j) = B(i, inv[j])
// with inv the inverse permutation.  One workgroup per patch.
template <typename T, int V>
__global__ __launch_bounds__(kBlock) void convert_sym_kernel(const int64_t* __restrict__ pptr,
                                                             const int64_t* __restrict__ foff64,
                                                             const int64_t* __restrict__ fofflp,
                                                             const int32_t* __restrict__ pidx,
                                                             const double* __restrict__ src, T* __restrict__ dst,
                                                             int ldt) {
    // LDS: the strip's kStrip source columns inv[r0 .. r0 + h - 1] (rows 0 .. w - 1,
    // leading dimension ldt, odd), then the inverse permutation (m ints)
    extern __shared__ double s_cols[];
    int32_t* s_inv = reinterpret_cast<int32_t*>(s_cols + (int64_t)kStrip * ldt);
    const int p = blockIdx.x;
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    // pidx is a permutation of 0 .. m-1 after a successful inversion (the host
    // checks the singularity status before this launch); entries outside the
    // range are ignored so that no index can leave the patch
    for (int t = threadIdx.x; t < m; t += kBlock) s_inv[t] = t;
    __syncthreads();
    for (int t = threadIdx.x; t < m; t += kBlock) {
        const int q = pidx[base + t];
        if (q >= 0 && q < m) s_inv[q] = t;
    }
    __syncthreads();
    const double* B = src + foff64[p];
    T* out = dst + fofflp[p];
    const int ns = (m + kStrip - 1) / kStrip;
    for (int s = 0; s < ns; ++s) {
        const int r0 = s * kStrip, h = min(kStrip, m - r0), hp = (h + V - 1) / V * V, w = r0 + h;
        // K_i^{-1}(j, i) = B(j, inv[i]) for the strip's rows i: whole column segments
        for (int e = threadIdx.x; e < h * w; e += kBlock) {
            const int q = e / w, j = e % w;
            s_cols[q * ldt + j] = B[j + (int64_t)s_inv[r0 + q] * m];
        }
        __syncthreads();
        T* S = out + sym_strip_offset(s, V);
        // strictly lower part (columns j < r0), then the diagonal block D (column
        // c: rows g(c) .. hp - 1) holding D(q, c) below the diagonal, D(c, c) / 2
        // on it and zero above it, so that the stored entries L satisfy
        // S = L + L^T exactly
        const int total = hp * w;
        for (int e = threadIdx.x; e < total; e += kBlock) {
            const int q = e % hp, j = e / hp, i = r0 + q;
            int64_t at = e;
            double f = 1.0;                       // the diagonal block stores lower(D) + diag(D) / 2
            if (j >= r0) {
                constexpr int PG = sym_pack(V);
                const int c = j - r0, g = c / PG * PG;
                if (q < g) continue;
                at = (int64_t)hp * r0 + sym_diag_offset(c, hp, PG) + (q - g);
                f = q > c ? 1.0 : (q == c ? 0.5 : 0.0);
            }
            double v = 0.0;
            if (i < m) v = f * (0.5 * (B[i + (int64_t)s_inv[j] * m] + s_cols[q * ldt + j]));
            if constexpr (sizeof(T) == 8) S[at] = v;
            else if constexpr (sizeof(T) == 4) S[at] = (T)v;
            else S[at] = __float2bfloat16((float)v);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Dense Gauss-Jordan inversion of one large matrix (the coarsest level) over
// the whole GPU, column-major N x N, panels of w columns:
//  * dense_panel_kernel: one workgroup of 512 threads holds the N x w panel
//    in registers (thread t owns physical rows t, t+512, ...) and eliminates
//    it with partial pivoting.  Rows are not moved: each thread tracks the
//    logical position of its rows (the swap "row k <-> row p" only exchanges
//    two logical positions), so a step costs two barriers: one to publish the
//    per-wave pivot candidates, one to publish the pivot row.  Ties go to the
//    lowest logical row, as in LU with partial pivoting.  The panel is written
//    back in logical order with its pivots.
//  * dense_swap_gather_kernel: applies the panel's row swaps to every other
//    column and copies the panel rows of those columns into T (w x N).
//  * dense_update_kernel: one wavefront per 16x16 tile outside the panel:
//    A[I, J] += (Q - E)[I, :] T[:, J] on MFMA f64 16x16x4.
//  * gj_unscramble_kernel: column swaps in reverse order, one thread per row.
// ---------------------------------------------------------------------------
constexpr int kDenseThreads = 512;

template <int R, int W>
__global__ __launch_bounds__(kDenseThreads) void dense_panel_kernel(double* __restrict__ A, int N, int k0, int w,
                                                                    int* __restrict__ piv, int* __restrict__ status,
                                                                    const double* __restrict__ tolp) {
    constexpr int NWV = kDenseThreads / kWave;
    __shared__ double s_cv[2][NWV];
    __shared__ int s_ci[2][NWV];     // logical row of the candidate
    __shared__ int s_cp[2][NWV];     // physical row of the candidate
    __shared__ double s_prow[2][W];
    __shared__ int s_phys_at[2];     // physical row currently at logical position k
    __shared__ int s_piv[W];
    extern __shared__ int s_phys[];  // logical -> physical for rows >= k0 (N entries)
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id();
    if (status[0] != INT32_MAX) return;
    const double tol = tolp[0];
    double v[R][W];
    int lpos[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * kDenseThreads;
        lpos[q] = r;
#pragma unroll
        for (int c = 0; c < W; ++c) v[q][c] = (r < N && c < w) ? A[r + (int64_t)(k0 + c) * N] : 0.0;
    }
    for (int i = tid; i < N; i += kDenseThreads) s_phys[i] = i;
    __syncthreads();
    for (int c = 0; c < w; ++c) {
        const int k = k0 + c, buf = c & 1;
        double bv = -1.0;
        int bl = INT_MAX, bp = -1;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + q * kDenseThreads;
            if (r < N && lpos[q] >= k) {
                double a = 0.0;
#pragma unroll
                for (int cc = 0; cc < W; ++cc) if (cc == c) a = fabs(v[q][cc]);
                if (a > bv || (a == bv && lpos[q] < bl)) { bv = a; bl = lpos[q]; bp = r; }
            }
        }
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off);
            const int ol = __shfl_xor(bl, off), op = __shfl_xor(bp, off);
            if (ov > bv || (ov == bv && ol < bl)) { bv = ov; bl = ol; bp = op; }
        }
        if (lane == 0) { s_cv[buf][wave] = bv; s_ci[buf][wave] = bl; s_cp[buf][wave] = bp; }
        if (tid == 0) s_phys_at[buf] = s_phys[k];
        __syncthreads();                                              // barrier A
        bv = s_cv[buf][0]; bl = s_ci[buf][0]; bp = s_cp[buf][0];
        for (int q = 1; q < NWV; ++q) {
            const double ov = s_cv[buf][q];
            const int ol = s_ci[buf][q];
            if (ov > bv || (ov == bv && ol < bl)) { bv = ov; bl = ol; bp = s_cp[buf][q]; }
        }
        if (bp < 0 || !(bv > tol)) {                                  // uniform decision
            if (tid == 0) atomicMin(status, 0);
            return;
        }
        const int rk = s_phys_at[buf];                                // physical row at logical k
        // owner of the pivot row publishes it
        if ((bp % kDenseThreads) == tid) {
            const int q = bp / kDenseThreads;
#pragma unroll
            for (int qq = 0; qq < R; ++qq)
                if (qq == q)
#pragma unroll
                    for (int cc = 0; cc < W; ++cc) s_prow[buf][cc] = v[qq][cc];
        }
        if (tid == 0) {
            s_piv[c] = bl;
            s_phys[bl] = rk;                                          // row k moves to logical bl
            s_phys[k] = bp;
        }
        __syncthreads();                                              // barrier B
        double prow[W];
#pragma unroll
        for (int cc = 0; cc < W; ++cc) prow[cc] = s_prow[buf][cc];
        double pc = 0.0;
#pragma unroll
        for (int cc = 0; cc < W; ++cc) if (cc == c) pc = prow[cc];
        const double d = 1.0 / pc;
        double srow[W];
#pragma unroll
        for (int cc = 0; cc < W; ++cc) srow[cc] = prow[cc] * d;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + q * kDenseThreads;
            if (r >= N) continue;
            if (r == bp) {
#pragma unroll
                for (int cc = 0; cc < W; ++cc) v[q][cc] = (cc == c) ? d : srow[cc];
                lpos[q] = k;
            } else {
                double f = 0.0;
#pragma unroll
                for (int cc = 0; cc < W; ++cc) if (cc == c) f = v[q][cc];
#pragma unroll
                for (int cc = 0; cc < W; ++cc) v[q][cc] = (cc == c) ? -f * d : v[q][cc] - f * srow[cc];
                if (r == rk) lpos[q] = bl;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * kDenseThreads;
        if (r >= N) continue;
#pragma unroll
        for (int c = 0; c < W; ++c)
            if (c < w) A[lpos[q] + (int64_t)(k0 + c) * N] = v[q][c];
    }
    if (tid < w) piv[k0 + tid] = s_piv[tid];
}

__global__ __launch_bounds__(kBlock) void dense_swap_gather_kernel(double* __restrict__ A, int N, int k0, int w,
                                                                   const int* __restrict__ piv,
                                                                   double* __restrict__ T,
                                                                   const int* __restrict__ status) {
    if (status[0] != INT32_MAX) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N || (j >= k0 && j < k0 + w)) return;
    double* cj = A + (int64_t)j * N;
    for (int c = 0; c < w; ++c) {
        const int pr = piv[k0 + c];
        if (pr != k0 + c) {
            const double t = cj[k0 + c];
            cj[k0 + c] = cj[pr];
            cj[pr] = t;
        }
    }
    for (int c = 0; c < w; ++c) T[c + (int64_t)j * kPanel] = cj[k0 + c];
}

__global__ __launch_bounds__(kBlock) void dense_update_kernel(double* __restrict__ A, int N, int k0, int w,
                                                              const double* __restrict__ T,
                                                              const int* __restrict__ status) {
    if (status[0] != INT32_MAX) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int nb16 = (N + 15) / 16;
    const int64_t tile = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    if (tile >= (int64_t)nb16 * nb16) return;
    const int jb = (int)(tile / nb16), ib = (int)(tile % nb16);
    if (jb * 16 >= k0 && jb * 16 + 15 < k0 + w) return;               // tile inside the panel
    const int li = lane & 15, lk = lane >> 4;
    const int j = jb * 16 + li;
    const bool jv = (j < N) && (j < k0 || j >= k0 + w);
    d4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = ib * 16 + lk + 4 * v;
        acc[v] = (jv && i < N) ? A[i + (int64_t)j * N] : 0.0;
    }
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
        const int kk = kt * 4 + lk;
        const double bop = (jv && kk < w) ? T[kk + (int64_t)j * kPanel] : 0.0;
        const int i = ib * 16 + li, ka = kt * 4 + lk;
        double aop = 0.0;
        if (i < N && ka < w) {
            aop = A[i + (int64_t)(k0 + ka) * N];
            if (i == k0 + ka) aop -= 1.0;
        }
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = ib * 16 + lk + 4 * v;
        if (jv && i < N) A[i + (int64_t)j * N] = acc[v];
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

// row sums |A_i.| (one thread per row, coalesced over rows) and tol = 1e-14 max_i
__global__ __launch_bounds__(kBlock) void row_abs_sum_kernel(const double* __restrict__ A, int N,
                                                             double* __restrict__ rs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += fabs(A[i + (int64_t)j * N]);
    rs[i] = s;
}

__global__ __launch_bounds__(kBlock) void max_tol_kernel(const double* __restrict__ rs, int N,
                                                         double* __restrict__ tol) {
    __shared__ double sh[kBlock / kWave];
    double m = 0.0;
    for (int i = threadIdx.x; i < N; i += kBlock) m = fmax(m, rs[i]);
    for (int off = kWave / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) tol[0] = 1e-14 * fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// s_j = sum_{slots t of DoF j, ascending patch id} w_t Y[t], or with one weight
// per DoF (wd) s_j = wd_j sum_t Y[t];  dn = a s_j + c d_j;
// x_j = (x_zero ? 0 : x_j) + dn;  d_j = dn when storing (Chebyshev direction).
// Richardson is a = omega, c = 0.
__global__ __launch_bounds__(kBlock) void scatter_kernel(int32_t n, const int32_t* __restrict__ sptr,
                                                         const int32_t* __restrict__ sslot,
                                                         const int4* __restrict__ sslot4,
                                                         const double* __restrict__ w, const double* __restrict__ wd,
                                                         const double* __restrict__ Y, double a, double c,
                                                         double* __restrict__ d, double* __restrict__ x, int flags) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double wj = wd ? wd[j] : 1.0;
    double s = 0.0;
    // the first four slots come from the padded copy, loaded together with the
    // slot range (no dependent index load); four slots in flight (indices
    // first, then the gathers); the sum runs over the slots in ascending order
    // (a missing slot adds +0)
    const int4 h = sslot4[j];
    const int beg = sptr[j], end = sptr[j + 1];
    int q[4] = {h.x, h.y, h.z, h.w};
    for (int t = beg;;) {
        double y[4], wq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            y[u] = q[u] >= 0 ? Y[q[u]] : 0.0;
            wq[u] = w && q[u] >= 0 ? w[q[u]] : 1.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s += w ? wq[u] * y[u] : y[u];
        t += 4;
        if (t >= end) break;
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = t + u < end ? sslot[t + u] : -1;
    }
    if (wd) s *= wj;
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
    const int lane = threadIdx.x & (kWave - 1), wave = wave_id();
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Partial dot products V[:, c] . w of one workgroup's rows, 8 columns at a
// time (all loads of a chunk in flight; one reduce-scatter over the wave and
// one LDS step per chunk), stored column-major for reduce_cols_kernel.
constexpr int kDotChunk = 8;

__global__ __launch_bounds__(kBlock) void multidot_partial_kernel(int64_t n, int ncol, const double* __restrict__ V,
                                                                  int64_t ldv, const double* __restrict__ w,
                                                                  double* __restrict__ partial) {
    constexpr int NW = kBlock / kWave;
    __shared__ double sh[kDotChunk][NW];
    const int lane = threadIdx.x & (kWave - 1), wave = wave_id();
    for (int c0 = 0; c0 < ncol; c0 += kDotChunk) {
        double acc[kDotChunk];
#pragma unroll
        for (int u = 0; u < kDotChunk; ++u) acc[u] = 0.0;
        for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
            const double wi = w[i];
#pragma unroll
            for (int u = 0; u < kDotChunk; ++u)
                if (c0 + u < ncol) acc[u] += V[i + (int64_t)(c0 + u) * ldv] * wi;
        }
        // wave sums of the 8 columns; lane l ends with column l / 8
        GroupReduce<double, kDotChunk, kWave, 1>::run(acc, lane);
        if (lane % (kWave / kDotChunk) == 0) sh[lane / (kWave / kDotChunk)][wave] = acc[0];
        __syncthreads();
        if (threadIdx.x < kDotChunk && c0 + (int)threadIdx.x < ncol) {
            const int u = threadIdx.x;
            partial[(int64_t)(c0 + u) * gridDim.x + blockIdx.x] = (sh[u][0] + sh[u][1]) + (sh[u][2] + sh[u][3]);
        }
        __syncthreads();
    }
}

// One Gram-Schmidt pass fused with the next reduction: w -= V h (h read from
// the device, the subtraction in the order of gemv_sub_kernel) and, from the
// same loaded basis values, the partial dot products V^T w of the updated w
// (NORM: the partial sum of w_i^2 instead).  ncol <= kGsMax.
constexpr int kGsMax = 32;

template <bool NORM>
__global__ __launch_bounds__(kBlock) void gs_update_kernel(int64_t n, int ncol, const double* __restrict__ V,
                                                           int64_t ldv, const double* __restrict__ h,
                                                           double* __restrict__ w, double* __restrict__ partial) {
    constexpr int NW = kBlock / kWave;
    constexpr int NA = NORM ? 1 : kGsMax;
    __shared__ double s_h[kGsMax];
    __shared__ double sh[NA][NW];
    const int lane = threadIdx.x & (kWave - 1), wave = wave_id();
    if (threadIdx.x < kGsMax) s_h[threadIdx.x] = (int)threadIdx.x < ncol ? h[threadIdx.x] : 0.0;
    __syncthreads();
    double acc[NA];
#pragma unroll
    for (int c = 0; c < NA; ++c) acc[c] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        double v[kGsMax];
#pragma unroll
        for (int c = 0; c < kGsMax; ++c) v[c] = c < ncol ? V[i + (int64_t)c * ldv] : 0.0;
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < kGsMax; ++c)
            if (c < ncol) s += v[c] * s_h[c];
        const double wi = w[i] - s;
        w[i] = wi;
        if constexpr (NORM) {
            acc[0] += wi * wi;
        } else {
#pragma unroll
            for (int c = 0; c < kGsMax; ++c) acc[c] += v[c] * wi;
        }
    }
    if constexpr (NORM) {
        for (int off = kWave / 2; off > 0; off >>= 1) acc[0] += __shfl_xor(acc[0], off);
        if (lane == 0) sh[0][wave] = acc[0];
    } else {
        // lane l ends with column l / 2
        GroupReduce<double, kGsMax, kWave, 1>::run(acc, lane);
        if (lane % 2 == 0) sh[lane / 2][wave] = acc[0];
    }
    __syncthreads();
    const int nout = NORM ? 1 : ncol;
    if ((int)threadIdx.x < nout) {
        const int c = threadIdx.x;
        partial[(int64_t)c * gridDim.x + blockIdx.x] = (sh[c][0] + sh[c][1]) + (sh[c][2] + sh[c][3]);
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

__global__ __launch_bounds__(kBlock) void axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b,
                                                       const double* __restrict__ y, double* __restrict__ z) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[i] = a * x[i] + b * y[i];
}

// X_c -= (dots[c] / zz) z for every system c (X: nrhs systems of length n, one after another)
__global__ __launch_bounds__(kBlock) void project_off_kernel(int64_t n, int nrhs, double* __restrict__ X,
                                                             const double* __restrict__ z,
                                                             const double* __restrict__ dots, double zz) {
    const int64_t total = n * nrhs;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = t / n, i = t - c * n;
        X[t] -= (dots[c] / zz) * z[i];
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
    if (A.rowblock && A.nrb > 0) {
        hipLaunchKernelGGL(rowblock_spmv_kernel, dim3(A.nrb), dim3(kBlock), 0, s, A.rblk, A.rowptr, A.col, A.val, x,
                           alpha, z, beta, y);
        return;
    }
    if (A.vec) {
        const int gridv = grid_for((int64_t)A.nrows * A.group, kBlock);
        switch (A.group) {
#define PHMG_SPMVV_CASE(G)                                                                                     \
    case G:                                                                                                    \
        hipLaunchKernelGGL((spmv_vec_kernel<G>), dim3(gridv), dim3(kBlock), 0, s, A.nrows, A.rowptr, A.col, A.val, \
                           x, alpha, z, beta, y);                                                              \
        return;
            PHMG_SPMVV_CASE(4)
            PHMG_SPMVV_CASE(8)
            PHMG_SPMVV_CASE(16)
#undef PHMG_SPMVV_CASE
            default:
                break;
        }
    }
    if (A.unroll == 8) {
        const int grid8 = grid_for((int64_t)A.nrows * A.group, kBlock);
        switch (A.group) {
#define PHMG_SPMV8_CASE(G)                                                                                       \
    case G:                                                                                                      \
        hipLaunchKernelGGL((spmv_kernel<G, false, 8>), dim3(grid8), dim3(kBlock), 0, s, A.nrows, A.rowptr, A.col, \
                           A.val, x, alpha, z, beta, y);                                                         \
        return;
            PHMG_SPMV8_CASE(4)
            PHMG_SPMV8_CASE(8)
            PHMG_SPMV8_CASE(16)
            PHMG_SPMV8_CASE(32)
#undef PHMG_SPMV8_CASE
            default:
                break;
        }
    }
    const int g = A.group;
    int grid = grid_for((int64_t)A.nrows * g, kBlock);
    if (A.xcd) grid = (grid + 7) / 8 * 8;
    switch (g * 2 + (A.xcd ? 1 : 0)) {
#define PHMG_SPMV_CASE(G)                                                                                        \
    case 2 * G:                                                                                                  \
        hipLaunchKernelGGL((spmv_kernel<G, false>), dim3(grid), dim3(kBlock), 0, s, A.nrows, A.rowptr, A.col,    \
                           A.val, x, alpha, z, beta, y);                                                         \
        break;                                                                                                   \
    case 2 * G + 1:                                                                                              \
        hipLaunchKernelGGL((spmv_kernel<G, true>), dim3(grid), dim3(kBlock), 0, s, A.nrows, A.rowptr, A.col,     \
                           A.val, x, alpha, z, beta, y);                                                         \
        break;
        PHMG_SPMV_CASE(2)
        PHMG_SPMV_CASE(4)
        PHMG_SPMV_CASE(8)
        PHMG_SPMV_CASE(16)
        PHMG_SPMV_CASE(32)
        PHMG_SPMV_CASE(64)
#undef PHMG_SPMV_CASE
        default:
            hipLaunchKernelGGL((spmv_kernel<8, false>), dim3(grid_for((int64_t)A.nrows * 8, kBlock)), dim3(kBlock), 0,
                               s, A.nrows, A.rowptr, A.col, A.val, x, alpha, z, beta, y);
    }
}

void launch_spmv_diff(hipStream_t s, const DevCsr& A1, const double* x1, const DevCsr& A2, const double* x2,
                      double* y) {
    if (A1.nrows <= 0) return;
    const int g = A2.group;
    const int grid = grid_for((int64_t)A1.nrows * g, kBlock);
    switch (g) {
#define PHMG_DIFF_CASE(G)                                                                                       \
    case G:                                                                                                     \
        hipLaunchKernelGGL(spmv_diff_kernel<G>, dim3(grid), dim3(kBlock), 0, s, A1.nrows, A1.rowptr, A1.col,    \
                           A1.val, x1, A2.rowptr, A2.col, A2.val, x2, y);                                       \
        break;
        PHMG_DIFF_CASE(2)
        PHMG_DIFF_CASE(4)
        PHMG_DIFF_CASE(8)
        PHMG_DIFF_CASE(16)
        PHMG_DIFF_CASE(32)
#undef PHMG_DIFF_CASE
        default:
            hipLaunchKernelGGL(spmv_diff_kernel<64>, dim3(grid_for((int64_t)A1.nrows * 64, kBlock)), dim3(kBlock), 0,
                               s, A1.nrows, A1.rowptr, A1.col, A1.val, x1, A2.rowptr, A2.col, A2.val, x2, y);
    }
}

void launch_extract(hipStream_t s, const Level& L, double* out) {
    if (L.npatch <= 0) return;
    const size_t lds = sizeof(double) * (size_t)kExtractRows * L.max_m + sizeof(int32_t) * (size_t)L.max_m;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)extract_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(extract_kernel, dim3(L.npatch), dim3(kBlock), lds, s, L.pptr, L.pdofs, L.foff, L.K.rowptr,
                       L.K.col, L.K.val, out, L.ptol);
}

int gj_lds_max_m() { return kGjLdsMax; }

void launch_patch_factor(hipStream_t s, const Level& L, double* A, hipStream_t aux, hipEvent_t ev_fork,
                         hipEvent_t ev_join) {
    if (L.npatch <= 0) return;
    static_assert(kGjLdsMax == 64, "size classes of gj_class");
    // patches too large for the registers (first in the launch order): panels in
    // LDS, the matrix in global memory; on the auxiliary stream when there is one
    const bool fork = aux && ev_fork && ev_join && L.gj_cnt[0] > 0;
    if (fork) {
        (void)hipEventRecord(ev_fork, s);
        (void)hipStreamWaitEvent(aux, ev_fork, 0);
    }
    if (L.gj_cnt[0] > 0) {
        const hipStream_t sb = fork ? aux : s;
        const int ldq = L.gj_max[0];
        if (ldq > kWideMinM && ldq <= kWideMaxM) {
            // 257-384 DoFs: 24-column panels, 512-thread workgroups, two per CU
            const size_t lds = sizeof(double) * (size_t)ldq * kWidePanel + sizeof(int) * (size_t)ldq;
            (void)hipFuncSetAttribute((const void*)gj_wide_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            hipLaunchKernelGGL(gj_wide_kernel, dim3(L.gj_cnt[0]), dim3(kWideThreads), lds, sb, L.pptr, L.foff, L.order,
                               A, L.ptol, L.pdofs, L.pdofs_perm, L.pidx, ldq, L.status);
        } else {
            const size_t lds = sizeof(double) * (size_t)ldq * kPanel + sizeof(int) * 2 * (size_t)ldq;
            const int R = (ldq + kBlock - 1) / kBlock;
            auto go = [&](auto kernel) {
                if (lds > 64 * 1024)
                    (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                hipLaunchKernelGGL(kernel, dim3(L.gj_cnt[0]), dim3(kBlock), lds, sb, L.pptr, L.foff, L.order, A,
                                   L.ptol, L.pdofs, L.pdofs_perm, L.pidx, ldq, L.status);
            };
            if (R <= 1) go(gj_kernel<1, 1>);
            else if (R <= 2) go(gj_kernel<2, 4>);
            else go(gj_kernel<4, 4>);
        }
        if (fork) (void)hipEventRecord(ev_join, aux);
    }
    struct Join {
        bool on;
        hipStream_t s;
        hipEvent_t e;
        ~Join() {
            if (on) (void)hipStreamWaitEvent(s, e, 0);
        }
    } join{fork, s, ev_join};
    // 65..144 DoFs: the matrix in the registers of the workgroup
    int first = L.gj_cnt[0];
    for (int c = 1; c <= 2; ++c) {
        launch_patch_factor_reg(s, L, A, first, L.gj_cnt[c], L.gj_max[c]);
        first += L.gj_cnt[c];
    }
    // the rest: the whole matrix in LDS
    const int nsmall = L.gj_cnt[3];
    if (nsmall <= 0) return;
    const int ldq = L.gj_max[3];
    const size_t lds = sizeof(double) * (size_t)ldq * ldq + sizeof(int) * 2 * (size_t)ldq;
    const int RW = (ldq + kWave - 1) / kWave;
    auto go = [&](auto kernel) {
        if (lds > 64 * 1024)
            (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kernel, dim3(nsmall), dim3(kBlock), lds, s, L.pptr, L.foff, L.order + first, A,
                           L.ptol, L.pdofs, L.pdofs_perm, L.pidx, ldq, L.status);
    };
    static_assert(kGjLdsMax <= kWave, "one row per lane");
    if (RW <= 1) go(gj_lds_kernel<1>);
}

void launch_convert_general(hipStream_t s, const Level& L, const double* src, void* dst, const int64_t* off) {
    if (L.npatch <= 0) return;
    if (L.prec == PHMG_PREC_F64)
        hipLaunchKernelGGL((convert_patch_kernel<double, factor_pad<double>()>), dim3(L.npatch), dim3(kBlock), 0, s,
                           L.pptr, L.foff, off, src, (double*)dst);
    else if (L.prec == PHMG_PREC_F32)
        hipLaunchKernelGGL((convert_patch_kernel<float, factor_pad<float>()>), dim3(L.npatch), dim3(kBlock), 0, s,
                           L.pptr, L.foff, off, src, (float*)dst);
    else
        hipLaunchKernelGGL((convert_patch_kernel<__hip_bfloat16, factor_pad<__hip_bfloat16>()>), dim3(L.npatch),
                           dim3(kBlock), 0, s, L.pptr, L.foff, off, src, (__hip_bfloat16*)dst);
}

void launch_convert_patches(hipStream_t s, const Level& L, const double* src, void* dst) {
    if (L.npatch <= 0) return;
    if (L.sym) {
        const int ldt = (int)L.max_m | 1;
        const size_t lds = sizeof(double) * (size_t)kStrip * ldt + sizeof(int32_t) * (size_t)L.max_m;
        if (lds > 64 * 1024) {
            (void)hipFuncSetAttribute((const void*)convert_sym_kernel<double, factor_pad<double>()>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            (void)hipFuncSetAttribute((const void*)convert_sym_kernel<float, factor_pad<float>()>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            (void)hipFuncSetAttribute((const void*)convert_sym_kernel<__hip_bfloat16, factor_pad<__hip_bfloat16>()>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        }
        if (L.prec == PHMG_PREC_F64)
            hipLaunchKernelGGL((convert_sym_kernel<double, factor_pad<double>()>), dim3(L.npatch), dim3(kBlock), lds, s,
                               L.pptr, L.foff, L.fofflp, L.pidx, src, (double*)dst, ldt);
        else if (L.prec == PHMG_PREC_F32)
            hipLaunchKernelGGL((convert_sym_kernel<float, factor_pad<float>()>), dim3(L.npatch), dim3(kBlock), lds, s,
                               L.pptr, L.foff, L.fofflp, L.pidx, src, (float*)dst, ldt);
        else
            hipLaunchKernelGGL((convert_sym_kernel<__hip_bfloat16, factor_pad<__hip_bfloat16>()>), dim3(L.npatch),
                               dim3(kBlock), lds, s, L.pptr, L.foff, L.fofflp, L.pidx, src, (__hip_bfloat16*)dst, ldt);
        return;
    }
    if (L.prec == PHMG_PREC_F64)
        hipLaunchKernelGGL((convert_patch_kernel<double, factor_pad<double>()>), dim3(L.npatch), dim3(kBlock), 0, s,
                           L.pptr, L.foff, L.fofflp, src, (double*)dst);
    else if (L.prec == PHMG_PREC_F32)
        hipLaunchKernelGGL((convert_patch_kernel<float, factor_pad<float>()>), dim3(L.npatch), dim3(kBlock), 0, s, L.pptr, L.foff,
                           L.fofflp, src, (float*)dst);
    else if (L.prec == PHMG_PREC_BF16)
        hipLaunchKernelGGL((convert_patch_kernel<__hip_bfloat16, factor_pad<__hip_bfloat16>()>), dim3(L.npatch), dim3(kBlock), 0, s, L.pptr,
                           L.foff, L.fofflp, src, (__hip_bfloat16*)dst);
}

void launch_scatter(hipStream_t s, const Level& L, double a, double c, double* d, bool store_d, double* x,
                    bool x_zero, bool transpose, const double* Y) {
    if (L.n <= 0) return;
    if (!Y) Y = L.Y;
    const int flags = (x_zero ? 1 : 0) | (c != 0.0 ? 2 : 0) | (store_d ? 4 : 0);
    const double* w = transpose || L.wdof ? nullptr : L.pweight;
    const double* wd = transpose ? nullptr : L.wdof;
    hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(L.n, kBlock)), dim3(kBlock), 0, s, L.n, L.sptr, L.sslot,
                       reinterpret_cast<const int4*>(L.sslot4), w, wd, Y, a, c, d, x, flags);
}

void launch_power_start(hipStream_t s, int64_t n, double* v) {
    hipLaunchKernelGGL(power_start_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, v);
}

void launch_scale_by_devnorm(hipStream_t s, int64_t n, const double* src, const double* norm2, double* dst) {
    hipLaunchKernelGGL(scale_by_devnorm_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n,
                       src, norm2, dst);
}

int coarse_panel_width(int N) {
    const int R = (N + kDenseThreads - 1) / kDenseThreads;
    return R <= 4 ? kPanel : (R <= 8 ? 8 : (R <= 16 ? 4 : 0));
}

namespace {
template <int R, int W>
void launch_dense_panel(hipStream_t s, double* A, int N, int k0, int w, int* piv, int* status, const double* tol) {
    hipLaunchKernelGGL((dense_panel_kernel<R, W>), dim3(1), dim3(kDenseThreads), sizeof(int) * N, s, A, N, k0, w,
                       piv, status, tol);
}
}  // namespace

void launch_dense_gj(hipStream_t s, double* A, int N, int* piv, int* status, double* tol, double* work) {
    // work: N doubles (row sums) + kPanel * N doubles (panel rows T)
    double* rs = work;
    double* T = work + N;
    hipLaunchKernelGGL(row_abs_sum_kernel, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, s, A, N, rs);
    hipLaunchKernelGGL(max_tol_kernel, dim3(1), dim3(kBlock), 0, s, rs, N, tol);
    const int R = (N + kDenseThreads - 1) / kDenseThreads;
    const int w0 = coarse_panel_width(N);
    const int nb16 = (N + 15) / 16;
    const int grid_upd = (int)(((int64_t)nb16 * nb16 * kWave + kBlock - 1) / kBlock);
    for (int k0 = 0; k0 < N; k0 += w0) {
        const int w = std::min(w0, N - k0);
        if (R <= 1) launch_dense_panel<1, kPanel>(s, A, N, k0, w, piv, status, tol);
        else if (R <= 2) launch_dense_panel<2, kPanel>(s, A, N, k0, w, piv, status, tol);
        else if (R <= 4) launch_dense_panel<4, kPanel>(s, A, N, k0, w, piv, status, tol);
        else if (R <= 8) launch_dense_panel<8, 8>(s, A, N, k0, w, piv, status, tol);
        else launch_dense_panel<16, 4>(s, A, N, k0, w, piv, status, tol);
        hipLaunchKernelGGL(dense_swap_gather_kernel, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, s, A, N, k0, w, piv,
                           T, status);
        hipLaunchKernelGGL(dense_update_kernel, dim3(grid_upd), dim3(kBlock), 0, s, A, N, k0, w, T, status);
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

void launch_coarse_solve_rows(hipStream_t s, const Level& L, const double* rows, const double* b, double* x) {
    hipLaunchKernelGGL(coarse_solve_kernel, dim3(grid_for((int64_t)L.n * kWave, kBlock)), dim3(kBlock), 0, s, L.n,
                       L.nb, rows, b, x);
}

void launch_coarse_solve(hipStream_t s, const Level& L, const double* b, double* x) {
    launch_coarse_solve_rows(s, L, L.cinv, b, x);
}

void launch_multidot(hipStream_t s, int64_t n, int ncol, const double* V, int64_t ldv, const double* w,
                     double* partial, double* out) {
    hipLaunchKernelGGL(multidot_partial_kernel, dim3(kRedBlocks), dim3(kBlock), 0, s, n, ncol, V, ldv, w, partial);
    hipLaunchKernelGGL(reduce_cols_kernel, dim3(ncol), dim3(kBlock), 0, s, kRedBlocks, partial, out);
}

void launch_project_off(hipStream_t s, int64_t n, int nrhs, double* X, const double* z, double zz, double* partial,
                        double* dots) {
    if (n <= 0 || nrhs <= 0) return;
    launch_multidot(s, n, nrhs, X, n, z, partial, dots);
    hipLaunchKernelGGL(project_off_kernel, dim3(std::min(grid_for(n * nrhs, kBlock), 4096)), dim3(kBlock), 0, s, n,
                       nrhs, X, z, dots, zz);
}

int gs_max_cols() { return kGsMax; }

void launch_gs_update(hipStream_t s, int64_t n, int ncol, const double* V, int64_t ldv, const double* h, double* w,
                      double* partial, double* out, bool norm) {
    if (norm)
        hipLaunchKernelGGL(gs_update_kernel<true>, dim3(kRedBlocks), dim3(kBlock), 0, s, n, ncol, V, ldv, h, w,
                           partial);
    else
        hipLaunchKernelGGL(gs_update_kernel<false>, dim3(kRedBlocks), dim3(kBlock), 0, s, n, ncol, V, ldv, h, w,
                           partial);
    hipLaunchKernelGGL(reduce_cols_kernel, dim3(norm ? 1 : ncol), dim3(kBlock), 0, s, kRedBlocks, partial, out);
}

void launch_gemv_sub(hipStream_t s, int64_t n, int ncol, const double* V, int64_t ldv, const double* h, double* w) {
    hipLaunchKernelGGL(gemv_sub_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, ncol, V,
                       ldv, h, w);
}

void launch_gemv_add(hipStream_t s, int64_t n, int ncol, const double* Z, int64_t ldz, const double* y, double* x) {
    hipLaunchKernelGGL(gemv_add_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, ncol, Z,
                       ldz, y, x);
}

void launch_axpby(hipStream_t s, int64_t n, double a, const double* x, double b, const double* y, double* z) {
    if (n <= 0) return;
    hipLaunchKernelGGL(axpby_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, a, x, b, y, z);
}

void launch_scale_copy(hipStream_t s, int64_t n, const double* src, double denom, double* dst) {
    hipLaunchKernelGGL(scale_copy_kernel, dim3(std::min(grid_for(n, kBlock), 4096)), dim3(kBlock), 0, s, n, src,
                       denom, dst);
}

}  // namespace phmg
