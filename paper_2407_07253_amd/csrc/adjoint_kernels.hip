// gfx950 kernels of the adjoint (transposed) relaxation: the operator
// M^T = sum_i R_i^T K_i^{-T} W_i R_i of the additive Schwarz sweep
// (eq. "eq:ASM") and the transposed coarse solve, from the factors the
// set-up stored for the forward sweep.
//
// The set-up keeps B_i = (P_i K_i)^{-1} with the pivoting permutation P_i as
// local positions pidx ((P_i r)_t = r[pidx[t]]), so K_i^{-1} = B_i P_i and
// K_i^{-T} = P_i^T B_i^T: the adjoint solve gathers W_i r[S_i] in the natural
// DoF order (gather and weighting swap places with the scatter), forms
// z = B_i^T v -- entry t is the dot product of the stored column t with v,
// a contiguous stream -- and writes z_t to local position pidx[t], where the
// unweighted DoF-centric scatter picks it up.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "phmg_internal.h"

namespace phmg {
namespace {

inline int grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (1 << 20)) g = 1 << 20;
    return (int)g;
}

__device__ inline float to_acc(__hip_bfloat16 v) { return __bfloat162float(v); }
__device__ inline float to_acc(float v) { return v; }
__device__ inline double to_acc(double v) { return v; }

// One workgroup per patch; each wavefront takes columns t = wave, wave + 4, ...
// U at a time (U independent column streams in flight), lanes striding the rows.
template <typename T, typename Acc, int V, int U>
__global__ __launch_bounds__(kBlock) void patch_apply_t_kernel(const int32_t* __restrict__ order,
                                                               const int64_t* __restrict__ pptr,
                                                               const int32_t* __restrict__ pdofs,
                                                               const int32_t* __restrict__ pidx,
                                                               const int64_t* __restrict__ foff,
                                                               const T* __restrict__ F,
                                                               const double* __restrict__ w,
                                                               const double* __restrict__ r,
                                                               double* __restrict__ Y) {
    constexpr int NW = kBlock / kWave;
    extern __shared__ double s_buf[];
    Acc* s_v = reinterpret_cast<Acc*>(s_buf);
    const int p = order[blockIdx.x];
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    const int ld = (m + factor_pad<T>() - 1) / factor_pad<T>() * factor_pad<T>();
    for (int t = threadIdx.x; t < m; t += kBlock) {
        const double v = r[pdofs[base + t]];
        s_v[t] = (Acc)(w ? w[base + t] * v : v);
    }
    __syncthreads();
    const T* A = F + foff[p];
    const int lane = threadIdx.x & (kWave - 1), wave = wave_id();
    for (int t0 = wave * U; t0 < m; t0 += NW * U) {
        Acc acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = 0;
        for (int i = lane; i < m; i += kWave) {
            const Acc vi = s_v[i];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (t0 + u < m) acc[u] += to_acc(A[(int64_t)(t0 + u) * ld + i]) * vi;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            Acc a = acc[u];
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) a += __shfl_xor(a, off);
            if (lane == 0 && t0 + u < m) Y[base + pidx[base + t0 + u]] = (double)a;
        }
    }
}


// Products of the adjoint and state vectors on the nonzeros of K (eq. of the
// adjoint gradient, dJ/dtheta = -sum_c lam_c^T (dK/dtheta) x_c):
// w_e = sum_c Lam[c][i_e] X[c][j_e] for every nonzero e = (i_e, j_e), systems
// stored one after another (length n each).  kPairLanes lanes per row.
constexpr int kPairLanes = 8;
__global__ __launch_bounds__(kBlock) void pair_products_kernel(int32_t n, const int32_t* __restrict__ rowptr,
                                                               const int32_t* __restrict__ col, int nrhs,
                                                               const double* __restrict__ X,
                                                               const double* __restrict__ Lam,
                                                               double* __restrict__ w) {
    const int lane = threadIdx.x & (kPairLanes - 1);
    const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kPairLanes;
    if (row >= n) return;
    for (int k = rowptr[row] + lane; k < rowptr[row + 1]; k += kPairLanes) {
        const int j = col[k];
        double s = 0.0;
        for (int c = 0; c < nrhs; ++c) s += Lam[(int64_t)c * n + row] * X[(int64_t)c * n + j];
        w[k] = s;
    }
}

template <typename T, typename Acc, int V, int U>
void launch_t_shape(hipStream_t s, const Level& L, const int64_t* off, const double* r) {
    hipLaunchKernelGGL((patch_apply_t_kernel<T, Acc, V, U>), dim3(L.npatch), dim3(kBlock), sizeof(Acc) * L.max_m, s,
                       L.order, L.pptr, L.pdofs, L.pidx, off, (const T*)L.factors, L.pweight, r, L.Y);
}

}  // namespace

void launch_patch_apply_t(hipStream_t s, const Level& L, const double* r) {
    if (L.npatch <= 0) return;
    if (L.sym) {                      // S_i^T = S_i: the forward kernel, weights at the gather
        launch_patch_apply_sym(s, L, r, L.pweight);
        return;
    }
    if (L.prec == PHMG_PREC_F32) launch_t_shape<float, float, 2, 4>(s, L, L.fofflp, r);
    else if (L.prec == PHMG_PREC_BF16) launch_t_shape<__hip_bfloat16, float, 4, 4>(s, L, L.fofflp, r);
    else launch_t_shape<double, double, 1, 4>(s, L, L.fofflp, r);
}

void launch_pair_products(hipStream_t s, const DevCsr& K, int nrhs, const double* X, const double* Lam,
                          double* w) {
    if (K.nrows <= 0) return;
    hipLaunchKernelGGL(pair_products_kernel, dim3(grid_for((int64_t)K.nrows * kPairLanes, kBlock)), dim3(kBlock), 0,
                       s, K.nrows, K.rowptr, K.col, nrhs, X, Lam, w);
}

void launch_coarse_solve_t(hipStream_t s, const Level& L, const double* b, double* x) {
    // the set-up keeps the coarse inverse column-major as well (L.cdense): read
    // row-major it is the transposed inverse, so the forward kernel applies it
    launch_coarse_solve_rows(s, L, L.cdense, b, x);
}

}  // namespace phmg
