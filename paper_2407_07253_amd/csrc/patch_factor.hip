// gfx950 batched inversion of the Vanka-star patch matrices: the set-up of the
// additive Schwarz smoother (Section 3.4: every patch system is solved exactly
// with an LU factorisation).  Each patch matrix K_i is turned into the explicit
// inverse B_i = (P_i K_i)^{-1} by Gauss-Jordan elimination with the pivots of LU
// with partial pivoting (largest |entry| in the column among the rows not yet
// pivoted, ties to the lowest logical row position), so the sweep streams one
// dense matrix per patch.
//
// Register-resident kernel (gj_reg_kernel): one workgroup per patch holds the
// whole matrix, padded to MT x MT tiles of 16 x 16, in the MFMA f64 16x16x4
// accumulators of its NW waves, so the matrix is read from and written to
// memory once.  Rows never move: row r of the registers is row r of K_i, and
// the pivot sequence is kept as logical positions (s_phys: logical position ->
// row, lpos: row -> logical position).  Per panel of 16 columns:
//   1. the waves holding the panel's tiles copy them to LDS (Q, m x 16);
//   2. the panel is eliminated in LDS by every thread (rows tid, tid + NT, ...):
//      pivot search, pivot row scaled, every other row reduced -- Gauss-Jordan
//      in the panel, two barriers per column;
//   3. the waves holding the pivot rows copy those rows of the other columns to
//      LDS (Prow, 16 x m);
//   4. every other tile takes the rank-16 update A[I, J] += (Q - E)[I, :]
//      A_old[piv, J] on MFMA (formed transposed, as the accumulator layout
//      wants: D = A_old[piv, J]^T (Q - E)[I, :]^T), E the unit entries at the
//      pivot rows; the panel's own tiles take Q.
// At the end row r is written to its logical position lpos(r), which gives the
// inverse of the row-permuted matrix, (P K_i)^{-1}, in the layout the rest of
// the set-up expects; the gather list pdofs_perm = pdofs[s_phys] applies P_i.
//
// MFMA f64 16x16x4 lane layout (lane l, accumulator element v):
//   A operand A[l % 16][l / 16], B operand B[l / 16][l % 16],
//   C/D element D[l / 16 + 4 v][l % 16].
// A tile (I, J) is kept transposed: element v of lane l is
// A[16 I + l % 16][16 J + l / 16 + 4 v].
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "phmg_internal.h"

namespace phmg {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// Move x from a lane of the same 16-lane row (DPP): CTRL 0xB1 / 0x4E swap lanes
// at distance 1 / 2 inside quads, 0x124 / 0x128 rotate the row by 4 / 8.
template <int CTRL>
__device__ inline int dpp_i(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
__device__ inline double readlane_d(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline double dpp_d(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// pivot candidates are ordered by |value| (larger first), then logical position
// (lower first): a total order, so every reduction shape picks the same pivot
__device__ inline bool cand_better(double ov, int ol, double v, int l) { return ov > v || (ov == v && ol < l); }
struct Cand {
    double v;
    int l, p;
};

// element e (runtime, 0..3) of a tile fragment
__device__ inline double pick4(const d4& x, int e) {
    const double lo = e & 1 ? x[1] : x[0];
    const double hi = e & 1 ? x[3] : x[2];
    return e & 2 ? hi : lo;
}

// NW = ceil(MT / RPW) waves; wave w owns tile rows w RPW .. w RPW + RPW - 1 in
// acc[0 .. RPW)[0 .. MT).  Panel s is tile column s; at its start every wave
// copies its rows of it to P (element v of lane l of P[ir] holds row 16 (w RPW +
// ir) + l % 16, panel column l / 16 + 4 v) and eliminates them there.  Per column
// c of the panel:
//   * the lanes of column group c % 4 hold the column's entries; the wave's
//     largest |entry| among rows not yet pivoted (logical position >= k) comes
//     from a DPP max over the 16-lane row, its holder from a ballot (ties: the
//     lowest logical position, a DPP min over the tied lanes);
//   * one lane posts (|pivot|, logical position, row) and the holder's lanes the
//     row's 16 panel entries times 1 / pivot (the pivot column holds 1 / pivot)
//     to LDS; one barrier; every thread picks the same winner among the NW posts
//     (posts alternate between two slots, so one barrier per column suffices);
//   * every row r takes P[r] - f_r post (f_r its entry in column c; column c
//     itself becomes -f_r / pivot), the pivot row becomes the post.
// Each wave holds several tile rows so the per-column overhead (reduction,
// ballot, winner pick, division) runs on few waves; two-wave workgroups at one
// wave per SIMD let two patches share a CU, each hiding the other's latencies.
template <int MT, int RPW>
__global__ __launch_bounds__((MT + RPW - 1) / RPW * 64) void gj_reg_kernel(
    const int64_t* __restrict__ pptr, const int64_t* __restrict__ foff, const int32_t* __restrict__ order,
    double* __restrict__ F, const double* __restrict__ ptol, const int32_t* __restrict__ pdofs,
    int32_t* __restrict__ pdofs_perm, int32_t* __restrict__ pidx, int* __restrict__ status) {
    constexpr int W = kPanel, NW = (MT + RPW - 1) / RPW, NT = NW * kWave, MP = MT * 16;
    __shared__ double Prow[W * MP];               // pivot rows of the other columns, row-major
    __shared__ Cand s_cand[2][NW];                // each wave's candidate, two slots
    __shared__ double s_crow[2][NW][W];           // the candidate rows' panel entries / pivot
    __shared__ int s_phys[MP];                    // logical position -> row (built at the end)

    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int li = lane & 15, lk = lane >> 4;
    const int p = order[blockIdx.x];
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    const int mt = (m + 15) >> 4;
    double* A = F + foff[p];
    const double tol = ptol[p];
    int row[RPW];                                 // this lane's rows
    bool live[RPW];
#pragma unroll
    for (int ir = 0; ir < RPW; ++ir) {
        row[ir] = 16 * (wave * RPW + ir) + li;
        live[ir] = row[ir] < m;
    }

    // the matrix into the accumulator tiles (zero outside m x m): acc[ir][J] is tile (w RPW + ir, J)
    d4 acc[RPW][MT];
#pragma unroll
    for (int ir = 0; ir < RPW; ++ir)
#pragma unroll
        for (int J = 0; J < MT; ++J)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 16 * J + lk + 4 * v;
                acc[ir][J][v] = (live[ir] && j < m) ? A[row[ir] + (int64_t)j * m] : 0.0;
            }
    int my_lpos[RPW];                             // logical positions of this lane's rows
#pragma unroll
    for (int ir = 0; ir < RPW; ++ir) my_lpos[ir] = live[ir] ? row[ir] : INT_MAX;

    for (int s = 0; s < mt; ++s) {
        const int k0 = 16 * s, w = min(W, m - k0);
        d4 P[RPW];
        int mypiv[RPW];                            // pivot index of each row in the panel, or -1
#pragma unroll
        for (int ir = 0; ir < RPW; ++ir) {
            P[ir] = acc[ir][0];
#pragma unroll
            for (int J = 1; J < MT; ++J)
                if (J == s) P[ir] = acc[ir][J];
            mypiv[ir] = -1;
        }
#pragma clang loop unroll(full)
        for (int c = 0; c < W; ++c) {
            if (c < w) {                           // uniform
                const int g = c & 3, e = c >> 2, k = k0 + c, slot = c & 1;
                const bool ingrp = lk == g;
                // this lane's rows' entries in column c, as held by the lanes of group g
                double f[RPW], aa[RPW];
                double am = -1.0;
#pragma unroll
                for (int ir = 0; ir < RPW; ++ir) {
                    f[ir] = __shfl(P[ir][e], li | (16 * g));
                    aa[ir] = (ingrp && my_lpos[ir] >= k) ? fabs(P[ir][e]) : -1.0;
                    am = fmax(am, aa[ir]);
                }
                am = fmax(am, dpp_d<0x128>(am));
                am = fmax(am, dpp_d<0x124>(am));
                am = fmax(am, dpp_d<0x4E>(am));
                am = fmax(am, dpp_d<0xB1>(am));
                const double wmax = readlane_d(am, 16 * g);
                // holder of the wave's candidate: (tile row wir, lane wlane)
                int nhit = 0, wir = -1, wlane = -1;
#pragma unroll
                for (int ir = 0; ir < RPW; ++ir) {
                    const uint64_t h = __ballot(wmax >= 0.0 && aa[ir] == wmax);
                    nhit += __popcll(h);
                    if (h && wir < 0) {
                        wir = ir;
                        wlane = __ffsll((unsigned long long)h) - 1;
                    }
                }
                if (nhit > 1) {                    // equal magnitudes: the lowest logical position
                    int lm = INT_MAX;
#pragma unroll
                    for (int ir = 0; ir < RPW; ++ir) lm = min(lm, aa[ir] == wmax ? my_lpos[ir] : INT_MAX);
                    lm = min(lm, dpp_i<0x128>(lm));
                    lm = min(lm, dpp_i<0x124>(lm));
                    lm = min(lm, dpp_i<0x4E>(lm));
                    lm = min(lm, dpp_i<0xB1>(lm));
                    const int minl = __builtin_amdgcn_readlane(lm, 16 * g);
                    wir = -1;
#pragma unroll
                    for (int ir = 0; ir < RPW; ++ir) {
                        const uint64_t h = __ballot(aa[ir] == wmax && my_lpos[ir] == minl);
                        if (h && wir < 0) {
                            wir = ir;
                            wlane = __ffsll((unsigned long long)h) - 1;
                        }
                    }
                }
                int wl = INT_MAX, wp = -1;
                double wv = 1.0;
                d4 pr = P[0];
#pragma unroll
                for (int ir = 0; ir < RPW; ++ir)
                    if (ir == wir) {
                        wl = __builtin_amdgcn_readlane(my_lpos[ir], wlane);
                        wv = readlane_d(P[ir][e], wlane);
                        wp = 16 * (wave * RPW + ir) + (wlane & 15);
                        pr = P[ir];
                    }
                const double dw = 1.0 / wv;
                if (lane == 0) s_cand[slot][wave] = Cand{wmax, wl, wp};
                if (wir >= 0 && li == (wlane & 15)) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) s_crow[slot][wave][lk + 4 * v] = (v == e && ingrp) ? dw : pr[v] * dw;
                }
                __syncthreads();
                // every thread reads all posts and picks the same winner
                Cand best = s_cand[slot][0];
                double crow[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) crow[v] = s_crow[slot][0][lk + 4 * v];
#pragma unroll
                for (int q = 1; q < NW; ++q) {
                    const Cand o = s_cand[slot][q];
                    double cr[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) cr[v] = s_crow[slot][q][lk + 4 * v];
                    const bool bq = cand_better(o.v, o.l, best.v, best.l);
                    best.v = bq ? o.v : best.v;
                    best.l = bq ? o.l : best.l;
                    best.p = bq ? o.p : best.p;
#pragma unroll
                    for (int v = 0; v < 4; ++v) crow[v] = bq ? cr[v] : crow[v];
                }
                if (best.p < 0 || !(best.v > tol)) {                     // uniform decision
                    if (tid == 0) atomicMin(status, p);
                    return;
                }
#pragma unroll
                for (int ir = 0; ir < RPW; ++ir) {
                    const bool isp = row[ir] == best.p;
                    const double gs = isp ? -1.0 : f[ir];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double t = (isp || (v == e && ingrp)) ? 0.0 : P[ir][v];
                        P[ir][v] = fma(-gs, crow[v], t);
                    }
                    mypiv[ir] = isp ? c : mypiv[ir];
                    my_lpos[ir] = isp ? k : (my_lpos[ir] == k ? best.l : my_lpos[ir]);
                }
            }
        }
#pragma unroll
        for (int ir = 0; ir < RPW; ++ir) {
#pragma unroll
            for (int J = 0; J < MT; ++J)
                if (J == s) acc[ir][J] = P[ir];
            // the pivot rows of the other columns to LDS
            if (mypiv[ir] >= 0) {
#pragma unroll
                for (int J = 0; J < MT; ++J)
                    if (J != s && J < mt) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) Prow[mypiv[ir] * MP + 16 * J + lk + 4 * v] = acc[ir][J][v];
                    }
            }
        }
        __syncthreads();
        // rank-16 update of the other tiles: (Q - E) is the eliminated panel in P
        double aop[RPW][4];
#pragma unroll
        for (int ir = 0; ir < RPW; ++ir)
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
                const int kk = 4 * kt + lk;
                aop[ir][kt] = kk < w ? P[ir][kt] - (mypiv[ir] == kk ? 1.0 : 0.0) : 0.0;
            }
#pragma unroll
        for (int J = 0; J < MT; ++J) {
            if (J == s || J >= mt) continue;
            double bop[4];
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
                const int kk = 4 * kt + lk;
                bop[kt] = kk < w ? Prow[kk * MP + 16 * J + li] : 0.0;
            }
#pragma unroll
            for (int ir = 0; ir < RPW; ++ir) {
                if (wave * RPW + ir >= MT) continue;
#pragma unroll
                for (int kt = 0; kt < 4; ++kt)
                    acc[ir][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(bop[kt], aop[ir][kt], acc[ir][J], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // row r goes to its logical position
#pragma unroll
    for (int ir = 0; ir < RPW; ++ir)
        if (live[ir] && lk == 0) s_phys[my_lpos[ir]] = row[ir];
    __syncthreads();
#pragma unroll
    for (int ir = 0; ir < RPW; ++ir) {
        if (!live[ir]) continue;
#pragma unroll
        for (int J = 0; J < MT; ++J)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 16 * J + lk + 4 * v;
                if (j < m) A[my_lpos[ir] + (int64_t)j * m] = acc[ir][J][v];
            }
    }
    for (int t = tid; t < m; t += NT) {
        pdofs_perm[base + t] = pdofs[base + s_phys[t]];
        pidx[base + t] = s_phys[t];
    }
}

template <int MT, int RPW>
void launch_reg(hipStream_t s, const Level& L, double* A, int first, int count) {
    hipLaunchKernelGGL((gj_reg_kernel<MT, RPW>), dim3(count), dim3((MT + RPW - 1) / RPW * kWave), 0, s, L.pptr,
                       L.foff, L.order + first, A, L.ptol, L.pdofs, L.pdofs_perm, L.pidx, L.status);
}

}  // namespace

int gj_reg_max_m() { return 144; }

// patches of the launch-order range [first, first + count), all of at most max_m DoFs
void launch_patch_factor_reg(hipStream_t s, const Level& L, double* A, int first, int count, int max_m) {
    if (count <= 0) return;
    if (max_m <= 96) launch_reg<6, 3>(s, L, A, first, count);
    else launch_reg<9, 5>(s, L, A, first, count);
}

}  // namespace phmg
