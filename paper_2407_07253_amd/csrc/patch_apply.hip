// gfx950 batched patch solve of the additive Schwarz sweep (Section 3.4,
// eq. "eq:ASM"): y_i = K_i^{-1} r[S_i] for every Vanka-star patch, streaming the
// explicit patch inverses stored by the set-up.  This is the dominant kernel of
// the solve phase (HBM-bound: every factor word is read once per sweep).
//
// General layout: patch i's inverse B_i = (P_i K_i)^{-1} is column-major with
// every column padded to a multiple of 16 bytes (ld = m rounded up to V = 2 /
// 4 / 8 rows for f64 / f32 / bf16); the gather list pdofs_perm already applies
// the pivot permutation, so y_i = B_i r[pdofs_perm(i)].
//
// Symmetric layout (symmetric level matrices): S_i = sym(K_i^{-1}) in row
// strips of 16 (strictly lower part + diagonal block, see phmg_internal.h);
// every stored off-diagonal entry is used twice, once as S(i, j) and once as
// S(j, i), so a sweep streams about half the bytes.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "phmg_internal.h"

namespace phmg {
namespace {

// One 16-byte load of V consecutive factor rows, widened to the accumulation type.
// NT: a non-temporal load.  A level whose factors exceed what the caches could
// keep between sweeps streams them this way, so the stream does not evict the
// level matrix and vectors that the next kernels of the cycle reuse.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef uint32_t nt_u4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Load16;
template <>
struct Load16<double> {
    static constexpr int V = 2;
    typedef double acc_t;
    template <bool NT>
    __device__ static inline void load(const double* p, double (&a)[2]) {
        const nt_d2* q = reinterpret_cast<const nt_d2*>(p);
        const nt_d2 v = NT ? __builtin_nontemporal_load(q) : *q;
        a[0] = v.x;
        a[1] = v.y;
    }
};
template <>
struct Load16<float> {
    static constexpr int V = 4;
    typedef float acc_t;
    template <bool NT>
    __device__ static inline void load(const float* p, float (&a)[4]) {
        const nt_f4* q = reinterpret_cast<const nt_f4*>(p);
        const nt_f4 v = NT ? __builtin_nontemporal_load(q) : *q;
        a[0] = v.x;
        a[1] = v.y;
        a[2] = v.z;
        a[3] = v.w;
    }
};
template <>
struct Load16<__hip_bfloat16> {
    static constexpr int V = 8;
    typedef float acc_t;
    template <bool NT>
    __device__ static inline void load(const __hip_bfloat16* p, float (&a)[8]) {
        const nt_u4* q = reinterpret_cast<const nt_u4*>(p);
        const nt_u4 v = NT ? __builtin_nontemporal_load(q) : *q;
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            a[2 * h] = __uint_as_float(w[h] << 16);
            a[2 * h + 1] = __uint_as_float(w[h] & 0xffff0000u);
        }
    }
};

// One workgroup per patch (launch order: decreasing m).  The patch's columns
// are cut into row groups of V rows (one 16-byte load each); with LPC row
// groups per column, thread t < S = LPC * (256 / LPC) owns row group t % LPC of
// the columns t / LPC, t / LPC + 256 / LPC, ... so the workgroup's loads form
// one contiguous stream (no idle lanes inside short columns) with U loads in
// flight per thread.  Columns taller than 256 row groups are processed in
// chunks of 256 groups.  Each thread sums its columns in ascending order; the
// 256 / LPC partial sums of a row are then added in ascending thread order, so
// the result does not depend on U (every compiled shape is bit-identical).
template <typename T, int U, bool NT>
__global__ __launch_bounds__(kBlock) void patch_apply_kernel(const int32_t* __restrict__ order,
                                                             const int64_t* __restrict__ pptr,
                                                             const int32_t* __restrict__ pdofs,
                                                             const int64_t* __restrict__ foff,
                                                             const T* __restrict__ F, const double* __restrict__ r,
                                                             double* __restrict__ Y, int ldbuf) {
    typedef typename Load16<T>::acc_t Acc;
    constexpr int V = Load16<T>::V;
    static_assert(V == factor_pad<T>(), "columns are padded to one 16-byte load");
    extern __shared__ double s_buf[];
    Acc* s_r = reinterpret_cast<Acc*>(s_buf);
    Acc* s_part = s_r + ldbuf;                                    // kBlock * V partial sums
    const int p = order[blockIdx.x];
    const int64_t base = pptr[p];
    const int m = (int)(pptr[p + 1] - base);
    const int ld = (m + V - 1) / V * V;
    for (int t = threadIdx.x; t < m; t += kBlock) s_r[t] = (Acc)r[pdofs[base + t]];
    __syncthreads();
    const T* A = F + foff[p];
    const int groups = ld / V;
    for (int g0 = 0; g0 < groups; g0 += kBlock) {
        const int lpc = min(groups - g0, kBlock);
        const int cps = kBlock / lpc;                             // columns per sweep of the workgroup
        const int t = threadIdx.x;
        const int rg = t % lpc, c0 = t / lpc;
        Acc acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = 0;
        if (c0 < cps) {
            const T* colbase = A + (int64_t)(g0 + rg) * V;
            int j = c0;
            for (; j + (U - 1) * cps < m; j += U * cps) {
                Acc a[U][V];
#pragma unroll
                for (int u = 0; u < U; ++u) Load16<T>::template load<NT>(colbase + (int64_t)(j + u * cps) * ld, a[u]);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const Acc rj = s_r[j + u * cps];
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[v] += a[u][v] * rj;
                }
            }
            for (; j < m; j += cps) {
                Acc a[V];
                Load16<T>::template load<NT>(colbase + (int64_t)j * ld, a);
                const Acc rj = s_r[j];
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] += a[v] * rj;
            }
        }
#pragma unroll
        for (int v = 0; v < V; ++v) s_part[t * V + v] = acc[v];
        __syncthreads();
        for (int i = threadIdx.x; i < lpc * V; i += kBlock) {
            const int g = i / V, v = i % V;
            const int row = (g0 + g) * V + v;
            if (row < m) {
                Acc sum = 0;
                for (int c = 0; c < cps; ++c) sum += s_part[(c * lpc + g) * V + v];
                Y[base + row] = (double)sum;
            }
        }
        __syncthreads();
    }
}

// Shapes the set-up autotuner chooses from: U loads in flight per thread.
template <typename T, int U>
void launch_shape(hipStream_t s, const Level& L, const double* r, double* Y) {
    typedef typename Load16<T>::acc_t Acc;
    const int ldbuf = (L.max_m + 1) & ~1;
    const size_t lds = sizeof(Acc) * ((size_t)ldbuf + (size_t)kBlock * Load16<T>::V);
    if (streams_factors(L, L.sym))
        hipLaunchKernelGGL((patch_apply_kernel<T, U, true>), dim3(L.npatch), dim3(kBlock), lds, s, L.order, L.pptr,
                           L.pdofs_perm, L.fofflp, (const T*)L.factors, r, Y, ldbuf);
    else
        hipLaunchKernelGGL((patch_apply_kernel<T, U, false>), dim3(L.npatch), dim3(kBlock), lds, s, L.order, L.pptr,
                           L.pdofs_perm, L.fofflp, (const T*)L.factors, r, Y, ldbuf);
}

template <typename T>
void launch_typed(hipStream_t s, const Level& L, const double* r, double* Y) {
    switch (L.apply_variant) {
        case 1: launch_shape<T, 2>(s, L, r, Y); break;
        case 2: launch_shape<T, 8>(s, L, r, Y); break;
        default: launch_shape<T, 4>(s, L, r, Y);
    }
}


// Symmetric layout, one workgroup per patch.  A wave covers a strip's 16 rows
// with RL = 16 / V row lanes (one 16-byte load each) and CL = 64 / RL column
// lanes; a work unit is one strip times 64 consecutive stored columns, i.e. RL
// loads per lane, each wave-wide load reading 1 KB of contiguous bytes.  Per
// loaded row group (rows i, column j) of the stored entries L (S = L + L^T)
// the lane adds L(i, j) r_j to its row partials and forms L(i, j) . r_i for column j.
// Column sums are scatter-reduced over the row lanes (each lane ends with one
// column), row sums are reduced over the column lanes, and both are added into
// partial result u % 4 in LDS (u the unit's number in strip-major order); units
// are dealt to the waves round-robin and the four partial results are summed in
// order at the end.  PF = true issues the loads of a wave's next unit before
// computing the current one; the arithmetic, and so every bit of the result, is
// the same for every shape.
constexpr int kUnitCols = 64;

template <typename T>
struct SymShape {
    static constexpr int V = Load16<T>::V;
    static constexpr int RL = kStrip / V;
    static constexpr int CL = kWave / RL;
    static constexpr int U = kUnitCols / CL;       // loads per lane per unit (= RL)
};

// next unit position after (s, c): the following 64 columns of the strip, or the next strip
__device__ inline bool sym_step(int& s, int& c, int ns, int m) {
    c += kUnitCols;
    if (c >= min(m, (s + 1) * kStrip)) {
        ++s;
        c = 0;
    }
    return s < ns;
}

// Loads of one unit without branches: a column past the strip's width reads
// the last stored column and a row group past the strip's height the last row
// group (both inside the patch's block, finite values); the caller multiplies
// such loads only by zero residual entries (rows >= m) or drops their sums
// (columns >= w).  In the diagonal block a row group above column c's stored
// groups is not stored: the lane reads the first stored group and zeroes it.
// DIAG: the unit reaches the diagonal block (columns >= 16 s).
template <typename T, bool NT, bool DIAG>
__device__ inline void sym_load(const T* A, int s, int c_lo, int m, int rl, int cl,
                                typename Load16<T>::acc_t (&a)[SymShape<T>::U][SymShape<T>::V]) {
    typedef SymShape<T> Sh;
    typedef typename Load16<T>::acc_t Acc;
    constexpr int V = Sh::V;
    const int r0 = s * kStrip, h = min(kStrip, m - r0), hp = (h + V - 1) / V * V, w = r0 + h;
    const T* S = A + sym_strip_offset(s, V);
    const int rg = min(rl * V, hp - V);
#pragma unroll
    for (int u = 0; u < Sh::U; ++u) {
        const int j = min(c_lo + cl + Sh::CL * u, w - 1);
        int64_t off = (int64_t)j * hp + rg;
        bool above = false;
        if (DIAG && j >= r0) {
            constexpr int PG = sym_pack(V);
            const int c = j - r0, g = c / PG * PG;
            above = rg < g;
            off = (int64_t)hp * r0 + sym_diag_offset(c, hp, PG) + (max(rg, g) - g);
        }
        Load16<T>::template load<NT>(S + off, a[u]);
        if (DIAG && sym_pack(V) < kStrip) {
#pragma unroll
            for (int v = 0; v < V; ++v) a[u][v] = above ? (Acc)0 : a[u][v];
        }
    }
}

// LDS length of the residual and of each partial result in the symmetric
// shapes: whole strips plus one unit, so the unit arithmetic may read rows and
// columns past m (zeros) without bound checks
inline int sym_ldbuf(int max_m) { return (max_m + kStrip - 1) / kStrip * kStrip + kUnitCols; }

// The arithmetic of one unit (strip s, stored columns c .. c + 63, factor
// values in a): with L the stored entries, row sums L(rows, cols) r_cols and
// column sums L(rows, j)^T r_rows, added into the partial result yw.
template <typename T>
__device__ inline void sym_unit(const typename Load16<T>::acc_t (&a)[SymShape<T>::U][SymShape<T>::V], int s, int c,
                                int m, int rl, int cl, int lane, const typename Load16<T>::acc_t* s_r,
                                typename Load16<T>::acc_t* yw) {
    typedef typename Load16<T>::acc_t Acc;
    typedef SymShape<T> Sh;
    constexpr int V = Sh::V, RL = Sh::RL, CL = Sh::CL, U = Sh::U;
    const int r0 = s * kStrip, w = min(m, r0 + kStrip);
    // the residual rows of the lane's row group: s_r is zero past m up to whole
    // strips plus one unit (sym_ldbuf), so no row needs a bound check, and the V
    // values come in one LDS vector read
    typedef Acc accv __attribute__((ext_vector_type(V)));
    const accv rv = *reinterpret_cast<const accv*>(s_r + r0 + rl * V);
    Acc rr[V];
#pragma unroll
    for (int v = 0; v < V; ++v) rr[v] = rv[v];
    Acc acc[V], d[U];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = (Acc)0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = c + cl + CL * u;
        const Acc rj = j < w ? s_r[j] : (Acc)0;
        Acc dd = (Acc)0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            acc[v] += a[u][v] * rj;
            dd += a[u][v] * rr[v];
        }
        d[u] = dd;
    }
    // column sums: scatter-reduce over the RL row lanes; the lane keeps column c + cl + CL * rl
    GroupReduce<Acc, U, RL, 1>::run(d, lane);
    {
        const int j = c + cl + CL * rl;
        if (j < w) yw[j] += d[0];
    }
    // row sums: reduce over the CL column lanes
    GroupReduce<Acc, V, CL, RL>::run(acc, lane);
    if (cl % (CL / V) == 0) {
        const int i = r0 + rl * V + cl / (CL / V);
        if (i < m) yw[i] += acc[0];
    }
}

// one unit's loads, dispatched on whether the unit reaches a packed diagonal
// block (a whole stored diagonal block, bfloat16, continues the column-major strip)
template <typename T, bool NT>
__device__ inline void sym_load_unit(const T* A, int s, int c, int m, int rl, int cl,
                                     typename Load16<T>::acc_t (&a)[SymShape<T>::U][SymShape<T>::V]) {
    if (sym_pack(SymShape<T>::V) < kStrip && c + kUnitCols > s * kStrip) sym_load<T, NT, true>(A, s, c, m, rl, cl, a);
    else sym_load<T, NT, false>(A, s, c, m, rl, cl, a);
}

// NWV wavefronts per workgroup (4, or 1 for levels of small patches, where a
// 4-wave workgroup would leave waves without units).  Unit u always adds into
// partial result u % 4, in increasing u, whichever wave runs it, so both
// shapes give identical bits.
constexpr int kSymParts = 4;

template <typename T, bool PF, int NWV, bool NT>
__global__ __launch_bounds__(kBlock) void patch_apply_sym_kernel(const int64_t* __restrict__ pinfo,
                                                                 const int32_t* __restrict__ pdofs,
                                                                 const T* __restrict__ F,
                                                                 const double* __restrict__ r,
                                                                 const double* __restrict__ gw,
                                                                 double* __restrict__ Y, int ldbuf) {
    typedef typename Load16<T>::acc_t Acc;
    typedef SymShape<T> Sh;
    constexpr int V = Sh::V, RL = Sh::RL, CL = Sh::CL, U = Sh::U;
    constexpr int NP = kSymParts, NTH = NWV * kWave;
    static_assert(V == factor_pad<T>() && U == RL && CL % V == 0, "strip and reduction shapes");
    static_assert(NP % NWV == 0, "unit classes per wave");
    extern __shared__ double s_buf[];
    Acc* s_r = reinterpret_cast<Acc*>(s_buf);
    Acc* s_y = s_r + ldbuf;                                       // NP partial results of ldbuf each
    // the patch at this launch position: first slot, factor offset and size in one read
    const int64_t* info = pinfo + 4 * (int64_t)blockIdx.x;
    const int64_t base = info[0];
    const T* A = F + info[1];
    const int m = (int)info[2];
    // the wave index as a wave-uniform value, so the walk over the wave's units
    // (s, c, sym_step) stays in scalar registers
    const int lane = threadIdx.x & (kWave - 1), wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int rl = lane % RL, cl = lane / RL;
    const int ns = (m + kStrip - 1) / kStrip;
    // this wave's first unit (unit number `wave` in strip-major order): its
    // factor loads are issued before the residual gather, which they do not need
    int s = 0, c = 0, unit = wave;
    bool ok = true;
    for (int q = 0; q < wave && ok; ++q) ok = sym_step(s, c, ns, m);
    Acc a[U][V];
    if (ok) sym_load_unit<T, NT>(A, s, c, m, rl, cl, a);
    for (int t = threadIdx.x; t < m; t += NTH) {
        const double v = r[pdofs[base + t]];
        s_r[t] = (Acc)(gw ? gw[base + t] * v : v);
    }
    for (int t = m + threadIdx.x; t < ldbuf; t += NTH) s_r[t] = (Acc)0;
    for (int t = threadIdx.x; t < NP * ldbuf; t += NTH) s_y[t] = (Acc)0;
    __syncthreads();
    bool first = true;
    while (ok) {
        int s2 = s, c2 = c;
        bool ok2 = true;
        for (int q = 0; q < NWV && ok2; ++q) ok2 = sym_step(s2, c2, ns, m);
        Acc* yw = s_y + (unit % NP) * ldbuf;
        Acc b[U][V];
        if (PF) {
            if (ok2) sym_load_unit<T, NT>(A, s2, c2, m, rl, cl, b);
        } else if (!first) {
            sym_load_unit<T, NT>(A, s, c, m, rl, cl, a);
        }
        first = false;
        sym_unit<T>(a, s, c, m, rl, cl, lane, s_r, yw);
        s = s2;
        c = c2;
        ok = ok2;
        unit += NWV;
        if (PF) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int v = 0; v < V; ++v) a[u][v] = b[u][v];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < m; t += NTH) {
        Acc sum = s_y[t];
#pragma unroll
        for (int q = 1; q < NP; ++q) sum += s_y[q * ldbuf + t];
        Y[base + t] = (double)sum;
    }
}

// Levels of small patches (at most kSmallUnits units, i.e. m <= 64): one wave
// per patch loads every unit of its patch before the residual gather, so a
// patch costs one memory latency instead of a chain of them.  Unit k adds into
// partial k % 4 as in patch_apply_sym_kernel, so the bits are the same.
constexpr int kSmallUnits = 4;

template <typename T, bool NT>
__global__ __launch_bounds__(kBlock) void patch_apply_sym_small_kernel(const int64_t* __restrict__ pinfo,
                                                                       const int32_t* __restrict__ pdofs,
                                                                       const T* __restrict__ F,
                                                                       const double* __restrict__ r,
                                                                       const double* __restrict__ gw,
                                                                       double* __restrict__ Y, int ldbuf) {
    typedef typename Load16<T>::acc_t Acc;
    typedef SymShape<T> Sh;
    constexpr int V = Sh::V, RL = Sh::RL, U = Sh::U, NU = kSmallUnits, NP = kSymParts;
    extern __shared__ double s_buf[];
    Acc* s_r = reinterpret_cast<Acc*>(s_buf);
    Acc* s_y = s_r + ldbuf;
    const int64_t* info = pinfo + 4 * (int64_t)blockIdx.x;   // the patch at this launch position
    const int64_t base = info[0];
    const T* A = F + info[1];
    const int m = (int)info[2];
    const int lane = threadIdx.x & (kWave - 1);
    const int rl = lane % RL, cl = lane / RL;
    const int ns = (m + kStrip - 1) / kStrip;
    Acc a[NU][U][V];
    int su[NU], cu[NU];
    bool oku[NU];
    int s = 0, c = 0;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        su[k] = s;
        cu[k] = c;
        oku[k] = ok;
        if (ok) {
            sym_load_unit<T, NT>(A, s, c, m, rl, cl, a[k]);
            ok = sym_step(s, c, ns, m);
        }
    }
    for (int t = lane; t < m; t += kWave) {
        const double v = r[pdofs[base + t]];
        s_r[t] = (Acc)(gw ? gw[base + t] * v : v);
    }
    for (int t = m + lane; t < ldbuf; t += kWave) s_r[t] = (Acc)0;
    for (int t = lane; t < NP * ldbuf; t += kWave) s_y[t] = (Acc)0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NU; ++k)
        if (oku[k]) sym_unit<T>(a[k], su[k], cu[k], m, rl, cl, lane, s_r, s_y + (k % NP) * ldbuf);
    __syncthreads();
    for (int t = lane; t < m; t += kWave) {
        Acc sum = s_y[t];
#pragma unroll
        for (int q = 1; q < NP; ++q) sum += s_y[q * ldbuf + t];
        Y[base + t] = (double)sum;
    }
}

template <typename T>
void launch_sym_small(hipStream_t s, const Level& L, const double* r, const double* gw, double* Y) {
    typedef typename Load16<T>::acc_t Acc;
    const int ldbuf = sym_ldbuf(L.max_m);
    const size_t lds = sizeof(Acc) * (size_t)ldbuf * (1 + kSymParts);
    if (streams_factors(L, L.sym))
        hipLaunchKernelGGL((patch_apply_sym_small_kernel<T, true>), dim3(L.npatch), dim3(kWave), lds, s, L.pinfo,
                           L.pdofs, (const T*)L.factors, r, gw, Y, ldbuf);
    else
        hipLaunchKernelGGL((patch_apply_sym_small_kernel<T, false>), dim3(L.npatch), dim3(kWave), lds, s, L.pinfo,
                           L.pdofs, (const T*)L.factors, r, gw, Y, ldbuf);
}

template <typename T, bool PF, int NWV>
void launch_sym_shape(hipStream_t s, const Level& L, const double* r, const double* gw, double* Y) {
    typedef typename Load16<T>::acc_t Acc;
    const int ldbuf = sym_ldbuf(L.max_m);
    const size_t lds = sizeof(Acc) * (size_t)ldbuf * (1 + kSymParts);
    if (streams_factors(L, L.sym)) {
        hipLaunchKernelGGL((patch_apply_sym_kernel<T, PF, NWV, true>), dim3(L.npatch), dim3(NWV * kWave), lds, s,
                           L.pinfo, L.pdofs, (const T*)L.factors, r, gw, Y, ldbuf);
    } else {
        hipLaunchKernelGGL((patch_apply_sym_kernel<T, PF, NWV, false>), dim3(L.npatch), dim3(NWV * kWave), lds, s,
                           L.pinfo, L.pdofs, (const T*)L.factors, r, gw, Y, ldbuf);
    }
}

// shapes: 0 / 1 four waves without / with prefetch, 2 / 3 one wave without / with prefetch,
// 4 (levels whose patches have at most 64 DoFs) one wave with every unit loaded ahead
template <typename T>
void launch_sym_typed(hipStream_t s, const Level& L, const double* r, const double* gw, double* Y) {
    switch (L.apply_variant) {
        case 4: launch_sym_small<T>(s, L, r, gw, Y); break;
        case 1: launch_sym_shape<T, true, 4>(s, L, r, gw, Y); break;
        case 2: launch_sym_shape<T, false, 1>(s, L, r, gw, Y); break;
        case 3: launch_sym_shape<T, true, 1>(s, L, r, gw, Y); break;
        default: launch_sym_shape<T, false, 4>(s, L, r, gw, Y);
    }
}

}  // namespace

int apply_variant_count(const Level& L) {
    // a patch of at most 64 DoFs has at most 4 strips of one 64-column unit each
    if (L.sym) return L.max_m <= 64 ? 5 : 4;
    return 3;
}

void launch_patch_apply_sym(hipStream_t s, const Level& L, const double* r, const double* gw, double* Y) {
    if (L.npatch <= 0) return;
    if (!Y) Y = L.Y;
    if (L.prec == PHMG_PREC_F32) launch_sym_typed<float>(s, L, r, gw, Y);
    else if (L.prec == PHMG_PREC_BF16) launch_sym_typed<__hip_bfloat16>(s, L, r, gw, Y);
    else launch_sym_typed<double>(s, L, r, gw, Y);
}

void launch_patch_apply(hipStream_t s, const Level& L, const double* r, double* Y) {
    if (L.npatch <= 0) return;
    if (!Y) Y = L.Y;
    if (L.sym) {
        launch_patch_apply_sym(s, L, r, nullptr, Y);
        return;
    }
    if (L.prec == PHMG_PREC_F32) launch_typed<float>(s, L, r, Y);
    else if (L.prec == PHMG_PREC_BF16) launch_typed<__hip_bfloat16>(s, L, r, Y);
    else launch_typed<double>(s, L, r, Y);
}

}  // namespace phmg
