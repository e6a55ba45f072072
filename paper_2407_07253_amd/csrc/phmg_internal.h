// Internal declarations of the gfx950 phMG library: device-side level data,
// the context, and the kernel launchers shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/phmg.h"

namespace phmg {

constexpr int kBlock = 256;          // threads per workgroup (4 wavefronts of 64)
constexpr int kWave = 64;
constexpr int kPanel = 16;           // Gauss-Jordan panel width = MFMA f64 16x16x4 tile edge
constexpr int kRedBlocks = 512;      // fixed grid of the deterministic reductions
constexpr int kBlockGsBlocks = 2048; // fixed grid of the block Gram-Schmidt passes (8 waves per SIMD)
constexpr int kBS = 16;              // columns of a block vector (right-hand sides solved together)
constexpr int kRbRows = 32;          // rows of an SpMV row block (8 lanes per row)
constexpr int kRbNnz = 1024;         // nonzeros of an SpMV row block (4 per thread)

// Leading dimension padding of the stored patch inverses: every column is
// padded to a multiple of 16 bytes (f64: 2 rows, f32: 4, bf16: 8; padding rows
// are zero) so the kernels issue aligned 16-byte loads.  (The set-up's own
// float64 work buffer is unpadded, m x m.)
template <typename T>
__host__ __device__ constexpr int factor_pad() { return 16 / (int)sizeof(T); }
inline int factor_pad_of(int prec) { return prec == PHMG_PREC_F64 ? 2 : (prec == PHMG_PREC_F32 ? 4 : 8); }

// Symmetric layout of a patch inverse S (used when the level matrix is
// symmetric): the rows are cut into strips of kStrip rows; strip s (rows
// [r0, r0 + h), r0 = 16 s) stores, with its height padded to the 16-byte row
// group V (hp = h rounded up to V, padding rows zero):
//   * the strictly lower part, columns [0, r0), column-major hp x r0;
//   * then its diagonal block D: column c (c < h) holds rows [g(c), hp) with
//     g(c) = c rounded down to the packing group PG = sym_pack(V) -- the row
//     group V for float64 / float32, the whole block for bfloat16, whose
//     kernels would spend more on the packed addressing than they save -- and
//     D(q, c) for q > c, D(c, c) / 2 on the diagonal, zero for the q < c that
//     fall inside the stored rows.  Column c starts at sym_diag_offset(c, hp, PG).
// With L the stored entries of all strips, S = L + L^T exactly (halving is
// exact), so a kernel adds both L r and L^T r over every stored entry alike.
// Strips are consecutive; a full strip takes 256 s + sym_diag_offset(16, 16, PG)
// elements (144 / 160 / 256 in the diagonal block for float64 / float32 / bfloat16).
constexpr int kStrip = 16;
__host__ __device__ constexpr int sym_pack(int V) { return V < 8 ? V : kStrip; }
__host__ __device__ constexpr int sym_diag_offset(int c, int hp, int PG) {
    return PG * (c / PG) * hp - PG * PG * (c / PG) * (c / PG - 1) / 2 + (c % PG) * (hp - (c / PG) * PG);
}
__host__ __device__ constexpr int64_t sym_strip_offset(int s, int V) {
    return (int64_t)128 * s * (s - 1) + (int64_t)sym_diag_offset(kStrip, kStrip, sym_pack(V)) * s;
}
__host__ __device__ inline int64_t sym_layout_size(int m, int V) {
    const int ns = (m + kStrip - 1) / kStrip;
    const int h = m - (ns - 1) * kStrip, hp = (h + V - 1) / V * V;
    return sym_strip_offset(ns - 1, V) + (int64_t)hp * kStrip * (ns - 1) + sym_diag_offset(h, hp, sym_pack(V));
}

struct DevCsr {
    int32_t nrows = 0, ncols = 0;
    int64_t nnz = 0;
    int32_t* rowptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
    int group = 8;                   // lanes per row in the SpMV (chosen by the set-up autotuner)
    bool xcd = false;                // XCD-contiguous row ranges in the SpMV (autotuned)
    bool tuned = false;
    // row blocks of at most kRbRows rows and kRbNnz nonzeros (absent when a row is longer)
    int32_t nrb = 0;
    int32_t* rblk = nullptr;         // nrb + 1 block boundaries (row indices)
    bool rowblock = false;           // SpMV kernel: row-block (else CSR with `group` lanes per row); autotuned
    int unroll = 4;                  // CSR SpMV: entries in flight per lane (4 or 8; autotuned)
    bool vec = false;                // CSR SpMV with 4 consecutive entries per lane (16-byte loads; autotuned)
    int bgroup = 1;                  // entries in flight per row in the block SpMM (autotuned on first use)
    bool bxcd = false;               // XCD-contiguous row ranges in the block SpMM (autotuned)
    int bquad = 0;                   // block SpMM with bquad (2 or 4) lanes per row, 16 / bquad columns of X
                                     // per lane, or 0: bgroup groups of 16 lanes per row (autotuned)
    bool btuned = false;
};

struct Level {
    int32_t n = 0;
    DevCsr K;
    DevCsr KT;                       // K^T (shares K's arrays when K is symmetric)
    DevCsr P;                        // prolongation from level+1 into this level (n x n_{l+1})
    DevCsr R;                        // restriction R = P^T (n_{l+1} x n)
    DevCsr RK;                       // R K (n_{l+1} x n): the restricted residual R b - (R K) x in one pass
    bool fuse_restrict = false;      // use RK (autotuned against the two-step residual + restriction)

    // Vanka-star patches (absent on the coarsest level)
    int32_t npatch = 0;
    int32_t max_m = 0;
    int64_t sum_m = 0, sum_m2 = 0;
    int64_t* pptr = nullptr;         // npatch + 1
    int32_t* pdofs = nullptr;        // sum_m
    int32_t* pdofs_perm = nullptr;   // sum_m: pdofs permuted by each patch's pivoting (gather of P r)
    int32_t* pidx = nullptr;         // sum_m: the pivoting permutation as local positions (P r)_t = r[pidx[t]]
    double* ptol = nullptr;          // npatch: singularity threshold 1e-14 ||K_i||_inf
    double* pweight = nullptr;       // sum_m or null (W_i = I)
    int64_t* foff = nullptr;         // offset of patch i's m_i x m_i block in the set-up buffer (ld = m)
    int64_t* fofflp = nullptr;       // offsets of the stored inverses (general: ld = m rounded up to
                                     // factor_pad; symmetric: strip layout)
    int64_t sum_lp[3] = {0, 0, 0};   // element counts of the stored f64 / f32 / bf16 layouts
    int64_t sum_ls[3] = {0, 0, 0};   // the same for the symmetric (strip) layout
    bool sym_ok = false;             // K is symmetric to rounding (entries within 1e-12 of the row scale)
    int storage = PHMG_STORAGE_AUTO; // requested layout of the stored inverses
    bool sym = false;                // the stored inverses use the symmetric strip layout
    int32_t* order = nullptr;        // launch order: patches by decreasing size
    std::vector<int32_t> horder;     // host copy of order
    int64_t* pinfo = nullptr;        // per launch position k: pptr[p], fofflp[p], m, p (p = order[k]),
                                     // so the patch solve reads its patch without the order indirection
    // patch inversion kernels by size class, over consecutive ranges of the launch order:
    // gj_cnt[0] patches inverted with the matrix in global memory (more than 144 DoFs),
    // gj_cnt[1..2] of 97-144 and 65-96 DoFs (matrix in registers), gj_cnt[3] of at most 64 (in LDS)
    int32_t gj_cnt[4] = {0, 0, 0, 0};
    int32_t gj_max[4] = {0, 0, 0, 0};      // largest patch of each class
    int32_t* sptr = nullptr;         // DoF -> slot map for the scatter (n + 1)
    int32_t* sslot = nullptr;        // sum_m slot indices, ascending patch id per DoF
    int32_t* sslot4 = nullptr;       // n x 4: each DoF's first four slots (-1 padded), read without sptr
    double* wdof = nullptr;          // n: the partition weight of each DoF when all its slots share one
                                     // (the scatter then scales the sum once); null: per-slot weights
    double* Y = nullptr;             // sum_m staging of the patch solutions
    void* factors = nullptr;         // explicit patch inverses in the stored layout, precision `prec`
    size_t factor_bytes = 0;         // allocated size of `factors` (kept across set-ups)
    double* work64 = nullptr;        // float64 set-up buffer, m x m per patch (kept across set-ups)
    std::vector<int64_t> hptr;       // host copy of pptr
    int prec = PHMG_PREC_F64;
    int apply_variant = 0;           // kernel shape of the patch solve (chosen by the set-up autotuner)
    int tuned_for = -1;              // precision the shape was tuned for

    // coarsest level: dense inverse of the (bordered) matrix, row-major
    double* cinv = nullptr;
    double* cnull = nullptr;
    double* cdense = nullptr;        // set-up work of the coarse inversion (kept across set-ups)
    int* cpiv = nullptr;
    double* cwork = nullptr;
    int32_t nb = 0;                  // n or n + 1

    // Chebyshev smoothing: direction vector and the eigenvalue estimate
    double* d = nullptr;
    double lmax = 0.0;

    // V-cycle work vectors
    double* r = nullptr;
    double* b = nullptr;
    double* x = nullptr;

    int* status = nullptr;           // device: smallest singular patch id (INT32_MAX = none)
    double* arn = nullptr;           // Arnoldi work space of the set-up (basis, w, partials, projections)
    int64_t arn_len = 0;
    bool ready = false;

    // block (multi-right-hand-side) work space, n x kBS interleaved, allocated on first use
    double* rb = nullptr;
    double* bb = nullptr;
    double* xb = nullptr;
    double* db = nullptr;
    double* Yb = nullptr;            // sum_m x kBS staging of the block patch solutions
    int block_variant = 0;           // kernel shape of the block patch solve (autotuned)
    int block_tuned_for = -1;
    // the block path always streams the general layout: on symmetric levels a
    // general copy is converted from the f64 set-up buffer on first block use
    // after each set-up
    void* bfactors = nullptr;
    size_t bfactor_bytes = 0;
    int64_t* bfoff = nullptr;
    int64_t setup_count = 0;         // completed set-ups of the level
    int64_t bconv_count = -1;        // set-up whose factors the general copy holds
};

// FGMRES work space: bases V (n x cap+1) and Z (n x cap), work vectors, the
// reduction partials and the device / pinned host scalars of one iteration.
struct Krylov {
    int cap = 0;
    int64_t n = 0;
    double* V = nullptr;
    double* Z = nullptr;
    double* w = nullptr;
    double* r = nullptr;
    double* partial = nullptr;       // kRedBlocks x (restart + 2) reduction partials
    int partial_cols = 0;
    double* hdev = nullptr;          // device scalars: h (restart + 1), h', ||w||^2
    double* hhost = nullptr;         // pinned host mirror, two slots (iterations alternate)
    hipEvent_t ev[2] = {nullptr, nullptr};   // "slot ready" events of the two host slots
};

struct Profile {
    unsigned mask = 0;
    double ms[PHMG_K_COUNT][PHMG_MAX_LEVELS] = {{0}};
    int64_t count[PHMG_K_COUNT][PHMG_MAX_LEVELS] = {{0}};
    struct Pending {
        int kernel, level;
        hipEvent_t e0, e1;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
};

}  // namespace phmg

struct phmg_ctx_s {
    hipStream_t stream = nullptr;
    int device = 0;                  // the HIP device current at create (owner of every buffer)
    std::vector<phmg::Level> L;
    phmg_cycle_opts opts{};
    std::vector<void*> allocs;
    // FGMRES / Arnoldi work space (level 0)
    phmg::Krylov kry;
    double* scal = nullptr;          // device scalars (norms) outside FGMRES
    phmg::Profile prof;
    // the preconditioner (one V-cycle) captured as a HIP graph on fixed buffers
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    hipGraph_t vgraph[2] = {nullptr, nullptr};      // [0] B, [1] B^T (adjoint cycle)
    hipGraphExec_t vexec[2] = {nullptr, nullptr};
    std::vector<uint64_t> vsig[2];                  // graph_signature() when each graph was captured
    struct SlotGraph {                              // a V-cycle captured straight on FGMRES basis slots
        const double* b;
        double* x;
        int t;
        std::vector<uint64_t> sig;
        hipGraph_t g;
        hipGraphExec_t e;
    };
    std::vector<SlotGraph> sgraphs;
    // set-up: one stream per level (default priority), fork / join events and
    // pinned status words
    std::vector<hipStream_t> sstreams;
    hipEvent_t fork_ev[2] = {nullptr, nullptr};   // large-patch inversion on a second stream
    std::vector<hipEvent_t> sevents;                // [0] fork, [1 + l] join of level l
    int32_t* status_host = nullptr;
    double* gin = nullptr;
    double* gout = nullptr;
    // kernel vector z of K_0 (set_kernel_vector) and the work space of its projection
    double* z0 = nullptr;
    double z0z0 = 0.0;
    double* zpartial = nullptr;      // kRedBlocks x kBS
    double* zdots = nullptr;         // kBS
    // adjoint gradients: dK/dtheta over K_0's nonzeros, the forcing map G and G^T
    bool have_sens = false;
    phmg::DevCsr S, G, GT;
    double* wpair = nullptr;         // nnz(K_0) products of the gradient contraction
    // block path: work vectors, FGMRES block basis and its captured V-cycle
    bool block_ready = false;
    int brestart_cap = 0;
    double* Vb = nullptr;
    double* Zb = nullptr;
    double* wb = nullptr;
    double* rvb = nullptr;
    double* bpartial = nullptr;      // kBlockGsBlocks x 32 x kBS
    double* bh = nullptr;            // device: h1 | h2 | hn2 | column scales
    double* bhhost = nullptr;        // pinned mirror of bh
    double* bgin = nullptr;
    double* bgout = nullptr;
    hipGraph_t bgraph[2] = {nullptr, nullptr};      // [0] block B, [1] block B^T
    hipGraphExec_t bexec[2] = {nullptr, nullptr};
    std::vector<uint64_t> bsig[2];
};

// The full-block-factorisation preconditioner: a velocity-block hierarchy (its
// own context) plus the saddle-point pieces and work vectors.
struct phmg_fbf_s {
    phmg_ctx A = nullptr;            // velocity-block hierarchy (not owned)
    phmg_ctx_s mem;                  // owner of the buffers below
    phmg::DevCsr K, B, BT, Sinv;
    int64_t n = 0, nu = 0, np = 0;
    double* yu = nullptr;
    double* t = nullptr;
    double* wu = nullptr;
    double* qu = nullptr;
    phmg::Krylov kry;
};

namespace phmg {

// Exchange with the lane whose id differs by MASK: lane-pair swaps inside a quad
// (MASK 1, 2) and the half-row rotation (MASK 8) are DPP moves on the VALU;
// other masks go through ds_bpermute.
// The wave's index in its workgroup as a wave-uniform value: the compiler then
// keeps loops and branches over it in scalar registers instead of running them
// under execution masks.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); }

template <int MASK>
__device__ inline float xor_shfl(float v) {
    if constexpr (MASK == 1 || MASK == 2 || MASK == 8) {
        constexpr int ctrl = MASK == 1 ? 0xB1 : (MASK == 2 ? 0x4E : 0x128);   // quad_perm / row_ror:8
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, false));
    } else {
        return __shfl_xor(v, MASK);
    }
}
template <int MASK>
__device__ inline double xor_shfl(double v) {
    if constexpr (MASK == 1 || MASK == 2 || MASK == 8) {
        constexpr int ctrl = MASK == 1 ? 0xB1 : (MASK == 2 ? 0x4E : 0x128);
        const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, 0xF, 0xF, false);
        return __hiloint2double(hi, lo);
    } else {
        return __shfl_xor(v, MASK);
    }
}

// One butterfly step across 32 (MASK 32) or 16 (MASK 16) lanes for a pair of
// values (lo, hi): the lane whose MASK bit is clear keeps lo and adds its
// partner's lo, the other keeps hi and adds its partner's hi.  The gfx950
// lane-swap instructions do the exchange for both values at once: after
// v_permlane32_swap (v_permlane16_swap) of (lo, hi) the two registers hold, in
// every lane, the kept value and the partner's copy of it (in one order or the
// other; the sum is the same bits either way).
template <int MASK>
__device__ inline float swap_sum(float lo, float hi) {
    static_assert(MASK == 16 || MASK == 32, "lane-swap distance");
    if constexpr (MASK == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
}
template <int MASK>
__device__ inline double swap_sum(double lo, double hi) {
    static_assert(MASK == 16 || MASK == 32, "lane-swap distance");
    const uint32_t l0 = (uint32_t)__double2loint(lo), l1 = (uint32_t)__double2hiint(lo);
    const uint32_t h0 = (uint32_t)__double2loint(hi), h1 = (uint32_t)__double2hiint(hi);
    if constexpr (MASK == 32) {
        const auto a = __builtin_amdgcn_permlane32_swap(l0, h0, false, false);
        const auto b = __builtin_amdgcn_permlane32_swap(l1, h1, false, false);
        return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
    } else {
        const auto a = __builtin_amdgcn_permlane16_swap(l0, h0, false, false);
        const auto b = __builtin_amdgcn_permlane16_swap(l1, h1, false, false);
        return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
    }
}

// Sum of N values over groups of G lanes (lane ids that differ only in the
// bits of (lane / STRIDE) % G), as a butterfly that first scatters: while more
// than one value is left, each level keeps half of the list (the upper half in
// the lane whose bit is set) and adds the partner's copy of that half.  On
// return, for N >= G, the lane with q = (lane / STRIDE) % G holds in x[0 ..
// N / G) the group sums of elements [q N / G, (q + 1) N / G); for N < G it
// holds in x[0] the sum of element q / (G / N).  The pairing is fixed, so the
// result is deterministic.  Every lane of the wave must be active.
template <typename Acc, int N, int G, int STRIDE>
struct GroupReduce {
    __device__ static inline void run(Acc* x, int lane) {
        if constexpr (G > 1) {
            constexpr int g = G / 2;
            if constexpr (N > 1) {
                constexpr int h = N / 2;
                if constexpr (g * STRIDE == 16 || g * STRIDE == 32) {
#pragma unroll
                    for (int e = 0; e < h; ++e) x[e] = swap_sum<g * STRIDE>(x[e], x[e + h]);
                } else {
                    const bool up = ((lane / STRIDE) & g) != 0;
#pragma unroll
                    for (int e = 0; e < h; ++e) {
                        const Acc lo = x[e], hi = x[e + h];
                        const Acc other = xor_shfl<g * STRIDE>(up ? lo : hi);
                        x[e] = (up ? hi : lo) + other;
                    }
                }
                GroupReduce<Acc, h, g, STRIDE>::run(x, lane);
            } else {
                x[0] += xor_shfl<g * STRIDE>(x[0]);
                GroupReduce<Acc, 1, g, STRIDE>::run(x, lane);
            }
        }
    }
};

// Every host-side value a captured V-cycle bakes into its kernel arguments
// (buffers, kernel variants, precisions, layouts, Chebyshev intervals, cycle
// options): a graph is replayed only while this is unchanged.
std::vector<uint64_t> graph_signature(phmg_ctx ctx);

// ---- launchers (kernels.hip) ------------------------------------------------
void launch_fill(hipStream_t s, int64_t n, double* x, double v);
void launch_fill_i32(hipStream_t s, int64_t n, int32_t* x, int32_t v);
// y = alpha * A x + beta * z   (z may be null, or alias y)
void launch_spmv(hipStream_t s, const DevCsr& A, const double* x, double alpha, const double* z, double beta,
                 double* y);
// y = A1 x1 - A2 x2 for two matrices with the same rows (lanes per row: A2.group)
void launch_spmv_diff(hipStream_t s, const DevCsr& A1, const double* x1, const DevCsr& A2, const double* x2,
                      double* y);
void launch_extract(hipStream_t s, const Level& L, double* out);
// invert every patch matrix of the level in place (stored as (P K_i)^{-1}, see kernels.hip).
// aux (optional): a second stream for the patches above 144 DoFs, forked from s with ev_fork and
// joined back into s with ev_join, so they run beside the register-resident kernel
void launch_patch_factor(hipStream_t s, const Level& L, double* A, hipStream_t aux = nullptr,
                         hipEvent_t ev_fork = nullptr, hipEvent_t ev_join = nullptr);
int gj_lds_max_m();   // largest patch the LDS-resident inversion takes
int gj_reg_max_m();   // largest patch the register-resident inversion takes (patch_factor.hip)
// register-resident inversion of the launch-order range [first, first + count), patches of at most max_m DoFs
void launch_patch_factor_reg(hipStream_t s, const Level& L, double* A, int first, int count, int max_m);
// size class of a patch for the inversion kernels (index into Level::gj_cnt): 0 above 144 DoFs
// (global-memory kernel), 1 for 97-144 and 2 for 65-96 (register-resident kernel), 3 up to 64
// (LDS-resident kernel).  (max_m is kept for callers; the classes depend on m alone.)
inline int gj_class(int64_t m, int64_t /*max_m*/) {
    if (m > 144) return 0;
    return m > 96 ? 1 : (m > 64 ? 2 : 3);
}
void launch_convert_patches(hipStream_t s, const Level& L, const double* src, void* dst);
// general layout (offsets off) from the f64 set-up buffer, whatever the level's stored layout
void launch_convert_general(hipStream_t s, const Level& L, const double* src, void* dst, const int64_t* off);
// Y: where the patch results go (null: the level's own staging L.Y, sum_m doubles)
void launch_patch_apply(hipStream_t s, const Level& L, const double* r, double* Y = nullptr);
// adjoint patch solve y_i = K_i^{-T} W_i r[S_i] from the same stored inverses (adjoint_kernels.hip)
// Patch inverses of more than kStreamBytes (in the given layout and the level's
// precision) are read with non-temporal loads: a stream that size would only
// evict, from the 256 MB last-level cache, the level matrix and vectors the
// rest of the cycle reads; smaller levels keep normal loads, so their factors
// can stay cached across a cycle's sweeps.
constexpr size_t kStreamBytes = size_t(64) << 20;
inline bool streams_factors(const Level& L, bool sym_layout) {
    const size_t es = L.prec == PHMG_PREC_F64 ? 8 : (L.prec == PHMG_PREC_F32 ? 4 : 2);
    return es * (size_t)(sym_layout ? L.sum_ls[L.prec] : L.sum_lp[L.prec]) > kStreamBytes;
}
void launch_patch_apply_t(hipStream_t s, const Level& L, const double* r);
int apply_variant_count(const Level& L);
// symmetric layout: y_i = S_i (g_i * r[S_i]) with g_i = W_i (gw != null, the adjoint sweep) or I
void launch_patch_apply_sym(hipStream_t s, const Level& L, const double* r, const double* gw, double* Y = nullptr);
// dn = a * sum_t w_t Y_t + c * d;  x = (x_zero ? 0 : x) + dn;  d = dn if store_d
// (c = 0: d is not read; d may be null when c = 0 and !store_d)
// transpose: the adjoint sweep's scatter (weights W_i were applied at the gather);
// Y: the staged patch results (null: L.Y)
void launch_scatter(hipStream_t s, const Level& L, double a, double c, double* d, bool store_d, double* x,
                    bool x_zero, bool transpose = false, const double* Y = nullptr);
void launch_power_start(hipStream_t s, int64_t n, double* v);
void launch_scale_by_devnorm(hipStream_t s, int64_t n, const double* src, const double* norm2, double* dst);
void launch_coarse_build(hipStream_t s, const Level& L, double* dense);
int coarse_panel_width(int N);   // 0 when N is too large for the dense coarse solve
// in-place inverse of a column-major N x N matrix over the whole GPU (status: INT32_MAX = ok);
// work holds (1 + kPanel) * N doubles
void launch_dense_gj(hipStream_t s, double* A, int N, int* piv, int* status, double* tol, double* work);
void launch_transpose(hipStream_t s, int n, const double* src, double* dst);
void launch_coarse_solve(hipStream_t s, const Level& L, const double* b, double* x);
// x[i] = sum_{j < n} rows[i * nb + j] b[j] (one wave per row)
void launch_coarse_solve_rows(hipStream_t s, const Level& L, const double* rows, const double* b, double* x);
void launch_coarse_solve_t(hipStream_t s, const Level& L, const double* b, double* x);   // transposed
// w_e = sum_c Lam_c[i_e] X_c[j_e] over the nonzeros of K (systems of length K.nrows one after another)
void launch_pair_products(hipStream_t s, const DevCsr& K, int nrhs, const double* X, const double* Lam,
                          double* w);
// FGMRES helpers
// out[c] = V[:, c] . w (c < ncol); partial holds kRedBlocks x ncol doubles
void launch_multidot(hipStream_t s, int64_t n, int ncol, const double* V, int64_t ldv, const double* w,
                     double* partial, double* out);
// w -= V h (ncol <= gs_max_cols()), then out = V^T w (ncol values) or, with norm, out[0] = w . w
void launch_gs_update(hipStream_t s, int64_t n, int ncol, const double* V, int64_t ldv, const double* h, double* w,
                      double* partial, double* out, bool norm);
int gs_max_cols();
void launch_gemv_sub(hipStream_t s, int64_t n, int ncol, const double* V, int64_t ldv, const double* h, double* w);
// X_c <- X_c - (z . X_c / zz) z for nrhs systems of length n (one after another); partial holds
// kRedBlocks x nrhs doubles, dots nrhs
void launch_project_off(hipStream_t s, int64_t n, int nrhs, double* X, const double* z, double zz, double* partial,
                        double* dots);
void launch_gemv_add(hipStream_t s, int64_t n, int ncol, const double* Z, int64_t ldz, const double* y, double* x);
void launch_scale_copy(hipStream_t s, int64_t n, const double* src, double denom, double* dst);  // dst = src / denom
void launch_copy(hipStream_t s, int64_t n, const double* src, double* dst);
void launch_axpby(hipStream_t s, int64_t n, double a, const double* x, double b, const double* y, double* z);

// nu relaxation sweeps on level l with explicit work buffers (phmg.hip): r and d
// of n doubles (residual, Chebyshev direction), Y of sum_m doubles (staged patch
// results); every buffer is written before it is read.  profile = false records
// no timing events even when profiling is enabled.
void relax_level(phmg_ctx ctx, int l, const double* b, double* x, int nu, bool x_zero, bool transpose, double* r,
                 double* d, double* Y, bool profile);
// resolve the allocation-free entry point's device array on the current device (noalloc.hip)
void noalloc_init_current_device();

// drop the captured block V-cycle (block.hip); called whenever set-up changes
void invalidate_block_graph(phmg_ctx ctx);

// ---- block launchers (block_kernels.hip): n x kBS interleaved vectors ---------
void launch_spmm(hipStream_t s, const DevCsr& A, const double* X, double alpha, const double* Z, double beta,
                 double* Y);
// transpose: Y_i = K_i^{-T} W_i X[S_i] (symmetric levels only: the general copy's K_i^{-1} with the
// weights at the gather)
void launch_block_apply(hipStream_t s, const Level& L, const double* X, bool transpose = false);
int block_variant_count(const Level& L);
// blocks of 16 rows per patch the symmetric-layout block solve is compiled for on this level
// (4, 9 or 14), or 0 when the level's block path streams the general layout
int block_sym_blocks(const Level& L);
// the symmetric-layout block solve of a level with block_sym_blocks(L) > 0, per factor precision
// (Y_i = S_i X[S_i, :] into L.Yb; gw: DoF weights applied to the gather, adjoint sweep)
void launch_block_sym_f64(hipStream_t s, const Level& L, const double* X, const double* gw);
void launch_block_sym_f32(hipStream_t s, const Level& L, const double* X, const double* gw);
void launch_block_sym_bf16(hipStream_t s, const Level& L, const double* X, const double* gw);
void launch_block_scatter(hipStream_t s, const Level& L, double a, double c, double* d, bool store_d, double* X,
                          bool x_zero, bool transpose = false);
void launch_block_coarse_solve(hipStream_t s, const Level& L, const double* B, double* X, bool transpose = false);
// mode 0: h = V^T w;  1: w -= V h, then h' = V^T w;  2: w -= V h, then ||w||^2 (per column)
void launch_block_gs(hipStream_t s, int mode, int64_t n, int ncol, const double* V, int64_t ldv, double* w,
                     const double* h, double* partial, double* out);
int block_gs_max_basis();
void launch_block_gemv_add(hipStream_t s, int64_t n, int ncol, const double* Z, int64_t ldz, const double* y,
                           double* X);
void launch_block_scale(hipStream_t s, int64_t n, const double* S, const double* cs, double* D);
void launch_interleave(hipStream_t s, int64_t n, int nrhs, const double* src, double* dst);
void launch_deinterleave(hipStream_t s, int64_t n, int nrhs, const double* src, double* dst);

}  // namespace phmg
