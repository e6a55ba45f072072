// Host runtime of the gfx950 phMG library: the C ABI declared in include/phmg.h.
//
// Validation and index preprocessing (R = P^T, DoF -> patch-slot map, launch
// order, factor offsets) run on the host once, in phmg_hierarchy_create.  All
// arithmetic of the solve path runs in the kernels of kernels.hip, enqueued on
// one HIP stream.  The host only orchestrates the cycle (Sections 3.1-3.2) and
// carries FGMRES's small Hessenberg / Givens recurrences (Section 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

#include "host_util.h"
#include "phmg_internal.h"

using namespace phmg;

namespace {


void check_csr(const phmg_csr& A, const std::string& who) {
    if (A.nrows < 0 || A.ncols < 0) fail(PHMG_EINVAL, who + "negative dimension");
    if (A.nnz < 0 || A.nnz >= (int64_t)INT32_MAX) fail(PHMG_EINVAL, who + "nnz out of range");
    if (!A.rowptr || (A.nnz > 0 && (!A.col || !A.val))) fail(PHMG_EINVAL, who + "null array");
    if (A.rowptr[0] != 0 || A.rowptr[A.nrows] != A.nnz) fail(PHMG_EINVAL, who + "rowptr does not span [0, nnz]");
    for (int32_t i = 0; i < A.nrows; ++i) {
        if (A.rowptr[i + 1] < A.rowptr[i]) fail(PHMG_EINVAL, who + "rowptr decreases at row " + std::to_string(i));
        for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
            const int32_t c = A.col[k];
            if (c < 0 || c >= A.ncols) fail(PHMG_EINVAL, who + "column index out of range in row " + std::to_string(i));
            if (k > A.rowptr[i] && A.col[k - 1] >= c)
                fail(PHMG_EINVAL, who + "columns not strictly ascending in row " + std::to_string(i));
            if (!std::isfinite(A.val[k])) fail(PHMG_EINVAL, who + "non-finite value in row " + std::to_string(i));
        }
    }
}

DevCsr upload_csr(phmg_ctx ctx, int32_t nrows, int32_t ncols, const std::vector<int32_t>& rp,
                  const std::vector<int32_t>& ci, const std::vector<double>& v) {
    DevCsr d;
    d.nrows = nrows;
    d.ncols = ncols;
    d.nnz = (int64_t)ci.size();
    d.rowptr = upload(ctx, rp.data(), (int64_t)rp.size());
    // 4 zero entries past the end: the 16-byte loads of the vector SpMV may read them
    {
        std::vector<int32_t> cp(ci);
        std::vector<double> vp(v);
        cp.resize(ci.size() + 4, 0);
        vp.resize(v.size() + 4, 0.0);
        d.col = upload(ctx, cp.data(), (int64_t)cp.size());
        d.val = upload(ctx, vp.data(), (int64_t)vp.size());
    }
    const double avg = nrows > 0 ? (double)d.nnz / nrows : 0.0;
    int g = 2;
    while (g < 64 && g * 3 < avg) g *= 2;   // about 3 nonzeros per lane
    d.group = g;
    // row blocks for the row-block SpMV kernel
    if (nrows > 0 && d.nnz > 0) {
        std::vector<int32_t> rb(1, 0);
        bool ok = true;
        for (int32_t i = 0; i < nrows && ok; ++i) {
            const int32_t len = rp[i + 1] - rp[i];
            if (len > kRbNnz) ok = false;
            const int32_t b0 = rb.back();
            if (i - b0 == kRbRows || rp[i + 1] - rp[b0] > kRbNnz) rb.push_back(i);
        }
        rb.push_back(nrows);
        if (ok) {
            d.nrb = (int32_t)rb.size() - 1;
            d.rblk = upload(ctx, rb.data(), (int64_t)rb.size());
        }
    }
    return d;
}

DevCsr upload_csr(phmg_ctx ctx, const phmg_csr& A) {
    std::vector<int32_t> rp(A.rowptr, A.rowptr + A.nrows + 1), ci(A.col, A.col + A.nnz);
    std::vector<double> v(A.val, A.val + A.nnz);
    return upload_csr(ctx, A.nrows, A.ncols, rp, ci, v);
}

// exact symmetry of a CSR matrix with sorted columns (structure and values)
bool is_symmetric(const phmg_csr& A) {
    if (A.nrows != A.ncols) return false;
    for (int32_t i = 0; i < A.nrows; ++i)
        for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
            const int32_t j = A.col[k];
            if (j < i) continue;
            // entry (i, j), j >= i, must equal (j, i): binary search in row j
            const int32_t* b0 = A.col + A.rowptr[j];
            const int32_t* b1 = A.col + A.rowptr[j + 1];
            const int32_t* f = std::lower_bound(b0, b1, i);
            if (f == b1 || *f != i || A.val[f - A.col] != A.val[k]) return false;
        }
    // each upper entry matched a distinct lower one; equal counts leave none unmatched
    int64_t lower = 0, upper = 0;
    for (int32_t i = 0; i < A.nrows; ++i)
        for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
            if (A.col[k] < i) ++lower;
            else if (A.col[k] > i) ++upper;
        }
    return lower == upper;
}

// Symmetric to rounding: the pattern is symmetric and every entry differs from
// its mirror by at most 1e-12 times the larger of the two rows' max |entry|
// (assembly sums the two mirrored entries in different orders).
bool near_symmetric(const phmg_csr& A) {
    if (A.nrows != A.ncols) return false;
    std::vector<double> rmax(A.nrows, 0.0);
    for (int32_t i = 0; i < A.nrows; ++i)
        for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) rmax[i] = std::max(rmax[i], std::fabs(A.val[k]));
    int64_t lower = 0, upper = 0;
    for (int32_t i = 0; i < A.nrows; ++i)
        for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
            const int32_t j = A.col[k];
            if (j < i) {
                ++lower;
                continue;
            }
            if (j == i) continue;
            ++upper;
            const int32_t* b0 = A.col + A.rowptr[j];
            const int32_t* b1 = A.col + A.rowptr[j + 1];
            const int32_t* f = std::lower_bound(b0, b1, i);
            if (f == b1 || *f != i) return false;
            if (std::fabs(A.val[f - A.col] - A.val[k]) > 1e-12 * std::max(rmax[i], rmax[j])) return false;
        }
    return lower == upper;
}

struct HostCsr {
    int32_t nrows = 0, ncols = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
};

HostCsr host_transpose(const phmg_csr& A) {
    HostCsr T;
    T.nrows = A.ncols;
    T.ncols = A.nrows;
    T.rp.assign(A.ncols + 1, 0);
    T.ci.resize(A.nnz);
    T.v.resize(A.nnz);
    for (int64_t k = 0; k < A.nnz; ++k) T.rp[A.col[k] + 1]++;
    for (int32_t j = 0; j < A.ncols; ++j) T.rp[j + 1] += T.rp[j];
    std::vector<int32_t> pos(T.rp.begin(), T.rp.end() - 1);
    for (int32_t i = 0; i < A.nrows; ++i)
        for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
            const int32_t q = pos[A.col[k]]++;
            T.ci[q] = i;
            T.v[q] = A.val[k];
        }
    return T;
}

DevCsr upload_transpose(phmg_ctx ctx, const phmg_csr& A) {
    HostCsr T = host_transpose(A);
    return upload_csr(ctx, T.nrows, T.ncols, T.rp, T.ci, T.v);
}

// C = A B (row by row with a dense accumulator; columns ascending in each row).
// Fails when C has 2^31 nonzeros or more.
HostCsr host_product(const HostCsr& A, const phmg_csr& B) {
    HostCsr C;
    C.nrows = A.nrows;
    C.ncols = B.ncols;
    C.rp.assign(A.nrows + 1, 0);
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int32_t> mark(B.ncols, -1), cols;
    for (int32_t i = 0; i < A.nrows; ++i) {
        cols.clear();
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t j = A.ci[k];
            const double a = A.v[k];
            for (int32_t q = B.rowptr[j]; q < B.rowptr[j + 1]; ++q) {
                const int32_t c = B.col[q];
                if (mark[c] != i) {
                    mark[c] = i;
                    acc[c] = 0.0;
                    cols.push_back(c);
                }
                acc[c] += a * B.val[q];
            }
        }
        std::sort(cols.begin(), cols.end());
        if ((int64_t)C.ci.size() + (int64_t)cols.size() >= ((int64_t)1 << 31))
            fail(PHMG_EINVAL, "R K has too many nonzeros");
        for (int32_t c : cols) {
            C.ci.push_back(c);
            C.v.push_back(acc[c]);
        }
        C.rp[i + 1] = (int32_t)C.ci.size();
    }
    return C;
}


// ----------------------------------------------------------------------------
// relaxation, cycle
// ----------------------------------------------------------------------------

}  // namespace

// nu smoothing steps on level l (eq. "eq:ASM"): damped Richardson, or the
// Chebyshev acceleration of the additive Schwarz operator used in the paper's
// experiments.  With x_zero the incoming x is ignored (treated as 0) and the
// first residual is b itself.  With transpose the sweep is the adjoint one:
// K^T and M^T = sum_i R_i^T K_i^{-T} W_i R_i (the same Chebyshev interval:
// M^T K^T has the spectrum of M K).  r (n), d (n) and Y (sum m) are the work
// buffers of the sweep: the residual, the Chebyshev direction and the staged
// patch results (each is written before it is read); profile = false records
// no timing events.
void phmg::relax_level(phmg_ctx ctx, int l, const double* b, double* x, int nu, bool x_zero, bool transpose,
                       double* rbuf, double* dbuf, double* Y, bool profile) {
    Level& L = ctx->L[l];
    hipStream_t s = ctx->stream;
    if (nu == 0) {
        if (x_zero) launch_fill(s, L.n, x, 0.0);
        return;
    }
    const unsigned saved_mask = ctx->prof.mask;
    if (!profile) ctx->prof.mask = 0;
    struct Restore {
        phmg_ctx c;
        unsigned m;
        ~Restore() { c->prof.mask = m; }
    } restore{ctx, saved_mask};
    const bool cheb = ctx->opts.smoother == PHMG_SMOOTHER_CHEBYSHEV;
    double theta = 0.0, delta = 0.0, sigma = 0.0, rho_prev = 0.0;
    if (cheb) {
        const double emin = ctx->opts.cheb_lo * L.lmax, emax = ctx->opts.cheb_hi * L.lmax;
        theta = 0.5 * (emax + emin);
        delta = 0.5 * (emax - emin);
        sigma = theta / delta;
        rho_prev = 1.0 / sigma;
    }
    for (int it = 0; it < nu; ++it) {
        const double* r = b;                         // x = 0: the residual is b itself
        if (!(it == 0 && x_zero)) {
            Timed t(ctx, PHMG_K_SPMV, l);
            launch_spmv(s, transpose ? L.KT : L.K, x, -1.0, b, 1.0, rbuf);
            r = rbuf;
        }
        {
            Timed t(ctx, PHMG_K_PATCH_APPLY, l);
            if (transpose) launch_patch_apply_t(s, L, r);
            else launch_patch_apply(s, L, r, Y);
        }
        Timed t(ctx, PHMG_K_SCATTER, l);
        const bool xz = it == 0 && x_zero;
        if (!cheb) {
            launch_scatter(s, L, ctx->opts.omega, 0.0, nullptr, false, x, xz, transpose, Y);
        } else if (it == 0) {
            launch_scatter(s, L, 1.0 / theta, 0.0, dbuf, nu > 1, x, xz, transpose, Y);
        } else {
            const double rho = 1.0 / (2.0 * sigma - rho_prev);
            launch_scatter(s, L, 2.0 * rho / delta, rho * rho_prev, dbuf, it + 1 < nu, x, false, transpose, Y);
            rho_prev = rho;
        }
    }
}

namespace {

void relax(phmg_ctx ctx, int l, const double* b, double* x, int nu, bool x_zero, bool transpose = false) {
    Level& L = ctx->L[l];
    relax_level(ctx, l, b, x, nu, x_zero, transpose, L.r, L.d, L.Y, true);
}

// Set-up autotuner of the patch-solve kernel shape: every compiled shape of the
// level's precision is timed on the level's own patches (HIP events around
// kTuneBatch back-to-back launches, best of three batches: one launch of a
// small level is not much longer than the events around it) and the fastest
// is kept.  Runs once per level and precision.
constexpr int kTuneBatch = 8;
int tune_key(const Level& L) { return L.prec + (L.sym ? 3 : 0); }

void tune_apply(phmg_ctx ctx, int l, hipStream_t s) {
    Level& L = ctx->L[l];
    if (L.tuned_for == tune_key(L) || L.npatch == 0) return;
    launch_fill(s, L.n, L.r, 1.0);
    hipEvent_t e0, e1;
    hipcheck(hipEventCreate(&e0), "hipEventCreate");
    hipcheck(hipEventCreate(&e1), "hipEventCreate");
    const int nv = apply_variant_count(L);
    int best = 0;
    float best_ms = 1e30f;
    for (int v = 0; v < nv; ++v) {
        L.apply_variant = v;
        launch_patch_apply(s, L, L.r);                      // warm-up
        float vbest = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            hipcheck(hipEventRecord(e0, s), "hipEventRecord");
            for (int b = 0; b < kTuneBatch; ++b) launch_patch_apply(s, L, L.r);
            hipcheck(hipEventRecord(e1, s), "hipEventRecord");
            hipcheck(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            hipcheck(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            vbest = std::min(vbest, ms);
        }
        if (vbest < best_ms) {
            best_ms = vbest;
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hipcheck(hipGetLastError(), "autotune launch");
    L.apply_variant = best;
    L.tuned_for = tune_key(L);
}

// Eigenvalues of a small real upper-Hessenberg matrix (row-major k x k) by the
// complex single-shift QR algorithm: Wilkinson shifts, Givens rotations,
// deflation at the bottom of the active block.
bool hessenberg_eigenvalues(std::vector<std::complex<double>> A, int k, std::vector<std::complex<double>>& ev) {
    using cd = std::complex<double>;
    auto a = [&](int i, int j) -> cd& { return A[(size_t)i * k + j]; };
    ev.clear();
    int n = k, iter = 0;
    std::vector<cd> cs(k), sn(k);
    while (n > 0) {
        if (n == 1) {
            ev.push_back(a(0, 0));
            break;
        }
        const double sub = std::abs(a(n - 1, n - 2));
        double scale = std::abs(a(n - 1, n - 1)) + std::abs(a(n - 2, n - 2));
        if (scale == 0.0) scale = 1.0;
        if (sub <= 1e-15 * scale) {
            ev.push_back(a(n - 1, n - 1));
            --n;
            iter = 0;
            continue;
        }
        if (++iter > 100 * k) return false;
        const cd p = a(n - 2, n - 2), q = a(n - 2, n - 1), r = a(n - 1, n - 2), t = a(n - 1, n - 1);
        const cd half_tr = 0.5 * (p + t), det = p * t - q * r;
        const cd disc = std::sqrt(half_tr * half_tr - det);
        const cd l1 = half_tr + disc, l2 = half_tr - disc;
        cd mu = std::abs(l1 - t) < std::abs(l2 - t) ? l1 : l2;
        if (iter % 11 == 10) mu += 0.75 * std::abs(r);      // exceptional shift
        for (int i = 0; i < n; ++i) a(i, i) -= mu;
        for (int i = 0; i + 1 < n; ++i) {
            const cd x = a(i, i), y = a(i + 1, i);
            const double rr = std::sqrt(std::norm(x) + std::norm(y));
            const cd c = rr == 0.0 ? cd(1.0) : x / rr, sg = rr == 0.0 ? cd(0.0) : y / rr;
            cs[i] = c;
            sn[i] = sg;
            for (int j = i; j < n; ++j) {
                const cd u = a(i, j), v = a(i + 1, j);
                a(i, j) = std::conj(c) * u + std::conj(sg) * v;
                a(i + 1, j) = -sg * u + c * v;
            }
        }
        for (int i = 0; i + 1 < n; ++i) {
            const cd c = cs[i], sg = sn[i];
            for (int rw = 0; rw <= i + 1; ++rw) {
                const cd u = a(rw, i), v = a(rw, i + 1);
                a(rw, i) = u * c + v * sg;
                a(rw, i + 1) = -u * std::conj(sg) + v * std::conj(c);
            }
        }
        for (int i = 0; i < n; ++i) a(i, i) += mu;
    }
    return true;
}

// Largest real part of the eigenvalues of H[0:k, 0:k] (H column-major, leading dimension ldh).
double ritz_max_real(const double* H, int ldh, int k) {
    std::vector<std::complex<double>> A((size_t)k * k), ev;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) A[(size_t)i * k + j] = H[(size_t)j * ldh + i];
    if (!hessenberg_eigenvalues(A, k, ev)) fail(PHMG_ESINGULAR, "Hessenberg QR did not converge");
    double mx = -INFINITY;
    for (const auto& e : ev) mx = std::max(mx, e.real());
    return mx;
}

void ensure_krylov(phmg_ctx ctx, int restart);
double device_norm(hipStream_t s, Krylov& kr, int64_t n, const double* v);

// Classical Gram-Schmidt twice against the ncol basis vectors V: h1 = V^T w,
// w -= V h1, h2 = V^T w, w -= V h2, hn2 = w . w.  The subtraction and the next
// products share one read of the basis (three passes instead of five).
void cgs2(hipStream_t s, double* partial, int64_t n, int ncol, const double* V, double* w, double* h1, double* h2,
          double* hn2) {
    launch_multidot(s, n, ncol, V, n, w, partial, h1);
    if (ncol <= gs_max_cols()) {
        launch_gs_update(s, n, ncol, V, n, h1, w, partial, h2, false);
        launch_gs_update(s, n, ncol, V, n, h2, w, partial, hn2, true);
    } else {
        launch_gemv_sub(s, n, ncol, V, n, h1, w);
        launch_multidot(s, n, ncol, V, n, w, partial, h2);
        launch_gemv_sub(s, n, ncol, V, n, h2, w);
        launch_multidot(s, n, 1, w, n, w, partial, hn2);
    }
}

// lambda_max(M^{-1} K): largest real Ritz value of eig_iters Arnoldi steps
// (CGS2) from v_0 = (1 + sin(j)/2) / ||.||, all vectors on the device in the
// level's own work space, on the level's set-up stream.  Every step's
// projections stay on the device (one column of S doubles per step: h, h',
// ||w||^2); the next basis vector is normalised with the device norm, and the
// host reads all columns once at the end.  Several levels run interleaved.
struct ArnoldiRun {
    int l = 0;
    hipStream_t s = nullptr;
    int64_t n = 0;
    int k = 0, S = 0;
    double *V = nullptr, *w = nullptr, *part = nullptr, *H = nullptr, *nrm = nullptr;
};

ArnoldiRun arnoldi_begin(phmg_ctx ctx, int l, hipStream_t s) {
    Level& L = ctx->L[l];
    ArnoldiRun a;
    a.l = l;
    a.s = s;
    a.n = L.n;
    a.k = (int)std::min<int64_t>(ctx->opts.eig_iters, L.n);
    a.S = 2 * (a.k + 1) + 1;
    const int64_t len = a.n * a.k + a.n + (int64_t)kRedBlocks * (a.k + 2) + (int64_t)a.S * a.k + 2;
    if (L.arn_len < len) {
        dfree(ctx, L.arn);
        L.arn = dalloc<double>(ctx, len);
        L.arn_len = len;
    }
    a.V = L.arn;
    a.w = a.V + a.n * a.k;
    a.part = a.w + a.n;
    a.H = a.part + (int64_t)kRedBlocks * (a.k + 2);
    a.nrm = a.H + (int64_t)a.S * a.k;
    launch_power_start(s, a.n, a.V);
    launch_multidot(s, a.n, 1, a.V, a.n, a.V, a.part, a.nrm);
    launch_scale_by_devnorm(s, a.n, a.V, a.nrm, a.V);
    return a;
}

void arnoldi_step(phmg_ctx ctx, const ArnoldiRun& a, int j) {
    Level& L = ctx->L[a.l];
    const hipStream_t s = a.s;
    const int64_t n = a.n;
    double* h1 = a.H + (int64_t)j * a.S;
    double* h2 = h1 + (a.k + 1);
    double* hn2 = h1 + 2 * (a.k + 1);
    launch_spmv(s, L.K, a.V + (int64_t)j * n, 1.0, nullptr, 0.0, L.r);
    launch_patch_apply(s, L, L.r);
    launch_scatter(s, L, 1.0, 0.0, nullptr, false, a.w, true);
    cgs2(s, a.part, n, j + 1, a.V, a.w, h1, h2, hn2);
    if (j + 1 < a.k) launch_scale_by_devnorm(s, n, a.w, hn2, a.V + (int64_t)(j + 1) * n);
}

double arnoldi_finish(const ArnoldiRun& a) {
    const int k = a.k, S = a.S;
    std::vector<double> hcols((size_t)S * k);
    hipcheck(hipMemcpyAsync(hcols.data(), a.H, sizeof(double) * S * k, hipMemcpyDeviceToHost, a.s), "D2H");
    hipcheck(hipStreamSynchronize(a.s), "hipStreamSynchronize");
    std::vector<double> H((size_t)(k + 1) * k, 0.0);
    int kk = k;
    for (int j = 0; j < k; ++j) {
        const double* c = hcols.data() + (size_t)j * S;
        for (int i = 0; i <= j; ++i) H[(size_t)j * (k + 1) + i] = c[i] + c[(k + 1) + i];
        const double hn = std::sqrt(c[2 * (k + 1)]);
        H[(size_t)j * (k + 1) + j + 1] = hn;
        if (hn == 0.0) {                 // exact breakdown: later columns are not used
            kk = j + 1;
            break;
        }
    }
    return ritz_max_real(H.data(), k + 1, kk);      // leading dimension k + 1, order kk
}

// One cycle on level l.  transpose gives the adjoint operator B^T: the same
// cycle with K^T, the adjoint sweeps and the transposed coarse solve (with
// equal pre- and post-smoothing the transposed algorithm is exactly B^T).
void cycle(phmg_ctx ctx, int l, const double* b, double* x, bool x_zero, bool transpose = false) {
    const int last = (int)ctx->L.size() - 1;
    hipStream_t s = ctx->stream;
    if (l == last) {
        if (transpose) launch_coarse_solve_t(s, ctx->L[l], b, x);
        else launch_coarse_solve(s, ctx->L[l], b, x);
        return;
    }
    Level& L = ctx->L[l];
    Level& C = ctx->L[l + 1];
    const int np = ctx->opts.n_plevels;
    const int nu = l < np ? ctx->opts.nu_p : ctx->opts.nu_h;
    relax(ctx, l, b, x, nu, x_zero, transpose);
    if (!transpose && L.fuse_restrict) {
        Timed t(ctx, PHMG_K_SPMV, l);
        launch_spmv_diff(s, L.R, b, L.RK, x, C.b);
    } else {
        {
            Timed t(ctx, PHMG_K_SPMV, l);
            launch_spmv(s, transpose ? L.KT : L.K, x, -1.0, b, 1.0, L.r);
        }
        {
            Timed t(ctx, PHMG_K_SPMV, l);
            launch_spmv(s, L.R, L.r, 1.0, nullptr, 0.0, C.b);
        }
    }
    if (l + 1 < np || l + 1 == last || l >= np) {
        cycle(ctx, l + 1, C.b, C.x, true, transpose);
    } else {
        for (int t = 0; t < ctx->opts.n_v; ++t) cycle(ctx, l + 1, C.b, C.x, t == 0, transpose);
    }
    {
        Timed t(ctx, PHMG_K_SPMV, l);
        launch_spmv(s, L.P, C.x, 1.0, x, 1.0, x);
    }
    relax(ctx, l, b, x, nu, false, transpose);
}

void vcycle(phmg_ctx ctx, const double* b, double* x, bool transpose = false) {
    if (ctx->opts.n_plevels == 0) {
        for (int t = 0; t < ctx->opts.n_v; ++t) cycle(ctx, 0, b, x, t == 0, transpose);
    } else {
        cycle(ctx, 0, b, x, true, transpose);
    }
}

void invalidate_slot_graphs(phmg_ctx ctx) {
    for (auto& g : ctx->sgraphs) {
        if (g.e) (void)hipGraphExecDestroy(g.e);
        if (g.g) (void)hipGraphDestroy(g.g);
    }
    ctx->sgraphs.clear();
}

void invalidate_graph(phmg_ctx ctx) {
    invalidate_block_graph(ctx);
    invalidate_slot_graphs(ctx);
    for (int t = 0; t < 2; ++t) {
        if (ctx->vexec[t]) (void)hipGraphExecDestroy(ctx->vexec[t]);
        if (ctx->vgraph[t]) (void)hipGraphDestroy(ctx->vgraph[t]);
        ctx->vexec[t] = nullptr;
        ctx->vgraph[t] = nullptr;
    }
}

}  // namespace

std::vector<uint64_t> phmg::graph_signature(phmg_ctx ctx) {
    std::vector<uint64_t> g;
    auto u = [&](uint64_t v) { g.push_back(v); };
    auto p = [&](const void* v) { g.push_back((uint64_t)(uintptr_t)v); };
    auto d = [&](double v) {
        uint64_t b;
        std::memcpy(&b, &v, sizeof b);
        g.push_back(b);
    };
    auto csr = [&](const DevCsr& A) {
        p(A.rowptr);
        p(A.col);
        p(A.val);
        p(A.rblk);
        u((uint64_t)A.group | (uint64_t)A.xcd << 8 | (uint64_t)A.rowblock << 9 | (uint64_t)A.unroll << 10 | (uint64_t)A.vec << 15 |
          (uint64_t)A.bgroup << 16 | (uint64_t)A.bxcd << 24 | (uint64_t)A.bquad << 25);
    };
    const phmg_cycle_opts& o = ctx->opts;
    u((uint64_t)o.nu_p | (uint64_t)o.nu_h << 16 | (uint64_t)o.n_v << 32 | (uint64_t)o.n_plevels << 48);
    u((uint64_t)o.smoother);
    d(o.omega);
    d(o.cheb_lo);
    d(o.cheb_hi);
    p(ctx->gin);
    p(ctx->gout);
    p(ctx->bgin);
    p(ctx->bgout);
    for (const Level& L : ctx->L) {
        csr(L.K);
        csr(L.KT);
        csr(L.P);
        csr(L.R);
        csr(L.RK);
        u((uint64_t)L.fuse_restrict);
        p(L.factors);
        p(L.fofflp);
        p(L.pinfo);
        p(L.bfactors);
        p(L.bfoff);
        p(L.Y);
        p(L.wdof);
        p(L.Yb);
        p(L.cinv);
        p(L.cdense);
        p(L.r);
        p(L.b);
        p(L.x);
        p(L.d);
        p(L.rb);
        p(L.bb);
        p(L.xb);
        p(L.db);
        u((uint64_t)L.prec | (uint64_t)L.sym << 8 | (uint64_t)L.apply_variant << 16 |
          (uint64_t)L.block_variant << 32);
        d(L.lmax);
    }
    return g;
}

namespace {

// Capture one V-cycle (b -> x) on a private stream.  The cycle launches
// kernels only (no copies, no memsets, no host synchronisation), so the graph
// replays it exactly; it is rebuilt whenever graph_signature() changes.
void capture_vcycle(phmg_ctx ctx, const double* b, double* x, bool transpose, hipGraph_t* graph,
                    hipGraphExec_t* exec) {
    if (!ctx->cap_stream) hipcheck(hipStreamCreate(&ctx->cap_stream), "hipStreamCreate");
    hipStream_t saved = ctx->stream;
    hipcheck(hipStreamSynchronize(saved), "hipStreamSynchronize");
    ctx->stream = ctx->cap_stream;
    hipcheck(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
        vcycle(ctx, b, x, transpose);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(ctx->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        ctx->stream = saved;
        throw;
    }
    ctx->stream = saved;
    hipcheck(hipStreamEndCapture(ctx->cap_stream, graph), "hipStreamEndCapture");
    hipcheck(hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0), "hipGraphInstantiate");
}

// the general-purpose graph: gin -> gout, with copies in and out around it
void build_graph(phmg_ctx ctx, bool transpose) {
    const int64_t n0 = ctx->L[0].n;
    if (!ctx->gin) {
        ctx->gin = dalloc<double>(ctx, n0);
        ctx->gout = dalloc<double>(ctx, n0);
    }
    const int t = transpose ? 1 : 0;
    capture_vcycle(ctx, ctx->gin, ctx->gout, transpose, &ctx->vgraph[t], &ctx->vexec[t]);
    ctx->vsig[t] = graph_signature(ctx);
}

// FGMRES applies the preconditioner to its basis slots V_j -> Z_j only: one graph
// per (slot, orientation) captured on the slots themselves saves the two copies
// of the general graph (at most kSlotGraphs of them; the slots' buffers live as
// long as the Krylov work space, which drops these graphs when it is reallocated)
constexpr size_t kSlotGraphs = 128;

void precond(phmg_ctx ctx, const double* b, double* x, bool transpose);

void precond_slot(phmg_ctx ctx, const double* b, double* x, bool transpose) {
    if (!ctx->use_graphs || ctx->prof.mask) {
        vcycle(ctx, b, x, transpose);
        return;
    }
    const int t = transpose ? 1 : 0;
    const std::vector<uint64_t> sig = graph_signature(ctx);
    for (auto& g : ctx->sgraphs) {
        if (g.b != b || g.x != x || g.t != t) continue;
        if (g.sig != sig) {
            (void)hipGraphExecDestroy(g.e);
            (void)hipGraphDestroy(g.g);
            g.e = nullptr;
            g.g = nullptr;
            capture_vcycle(ctx, b, x, transpose, &g.g, &g.e);
            g.sig = sig;
        }
        hipcheck(hipGraphLaunch(g.e, ctx->stream), "hipGraphLaunch");
        return;
    }
    if (ctx->sgraphs.size() >= kSlotGraphs) {
        precond(ctx, b, x, transpose);
        return;
    }
    phmg_ctx_s::SlotGraph g{b, x, t, sig, nullptr, nullptr};
    capture_vcycle(ctx, b, x, transpose, &g.g, &g.e);
    ctx->sgraphs.push_back(std::move(g));
    hipcheck(hipGraphLaunch(ctx->sgraphs.back().e, ctx->stream), "hipGraphLaunch");
}

// x <- B b (one preconditioner application): the captured graph when graphs
// are on and no per-kernel profiling is requested, the eager launches otherwise.
void precond(phmg_ctx ctx, const double* b, double* x, bool transpose) {
    if (!ctx->use_graphs || ctx->prof.mask) {
        vcycle(ctx, b, x, transpose);
        return;
    }
    const int t = transpose ? 1 : 0;
    if (ctx->vexec[t] && ctx->vsig[t] != graph_signature(ctx)) {
        (void)hipGraphExecDestroy(ctx->vexec[t]);
        (void)hipGraphDestroy(ctx->vgraph[t]);
        ctx->vexec[t] = nullptr;
        ctx->vgraph[t] = nullptr;
    }
    if (!ctx->vexec[t]) build_graph(ctx, transpose);
    const int64_t n0 = ctx->L[0].n;
    launch_copy(ctx->stream, n0, b, ctx->gin);
    hipcheck(hipGraphLaunch(ctx->vexec[t], ctx->stream), "hipGraphLaunch");
    launch_copy(ctx->stream, n0, ctx->gout, x);
}

// Set-up autotuner of the SpMV: lanes per row of one matrix, timed once.
// SpMV kernel variants: 0-5 CSR with 2, 4, ..., 64 lanes per row, 6-11 the same
// with XCD-contiguous row ranges, 12 the row-block kernel (when the matrix has
// row blocks), 13-16 CSR with 4, 8, 16, 32 lanes per row and 8 entries in
// flight per lane, 17-19 CSR with 4, 8, 16 lanes per row and 4 consecutive
// entries per lane (16-byte loads).
constexpr int kSpmvVariants = 20;
bool spmv_variant_ok(const DevCsr& A, int v) { return v >= 0 && v < kSpmvVariants && (v != 12 || A.nrb > 0); }
void set_spmv_variant(DevCsr& A, int v) {
    A.rowblock = v == 12;
    A.unroll = 4;
    A.vec = false;
    if (v >= 17) {
        A.group = 4 << (v - 17);
        A.xcd = false;
        A.vec = true;
    } else if (v < 12) {
        A.group = 2 << (v % 6);
        A.xcd = v >= 6;
    } else if (v > 12) {
        A.group = 4 << (v - 13);
        A.xcd = false;
        A.unroll = 8;
    }
}
int spmv_variant_of(const DevCsr& A) {
    if (A.rowblock) return 12;
    int lg = 0;
    while ((2 << lg) < A.group) ++lg;
    if (A.vec) return 17 + (lg - 1);
    if (A.unroll == 8) return 13 + (lg - 1);
    return lg + (A.xcd ? 6 : 0);
}

// Matrices with fewer rows than this are latency-bound inside the cycle, where
// their data is no longer in cache: timing them in isolation (hot caches) would
// mislead, so they get the lanes-per-row that needs one pass of 4 entries per
// lane for an average row (fewest dependent loads).
constexpr int kSmallRows = 16384;
int lanes_for(double avg_row) {
    int g = 2;
    while (g < 64 && 4 * g < avg_row) g *= 2;
    return g;
}

void tune_spmv(phmg_ctx ctx, DevCsr& A, const double* x, double* y) {
    if (A.tuned || A.nrows == 0) return;
    if (A.nrows < kSmallRows) {
        A.group = lanes_for((double)A.nnz / A.nrows);
        A.xcd = false;
        A.rowblock = false;
        A.unroll = 4;
        A.vec = false;
        A.tuned = true;
        return;
    }
    hipStream_t s = ctx->stream;
    hipEvent_t e0, e1;
    hipcheck(hipEventCreate(&e0), "hipEventCreate");
    hipcheck(hipEventCreate(&e1), "hipEventCreate");
    int best_v = 0;
    float best_ms = 1e30f;
    for (int cand = 0; cand < kSpmvVariants; ++cand) {
        if (!spmv_variant_ok(A, cand)) continue;
        set_spmv_variant(A, cand);
        launch_spmv(s, A, x, 1.0, nullptr, 0.0, y);
        float gbest = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            hipcheck(hipEventRecord(e0, s), "hipEventRecord");
            for (int b = 0; b < kTuneBatch; ++b) launch_spmv(s, A, x, 1.0, nullptr, 0.0, y);
            hipcheck(hipEventRecord(e1, s), "hipEventRecord");
            hipcheck(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            hipcheck(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            gbest = std::min(gbest, ms);
        }
        if (gbest < best_ms) {
            best_ms = gbest;
            best_v = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hipcheck(hipGetLastError(), "spmv autotune launch");
    set_spmv_variant(A, best_v);
    A.tuned = true;
}


// lanes per row of the fused restricted residual (stored in RK.group), and
// whether it beats the two-step residual + restriction with their own tuned
// kernels; timed once (after tune_spmv of K and R)
void tune_spmv_diff(phmg_ctx ctx, Level& L, const double* x, double* y) {
    DevCsr& A = L.RK;
    if (A.tuned || A.nrows == 0) return;
    if (A.nrows < kSmallRows) {              // one launch instead of two always wins here
        A.group = lanes_for((double)(A.nnz + L.R.nnz) / A.nrows);
        A.tuned = true;
        L.fuse_restrict = true;
        return;
    }
    hipStream_t s = ctx->stream;
    hipEvent_t e0, e1;
    hipcheck(hipEventCreate(&e0), "hipEventCreate");
    hipcheck(hipEventCreate(&e1), "hipEventCreate");
    int best = A.group;
    float best_ms = 1e30f;
    for (int g = 2; g <= 64; g *= 2) {
        A.group = g;
        launch_spmv_diff(s, L.R, x, A, x, y);
        float gbest = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            hipcheck(hipEventRecord(e0, s), "hipEventRecord");
            for (int b = 0; b < kTuneBatch; ++b) launch_spmv_diff(s, L.R, x, A, x, y);
            hipcheck(hipEventRecord(e1, s), "hipEventRecord");
            hipcheck(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            hipcheck(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            gbest = std::min(gbest, ms);
        }
        if (gbest < best_ms) {
            best_ms = gbest;
            best = g;
        }
    }
    float two = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
        hipcheck(hipEventRecord(e0, s), "hipEventRecord");
        for (int b = 0; b < kTuneBatch; ++b) {
            launch_spmv(s, L.K, x, -1.0, x, 1.0, L.r);
            launch_spmv(s, L.R, L.r, 1.0, nullptr, 0.0, y);
        }
        hipcheck(hipEventRecord(e1, s), "hipEventRecord");
        hipcheck(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        hipcheck(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (rep > 0) two = std::min(two, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hipcheck(hipGetLastError(), "spmv autotune launch");
    A.group = best;
    A.tuned = true;
    L.fuse_restrict = best_ms < two;
}

// Set-up of levels [lo, hi): SpMV tuning and the stored layout on the context
// stream, then every level's factorisation, conversion and eigenvalue
// estimate on a stream of its own (levels are independent), so the small,
// latency-bound levels overlap the large one.  Synchronous: all level streams
// are drained before returning, also when a level fails.
void setup_levels(phmg_ctx ctx, int lo, int hi) {
    const int nl = (int)ctx->L.size();
    const int last = nl - 1;
    hipStream_t s0 = ctx->stream;
    // (captured graphs stay valid while graph_signature() is unchanged; the
    // set-up reuses its buffers, so repeated set-ups keep them)
    for (int l = lo; l < hi; ++l) {
        Level& L = ctx->L[l];
        L.ready = false;
        if (l < last) {
            Level& C = ctx->L[l + 1];
            launch_fill(s0, L.n, L.d, 1.0);
            launch_fill(s0, C.n, C.x, 1.0);
            tune_spmv(ctx, L.K, L.d, L.r);
            if (L.KT.rowptr != L.K.rowptr) tune_spmv(ctx, L.KT, L.d, L.r);   // adjoint cycle
            tune_spmv(ctx, L.R, L.d, C.b);
            tune_spmv(ctx, L.P, C.x, L.r);
            tune_spmv_diff(ctx, L, L.d, C.b);
        }
        if (l == last) {
            if (!L.cdense) {
                L.cdense = dalloc<double>(ctx, (int64_t)L.nb * L.nb);
                L.cpiv = dalloc<int>(ctx, L.nb);
                L.cwork = dalloc<double>(ctx, (int64_t)(1 + kPanel) * L.nb);
            }
            if (!L.cinv) L.cinv = dalloc<double>(ctx, (int64_t)L.nb * L.nb);
            continue;
        }
        if (!L.work64) L.work64 = dalloc<double>(ctx, L.sum_m2);
        // the stored inverses in the level's precision: general layout (columns
        // padded to 16 bytes) or the symmetric strip layout
        const size_t es = L.prec == PHMG_PREC_F64 ? 8 : (L.prec == PHMG_PREC_F32 ? 4 : 2);
        L.sym = L.sym_ok && L.storage == PHMG_STORAGE_AUTO;
        const int64_t cnt = L.sym ? L.sum_ls[L.prec] : L.sum_lp[L.prec];
        std::vector<int64_t> off(L.npatch);
        {
            const std::vector<int64_t>& hp = L.hptr;
            const int V = factor_pad_of(L.prec);
            int64_t acc = 0;
            for (int32_t i = 0; i < L.npatch; ++i) {
                const int64_t m = hp[i + 1] - hp[i];
                off[i] = acc;
                acc += L.sym ? sym_layout_size((int)m, V) : (m + V - 1) / V * V * m;
            }
            // the allocation below is sized at create (sum_lp); the layout must match it exactly
            if (acc != cnt) fail(PHMG_EINVAL, lvl(l) + "internal: reduced-precision layout size mismatch");
        }
        if (!L.fofflp) L.fofflp = dalloc<int64_t>(ctx, L.npatch);
        hipcheck(hipMemcpy(L.fofflp, off.data(), sizeof(int64_t) * (size_t)L.npatch, hipMemcpyHostToDevice),
                 "hipMemcpy H2D");
        {
            std::vector<int64_t> info(4 * (size_t)L.npatch);
            for (int32_t k = 0; k < L.npatch; ++k) {
                const int32_t q = L.horder[k];
                info[4 * (size_t)k] = L.hptr[q];
                info[4 * (size_t)k + 1] = off[q];
                info[4 * (size_t)k + 2] = L.hptr[q + 1] - L.hptr[q];
                info[4 * (size_t)k + 3] = q;
            }
            if (!L.pinfo) L.pinfo = dalloc<int64_t>(ctx, 4 * (int64_t)L.npatch);
            if (!info.empty())
                hipcheck(hipMemcpy(L.pinfo, info.data(), sizeof(int64_t) * info.size(), hipMemcpyHostToDevice),
                         "hipMemcpy H2D");
        }
        const size_t bytes = es * (size_t)std::max<int64_t>(cnt, 1);
        if (!L.factors || L.factor_bytes < bytes) {
            if (L.factors) dfree(ctx, L.factors);
            L.factors = nullptr;
            L.factor_bytes = 0;
            void* p = nullptr;
            if (hipMalloc(&p, bytes) != hipSuccess) {
                (void)hipGetLastError();
                fail(PHMG_ENOMEM, lvl(l) + "factor allocation failed");
            }
            ctx->allocs.push_back(p);
            L.factors = p;
            L.factor_bytes = bytes;
        }
    }
    // set-up streams, forked after everything enqueued so far on the context stream:
    // the finest level (the longest chain) on one, the intermediate levels one after
    // another on a second, the dense coarse inverse on a third.  Three streams plus the
    // context stream stay within the four hardware queues a process gets by default,
    // so no other level's kernels queue up behind the finest level's or in front of them.
    const int nstreams = std::min(nl, 3);
    while ((int)ctx->sstreams.size() < nstreams) {
        hipStream_t st = nullptr;
        hipcheck(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
        ctx->sstreams.push_back(st);
    }
    auto sst = [&](int l) -> hipStream_t {
        return ctx->sstreams[l == 0 ? 0 : (l == last ? nstreams - 1 : 1)];
    };
    while ((int)ctx->sevents.size() < nl + 1) {
        hipEvent_t e = nullptr;
        hipcheck(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
        ctx->sevents.push_back(e);
    }
    if (!ctx->status_host)
        hipcheck(hipHostMalloc((void**)&ctx->status_host, sizeof(int32_t) * nl), "hipHostMalloc");
    hipcheck(hipEventRecord(ctx->sevents[0], s0), "hipEventRecord");
    struct Drain {                                  // every exit waits for all set-up streams
        phmg_ctx c;
        ~Drain() {
            for (auto st : c->sstreams) (void)hipStreamSynchronize(st);
        }
    } drain{ctx};
    for (int l = lo; l < hi; ++l)
        hipcheck(hipStreamWaitEvent(sst(l), ctx->sevents[0], 0), "hipStreamWaitEvent");
    // factorisations
    for (int l = lo; l < hi; ++l) {
        Level& L = ctx->L[l];
        hipStream_t s = sst(l);
        launch_fill_i32(s, 1, L.status, INT32_MAX);
        if (l == last) {
            launch_coarse_build(s, L, L.cdense);
            {
                Timed t(ctx, PHMG_K_FACTOR, l, s);
                launch_dense_gj(s, L.cdense, L.nb, L.cpiv, L.status, ctx->scal + 4, L.cwork);
                hipcheck(hipGetLastError(), "coarse factorisation launch");
            }
            launch_transpose(s, L.nb, L.cdense, L.cinv);
        } else {
            {
                Timed t(ctx, PHMG_K_EXTRACT, l, s);
                launch_extract(s, L, L.work64);
                hipcheck(hipGetLastError(), "extract launch");
            }
            {
                Timed t(ctx, PHMG_K_FACTOR, l, s);
                // patches above 144 DoFs on the coarse inverse's stream, beside the smaller ones
                if (nstreams >= 3) {
                    if (!ctx->fork_ev[0]) {
                        for (auto& e : ctx->fork_ev)
                            hipcheck(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
                    }
                    launch_patch_factor(s, L, L.work64, sst(last), ctx->fork_ev[0], ctx->fork_ev[1]);
                } else {
                    launch_patch_factor(s, L, L.work64);
                }
                hipcheck(hipGetLastError(), "patch factorisation launch");
            }
        }
        hipcheck(hipMemcpyAsync(ctx->status_host + l, L.status, sizeof(int32_t), hipMemcpyDeviceToHost, s), "D2H");
        // a singular patch stops its elimination early and leaves its pivot lists
        // (pdofs_perm, pidx) unwritten; the conversion never indexes outside the
        // patch with them, and the status is checked before any result is used
        if (l < last) {
            launch_convert_patches(s, L, L.work64, L.factors);
            hipcheck(hipGetLastError(), "convert launch");
        }
    }
    auto check_status = [&](int l) {
        const int32_t st = ctx->status_host[l];
        if (st == INT32_MAX) return;
        if (l == last) fail(PHMG_ESINGULAR, lvl(l) + "coarse matrix is singular");
        fail(PHMG_ESINGULAR, lvl(l) + "patch " + std::to_string(st) + " is singular");
    };
    // first set-up of a level in its layout: time the patch-solve shapes (synchronous)
    for (int l = lo; l < hi && l < last; ++l) {
        Level& L = ctx->L[l];
        if (L.tuned_for == tune_key(L) || L.npatch == 0) continue;
        hipcheck(hipStreamSynchronize(sst(l)), "hipStreamSynchronize");
        check_status(l);
        tune_apply(ctx, l, sst(l));
    }
    std::vector<double> lmax(nl, 0.0);
    if (ctx->opts.smoother == PHMG_SMOOTHER_CHEBYSHEV) {
        std::vector<ArnoldiRun> runs;
        for (int l = lo; l < hi && l < last; ++l) runs.push_back(arnoldi_begin(ctx, l, sst(l)));
        int kmax = 0;
        for (const auto& a : runs) kmax = std::max(kmax, a.k);
        for (int j = 0; j < kmax; ++j)
            for (const auto& a : runs)
                if (j < a.k) arnoldi_step(ctx, a, j);
        for (const auto& a : runs) lmax[a.l] = arnoldi_finish(a);      // synchronises the level's stream
    }
    for (int l = lo; l < hi; ++l) {
        hipcheck(hipStreamSynchronize(sst(l)), "hipStreamSynchronize");
        check_status(l);
    }
    if (ctx->opts.smoother == PHMG_SMOOTHER_CHEBYSHEV)
        for (int l = lo; l < hi && l < last; ++l) {
            if (!(lmax[l] > 0.0) || !std::isfinite(lmax[l]))
                fail(PHMG_ESINGULAR, lvl(l) + "eigenvalue estimate of M^{-1}K is not positive and finite");
            ctx->L[l].lmax = lmax[l];
        }
    for (int l = lo; l < hi; ++l) {
        hipcheck(hipEventRecord(ctx->sevents[1 + l], sst(l)), "hipEventRecord");
        hipcheck(hipStreamWaitEvent(s0, ctx->sevents[1 + l], 0), "hipStreamWaitEvent");
    }
    for (int l = lo; l < hi; ++l) {
        ctx->L[l].ready = true;
        ++ctx->L[l].setup_count;
    }
}

double device_norm(hipStream_t s, Krylov& kr, int64_t n, const double* v) {
    launch_multidot(s, n, 1, v, n, v, kr.partial, kr.hdev);
    hipcheck(hipMemcpyAsync(kr.hhost, kr.hdev, sizeof(double), hipMemcpyDeviceToHost, s), "D2H");
    hipcheck(hipStreamSynchronize(s), "hipStreamSynchronize");
    return std::sqrt(kr.hhost[0]);
}

// FGMRES work space for vectors of length n and `restart` basis vectors; the
// device memory is owned (and freed) through `owner`.
void ensure_krylov(phmg_ctx owner, Krylov& kr, int64_t n, int restart) {
    if (kr.cap >= restart && kr.n == n) return;
    dfree(owner, kr.V);
    dfree(owner, kr.Z);
    dfree(owner, kr.hdev);
    if (kr.hhost) (void)hipHostFree(kr.hhost);
    kr.hhost = nullptr;
    if (kr.n != n) {
        dfree(owner, kr.w);
        dfree(owner, kr.r);
        kr.w = kr.r = nullptr;
    }
    kr.V = dalloc<double>(owner, n * (restart + 1));
    kr.Z = dalloc<double>(owner, n * restart);
    kr.hdev = dalloc<double>(owner, 2 * (restart + 2) + 4);
    if (!kr.w) kr.w = dalloc<double>(owner, n);
    if (!kr.r) kr.r = dalloc<double>(owner, n);
    if (kr.partial_cols < restart + 2) {
        dfree(owner, kr.partial);
        kr.partial = dalloc<double>(owner, (int64_t)kRedBlocks * (restart + 2));
        kr.partial_cols = restart + 2;
    }
    hipcheck(hipHostMalloc((void**)&kr.hhost, sizeof(double) * 2 * (2 * (restart + 2) + 4)), "hipHostMalloc");
    for (auto& e : kr.ev)
        if (!e) hipcheck(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    kr.cap = restart;
    kr.n = n;
}

void ensure_krylov(phmg_ctx ctx, int restart) {
    const double* v = ctx->kry.V;
    ensure_krylov(ctx, ctx->kry, ctx->L[0].n, restart);
    if (ctx->kry.V != v) invalidate_slot_graphs(ctx);     // graphs captured on the old slots
}

// Restarted FGMRES (the reading of the solver paragraph of Section 4; see the
// ABI notes): matvec(x, alpha, z, beta, y) forms y = alpha A x + beta z,
// precond(v, z) forms z = B v.  CGS2 on the device, Hessenberg and Givens on
// the host.  The next basis vector is normalised with the device norm, so the
// GPU work of iteration j + 1 is enqueued before the host waits for the
// projections of iteration j (one iteration of look-ahead): the host's Givens
// step and the copy latency overlap GPU work.  When iteration j ends the cycle
// the look-ahead iteration's results are simply not used (its writes go to
// Z_{j+1}, V_{j+2}, w and the scalar slots only).
template <class MatVec, class Prec>
phmg_status fgmres_core(hipStream_t s, Krylov& kr, int64_t n, MatVec matvec, Prec precond, const double* b,
                        double* x, double rtol, int restart, int maxit, int* iters_out, double* relres_out) {
    double* V = kr.V;
    double* Z = kr.Z;
    double* w = kr.w;
    double* r = kr.r;
    const int hs = 2 * (restart + 2) + 1;        // scalars copied per iteration
    const int slot = 2 * (kr.cap + 2) + 4;       // host slot stride
    double* h1 = kr.hdev;
    double* h2 = kr.hdev + (restart + 2);
    double* hn2 = kr.hdev + 2 * (restart + 2);

    matvec(x, -1.0, b, 1.0, r);
    double beta = device_norm(s, kr, n, r);
    if (!std::isfinite(beta)) fail(PHMG_EINVAL, "b or the initial x holds a NaN or Inf (||b - K x_0|| is not finite)");
    const double r0 = beta;
    const double target = rtol * r0;
    int iters = 0;
    if (r0 == 0.0 || beta <= target) {
        *iters_out = 0;
        *relres_out = r0 == 0.0 ? 0.0 : beta / r0;
        return PHMG_OK;
    }
    bool converged = false;
    std::vector<double> H((restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), y(restart);
    auto Hij = [&](int i, int j) -> double& { return H[(size_t)j * (restart + 1) + i]; };
    // enqueue the GPU work of iteration j: Z_j = B V_j, w = A Z_j, CGS2 projections,
    // copy to host slot j % 2, V_{j+1} = w / ||w|| (when a further basis vector exists)
    auto issue = [&](int j) {
        double* vj = V + (int64_t)j * n;
        double* zj = Z + (int64_t)j * n;
        precond(vj, zj);
        matvec(zj, 1.0, nullptr, 0.0, w);
        cgs2(s, kr.partial, n, j + 1, V, w, h1, h2, hn2);
        hipcheck(hipMemcpyAsync(kr.hhost + (j & 1) * slot, kr.hdev, sizeof(double) * hs, hipMemcpyDeviceToHost, s),
                 "D2H");
        hipcheck(hipEventRecord(kr.ev[j & 1], s), "hipEventRecord");
        if (j + 1 <= restart - 1) launch_scale_by_devnorm(s, n, w, hn2, V + (int64_t)(j + 1) * n);
    };
    for (;;) {
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        launch_scale_copy(s, n, r, beta, V);
        int ncols = 0;
        double hn = 0.0;
        issue(0);
        for (int j = 0; j < restart; ++j) {
            if (j + 1 < restart && iters + 1 < maxit) issue(j + 1);      // look-ahead
            hipcheck(hipEventSynchronize(kr.ev[j & 1]), "hipEventSynchronize");
            const double* hh1 = kr.hhost + (j & 1) * slot;
            const double* hh2 = hh1 + (restart + 2);
            hn = std::sqrt(hh1[2 * (restart + 2)]);
            for (int i = 0; i <= j; ++i) Hij(i, j) = hh1[i] + hh2[i];
            Hij(j + 1, j) = hn;
            for (int i = 0; i < j; ++i) {
                const double a = Hij(i, j), c = Hij(i + 1, j);
                Hij(i, j) = cs[i] * a + sn[i] * c;
                Hij(i + 1, j) = -sn[i] * a + cs[i] * c;
            }
            const double a = Hij(j, j), c = Hij(j + 1, j);
            const double rho = std::hypot(a, c);
            cs[j] = a / rho;
            sn[j] = c / rho;
            Hij(j, j) = rho;
            Hij(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++iters;
            ncols = j + 1;
            if (std::fabs(g[j + 1]) <= target || hn == 0.0 || iters >= maxit) break;
        }
        for (int i = ncols - 1; i >= 0; --i) {
            double acc = g[i];
            for (int k = i + 1; k < ncols; ++k) acc -= Hij(i, k) * y[k];
            y[i] = acc / Hij(i, i);
        }
        double* yd = h2;   // the y coefficients reuse h' (stream order: after any look-ahead work)
        hipcheck(hipMemcpyAsync(yd, y.data(), sizeof(double) * ncols, hipMemcpyHostToDevice, s), "H2D");
        launch_gemv_add(s, n, ncols, Z, n, yd, x);
        matvec(x, -1.0, b, 1.0, r);
        beta = device_norm(s, kr, n, r);
        if (beta <= target) {
            converged = true;
            break;
        }
        if (iters >= maxit) break;
        // restart: cycle exhausted, optimistic Givens estimate, or exact breakdown
    }
    *iters_out = iters;
    *relres_out = beta / r0;
    return converged ? PHMG_OK : PHMG_ENOCONV;
}

// transpose: the adjoint solve K^T x = b, right-preconditioned by B^T.
phmg_status fgmres(phmg_ctx ctx, const double* b, double* x, double rtol, int restart, int maxit, int* iters_out,
                   double* relres_out, bool transpose = false) {
    Level& L0 = ctx->L[0];
    hipStream_t s = ctx->stream;
    ensure_krylov(ctx, restart);
    const DevCsr& A = transpose ? L0.KT : L0.K;
    auto matvec = [&](const double* xx, double alpha, const double* z, double beta, double* y) {
        launch_spmv(s, A, xx, alpha, z, beta, y);
    };
    auto prec = [&](const double* v, double* z) { precond_slot(ctx, v, z, transpose); };
    return fgmres_core(s, ctx->kry, L0.n, matvec, prec, b, x, rtol, restart, maxit, iters_out, relres_out);
}

void destroy_all(phmg_ctx ctx) {
    invalidate_graph(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (auto st : ctx->sstreams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (auto e : ctx->sevents) (void)hipEventDestroy(e);
    for (auto e : ctx->fork_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->status_host) (void)hipHostFree(ctx->status_host);
    for (auto& it : ctx->prof.pending) {
        (void)hipEventDestroy(it.e0);
        (void)hipEventDestroy(it.e1);
    }
    for (auto e : ctx->prof.pool) (void)hipEventDestroy(e);
    for (void* p : ctx->allocs) (void)hipFree(p);
    if (ctx->kry.hhost) (void)hipHostFree(ctx->kry.hhost);
    for (auto e : ctx->kry.ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->bhhost) (void)hipHostFree(ctx->bhhost);
    delete ctx;
}

}  // namespace

extern "C" {

const char* phmg_last_error(void) { return g_last_error.c_str(); }

phmg_status phmg_ritz_max_real(const double* H, int ldh, int k, double* out) {
    return guarded([&]() -> phmg_status {
        if (!H || !out || k < 1 || ldh < k) fail(PHMG_EINVAL, "invalid Hessenberg matrix arguments");
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < k; ++i)
                if (!std::isfinite(H[(size_t)j * ldh + i])) fail(PHMG_EINVAL, "non-finite Hessenberg entry");
        *out = ritz_max_real(H, ldh, k);
        return PHMG_OK;
    });
}

phmg_status phmg_hierarchy_create(const phmg_hierarchy_desc* desc, const phmg_cycle_opts* opts, void* stream,
                                  phmg_ctx* out) {
    phmg_ctx ctx = nullptr;
    phmg_status st = guarded([&]() -> phmg_status {
        if (!desc || !opts || !out) fail(PHMG_EINVAL, "null argument");
        *out = nullptr;
        const int nl = desc->nlevels;
        if (nl < 2 || nl > PHMG_MAX_LEVELS) fail(PHMG_EINVAL, "nlevels must be in [2, 16]");
        if (!desc->K || !desc->P || !desc->patches) fail(PHMG_EINVAL, "null level array");
        if (opts->nu_p < 0 || opts->nu_h < 0 || opts->n_v < 1 || opts->n_plevels < 0 || opts->n_plevels > nl - 1 ||
            !std::isfinite(opts->omega))
            fail(PHMG_EINVAL, "invalid cycle options");
        if (opts->smoother != PHMG_SMOOTHER_RICHARDSON && opts->smoother != PHMG_SMOOTHER_CHEBYSHEV)
            fail(PHMG_EINVAL, "invalid cycle options: unknown smoother");
        if (opts->smoother == PHMG_SMOOTHER_CHEBYSHEV &&
            (opts->eig_iters < 1 || !(opts->cheb_lo >= 0.0) || !(opts->cheb_hi > opts->cheb_lo) ||
             !std::isfinite(opts->cheb_hi)))
            fail(PHMG_EINVAL, "invalid cycle options: Chebyshev needs eig_iters >= 1 and 0 <= cheb_lo < cheb_hi");
        // --- validation (host, before any device work)
        for (int l = 0; l < nl; ++l) {
            const phmg_csr& K = desc->K[l];
            check_csr(K, lvl(l) + "K: ");
            if (K.nrows != K.ncols || K.nrows < 1) fail(PHMG_EINVAL, lvl(l) + "K must be square and non-empty");
        }
        for (int l = 0; l + 1 < nl; ++l) {
            const phmg_csr& P = desc->P[l];
            check_csr(P, lvl(l) + "P: ");
            if (P.nrows != desc->K[l].nrows || P.ncols != desc->K[l + 1].nrows)
                fail(PHMG_EINVAL, lvl(l) + "P must be n_l x n_{l+1}");
            const phmg_patches& pt = desc->patches[l];
            if (pt.npatch < 1 || !pt.ptr || !pt.dofs) fail(PHMG_EINVAL, lvl(l) + "missing patches");
            if (pt.ptr[0] != 0) fail(PHMG_EINVAL, lvl(l) + "patch ptr[0] != 0");
            const int32_t n = desc->K[l].nrows;
            for (int32_t i = 0; i < pt.npatch; ++i) {
                const int64_t m = pt.ptr[i + 1] - pt.ptr[i];
                if (m < 1 || m > PHMG_MAX_PATCH)
                    fail(PHMG_EINVAL, lvl(l) + "patch " + std::to_string(i) + " size " + std::to_string(m) +
                                          " outside [1, " + std::to_string(PHMG_MAX_PATCH) + "]");
                for (int64_t t = pt.ptr[i]; t < pt.ptr[i + 1]; ++t) {
                    const int32_t d = pt.dofs[t];
                    if (d < 0 || d >= n) fail(PHMG_EINVAL, lvl(l) + "patch " + std::to_string(i) + " dof out of range");
                    if (t > pt.ptr[i] && pt.dofs[t - 1] >= d)
                        fail(PHMG_EINVAL, lvl(l) + "patch " + std::to_string(i) + " dofs not strictly ascending");
                    if (pt.weight && !std::isfinite(pt.weight[t]))
                        fail(PHMG_EINVAL, lvl(l) + "patch " + std::to_string(i) + " non-finite weight");
                }
            }
            if (pt.ptr[pt.npatch] >= (int64_t)INT32_MAX) fail(PHMG_EINVAL, lvl(l) + "too many patch slots");
        }
        const int32_t nc = desc->K[nl - 1].nrows;
        if (nc > PHMG_MAX_COARSE)
            fail(PHMG_EINVAL, "coarsest level has " + std::to_string(nc) + " DoFs; the dense coarse solve supports at most " +
                                  std::to_string(PHMG_MAX_COARSE));
        if (desc->coarse_null)
            for (int32_t i = 0; i < nc; ++i)
                if (!std::isfinite(desc->coarse_null[i])) fail(PHMG_EINVAL, "non-finite coarse_null");

        ctx = new phmg_ctx_s();
        ctx->stream = (hipStream_t)stream;
        hipcheck(hipGetDevice(&ctx->device), "hipGetDevice");
        noalloc_init_current_device();
        ctx->opts = *opts;
        ctx->L.resize(nl);
        for (int l = 0; l < nl; ++l) {
            Level& L = ctx->L[l];
            L.n = desc->K[l].nrows;
            L.K = upload_csr(ctx, desc->K[l]);
            // K^T for the adjoint path: the same arrays when K is symmetric (the
            // Stokes matrices are), otherwise an explicit transposed copy
            L.KT = is_symmetric(desc->K[l]) ? L.K : upload_transpose(ctx, desc->K[l]);
            L.sym_ok = near_symmetric(desc->K[l]);
            L.r = dalloc<double>(ctx, L.n);
            L.d = dalloc<double>(ctx, L.n);
            L.status = dalloc<int>(ctx, 1);
            if (l > 0) {
                L.b = dalloc<double>(ctx, L.n);
                L.x = dalloc<double>(ctx, L.n);
            }
            if (l + 1 < nl) {
                L.P = upload_csr(ctx, desc->P[l]);
                {
                    HostCsr R = host_transpose(desc->P[l]);
                    L.R = upload_csr(ctx, R.nrows, R.ncols, R.rp, R.ci, R.v);
                    // the restricted residual R (b - K x) = R b - (R K) x in one pass when
                    // R K is not larger than K (the cycle never needs the fine residual itself)
                    HostCsr RK = host_product(R, desc->K[l]);
                    if ((int64_t)RK.ci.size() <= L.K.nnz)
                        L.RK = upload_csr(ctx, RK.nrows, RK.ncols, RK.rp, RK.ci, RK.v);
                }
                const phmg_patches& pt = desc->patches[l];
                L.npatch = pt.npatch;
                L.sum_m = pt.ptr[pt.npatch];
                std::vector<int64_t> foff(pt.npatch);
                std::vector<int32_t> order(pt.npatch);
                int64_t acc = 0;
                int32_t mx = 0;
                for (int32_t i = 0; i < pt.npatch; ++i) {
                    const int64_t m = pt.ptr[i + 1] - pt.ptr[i];
                    foff[i] = acc;
                    acc += m * m;
                    mx = std::max<int32_t>(mx, (int32_t)m);
                    order[i] = i;
                }
                L.sum_m2 = acc;
                L.max_m = mx;
                for (int32_t i = 0; i < pt.npatch; ++i) {
                    const int64_t m = pt.ptr[i + 1] - pt.ptr[i];
                    for (int pr = PHMG_PREC_F64; pr <= PHMG_PREC_BF16; ++pr) {
                        const int V = factor_pad_of(pr);
                        L.sum_lp[pr] += (m + V - 1) / V * V * m;
                        L.sum_ls[pr] += sym_layout_size((int)m, V);
                    }
                }
                std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
                    return pt.ptr[a + 1] - pt.ptr[a] > pt.ptr[b + 1] - pt.ptr[b];
                });
                // inversion kernel classes: consecutive ranges of the launch order (decreasing m)
                for (int32_t i = 0; i < pt.npatch; ++i) {
                    const int64_t m = pt.ptr[order[i] + 1] - pt.ptr[order[i]];
                    const int c = gj_class(m, mx);
                    L.gj_cnt[c]++;
                    L.gj_max[c] = std::max<int32_t>(L.gj_max[c], (int32_t)m);
                }
                // DoF -> slots, ascending slot (= ascending patch id) per DoF
                std::vector<int32_t> sptr(L.n + 1, 0), sslot(L.sum_m);
                for (int64_t t = 0; t < L.sum_m; ++t) sptr[pt.dofs[t] + 1]++;
                for (int32_t j = 0; j < L.n; ++j) sptr[j + 1] += sptr[j];
                std::vector<int32_t> pos(sptr.begin(), sptr.end() - 1);
                for (int64_t t = 0; t < L.sum_m; ++t) sslot[pos[pt.dofs[t]]++] = (int32_t)t;
                L.pptr = upload(ctx, pt.ptr, pt.npatch + 1);
                L.hptr.assign(pt.ptr, pt.ptr + pt.npatch + 1);
                L.pdofs = upload(ctx, pt.dofs, L.sum_m);
                // pivot lists start as the identity, so a patch whose inversion stops
                // (singular) keeps valid indices for every later gather
                L.pdofs_perm = upload(ctx, pt.dofs, L.sum_m);
                {
                    std::vector<int32_t> ident(L.sum_m);
                    for (int32_t i = 0; i < pt.npatch; ++i)
                        for (int64_t t = pt.ptr[i]; t < pt.ptr[i + 1]; ++t) ident[t] = (int32_t)(t - pt.ptr[i]);
                    L.pidx = upload(ctx, ident.data(), L.sum_m);
                }
                L.ptol = dalloc<double>(ctx, pt.npatch);
                L.pweight = pt.weight ? upload(ctx, pt.weight, L.sum_m) : nullptr;
                L.foff = upload(ctx, foff.data(), pt.npatch);
                L.order = upload(ctx, order.data(), pt.npatch);
                L.horder = order;
                L.sptr = upload(ctx, sptr.data(), L.n + 1);
                L.sslot = upload(ctx, sslot.data(), L.sum_m);
                {
                    std::vector<int32_t> s4((size_t)L.n * 4, -1);
                    for (int32_t j = 0; j < L.n; ++j)
                        for (int32_t k = sptr[j], u = 0; k < sptr[j + 1] && u < 4; ++k, ++u) s4[(size_t)j * 4 + u] = sslot[k];
                    L.sslot4 = upload(ctx, s4.data(), (int64_t)L.n * 4);
                }
                if (pt.weight) {
                    // weights that depend on the DoF alone (e.g. 1 / number of patches
                    // holding it): sum_i w_ij y_ij = w_j sum_i y_ij, one weight per DoF
                    std::vector<double> wd(L.n, 1.0);
                    bool per_dof = true;
                    for (int32_t j = 0; j < L.n && per_dof; ++j)
                        for (int32_t k = sptr[j]; k < sptr[j + 1]; ++k) {
                            if (k == sptr[j]) wd[j] = pt.weight[sslot[k]];
                            else if (pt.weight[sslot[k]] != wd[j]) per_dof = false;
                        }
                    if (per_dof) L.wdof = upload(ctx, wd.data(), L.n);
                }
                L.Y = dalloc<double>(ctx, L.sum_m);
            } else {
                L.nb = desc->coarse_null ? L.n + 1 : L.n;
                if (desc->coarse_null) L.cnull = upload(ctx, desc->coarse_null, L.n);
            }
        }
        ctx->kry.partial = dalloc<double>(ctx, (int64_t)kRedBlocks * 4);
        ctx->kry.partial_cols = 4;
        ctx->scal = dalloc<double>(ctx, 8);
        ctx->L[0].x = dalloc<double>(ctx, ctx->L[0].n);   // level-0 work vector (level 0 has no cycle x)
        *out = ctx;
        return PHMG_OK;
    });
    if (st != PHMG_OK && ctx) {
        destroy_all(ctx);
        if (out) *out = nullptr;
    }
    return st;
}

phmg_status phmg_hierarchy_destroy(phmg_ctx ctx) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        (void)hipStreamSynchronize(ctx->stream);
        destroy_all(ctx);
        return PHMG_OK;
    });
}

phmg_status phmg_set_patch_storage(phmg_ctx ctx, int level, phmg_storage storage) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        if (level < 0 || level >= (int)ctx->L.size() - 1) fail(PHMG_EINVAL, "level out of range");
        if (storage != PHMG_STORAGE_AUTO && storage != PHMG_STORAGE_GENERAL) fail(PHMG_EINVAL, "unknown storage");
        Level& L = ctx->L[level];
        if (L.storage != storage) {
            L.storage = storage;
            L.ready = false;
            invalidate_graph(ctx);
        }
        return PHMG_OK;
    });
}

phmg_status phmg_set_precision(phmg_ctx ctx, int level, phmg_precision prec) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        if (level < 0 || level >= (int)ctx->L.size() - 1) fail(PHMG_EINVAL, "level out of range");
        if (prec != PHMG_PREC_F64 && prec != PHMG_PREC_F32 && prec != PHMG_PREC_BF16)
            fail(PHMG_EINVAL, "unknown precision");
        Level& L = ctx->L[level];
        if (L.prec != prec) {
            L.prec = prec;
            L.ready = false;
            invalidate_graph(ctx);
        }
        return PHMG_OK;
    });
}

phmg_status phmg_set_graphs(phmg_ctx ctx, int on) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        ctx->use_graphs = on != 0;
        if (!ctx->use_graphs) invalidate_graph(ctx);
        return PHMG_OK;
    });
}

phmg_status phmg_relax_setup(phmg_ctx ctx, int level) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        const int nl = (int)ctx->L.size();
        if (level >= nl) fail(PHMG_EINVAL, "level out of range");
        if (level < 0) setup_levels(ctx, 0, nl);
        else setup_levels(ctx, level, level + 1);
        return PHMG_OK;
    });
}

phmg_status phmg_relax_apply(phmg_ctx ctx, int level, const double* b, double* x, int nu) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !b || !x) fail(PHMG_EINVAL, "null argument");
        if (level < 0 || level >= (int)ctx->L.size() - 1) fail(PHMG_EINVAL, "level out of range (coarsest has no patches)");
        if (nu < 0) fail(PHMG_EINVAL, "nu < 0");
        if (!ctx->L[level].ready) fail(PHMG_ESTATE, lvl(level) + "relax_setup has not been run");
        relax(ctx, level, b, x, nu, false);
        hipcheck(hipGetLastError(), "kernel launch");
        return PHMG_OK;
    });
}

phmg_status phmg_vcycle(phmg_ctx ctx, const double* b, double* x) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !b || !x) fail(PHMG_EINVAL, "null argument");
        require_ready(ctx);
        precond(ctx, b, x, false);
        hipcheck(hipGetLastError(), "kernel launch");
        return PHMG_OK;
    });
}

phmg_status phmg_fgmres_solve(phmg_ctx ctx, const double* b, double* x, double rtol, int restart, int maxit,
                              int* iters, double* relres) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !b || !x || !iters || !relres) fail(PHMG_EINVAL, "null argument");
        if (restart < 1 || maxit < 1 || !(rtol >= 0.0)) fail(PHMG_EINVAL, "invalid rtol / restart / maxit");
        require_ready(ctx);
        const phmg_status st = fgmres(ctx, b, x, rtol, restart, maxit, iters, relres);
        hipcheck(hipGetLastError(), "kernel launch");
        if (st == PHMG_ENOCONV) g_last_error = "FGMRES reached maxit without converging";
        return st;
    });
}

phmg_status phmg_relax_apply_transposed(phmg_ctx ctx, int level, const double* b, double* x, int nu) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !b || !x) fail(PHMG_EINVAL, "null argument");
        if (level < 0 || level >= (int)ctx->L.size() - 1) fail(PHMG_EINVAL, "level out of range (coarsest has no patches)");
        if (nu < 0) fail(PHMG_EINVAL, "nu < 0");
        if (!ctx->L[level].ready) fail(PHMG_ESTATE, lvl(level) + "relax_setup has not been run");
        relax(ctx, level, b, x, nu, false, true);
        hipcheck(hipGetLastError(), "kernel launch");
        return PHMG_OK;
    });
}

phmg_status phmg_vcycle_transposed(phmg_ctx ctx, const double* b, double* x) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !b || !x) fail(PHMG_EINVAL, "null argument");
        require_ready(ctx);
        precond(ctx, b, x, true);
        hipcheck(hipGetLastError(), "kernel launch");
        return PHMG_OK;
    });
}

phmg_status phmg_fgmres_solve_transposed(phmg_ctx ctx, const double* b, double* x, double rtol, int restart,
                                         int maxit, int* iters, double* relres) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !b || !x || !iters || !relres) fail(PHMG_EINVAL, "null argument");
        if (restart < 1 || maxit < 1 || !(rtol >= 0.0)) fail(PHMG_EINVAL, "invalid rtol / restart / maxit");
        require_ready(ctx);
        const phmg_status st = fgmres(ctx, b, x, rtol, restart, maxit, iters, relres, true);
        hipcheck(hipGetLastError(), "kernel launch");
        if (st == PHMG_ENOCONV) g_last_error = "FGMRES (transposed) reached maxit without converging";
        return st;
    });
}

phmg_status phmg_set_sensitivities(phmg_ctx ctx, const phmg_csr* S, const phmg_csr* G) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !S || !G) fail(PHMG_EINVAL, "null argument");
        const DevCsr& K0 = ctx->L[0].K;
        check_csr(*S, "sensitivities: ");
        check_csr(*G, "forcing map: ");
        if (S->ncols != K0.nnz)
            fail(PHMG_EINVAL, "sensitivities: ncols must equal nnz(K_0) = " + std::to_string(K0.nnz));
        if (G->nrows != ctx->L[0].n) fail(PHMG_EINVAL, "forcing map: nrows must equal n_0");
        if (ctx->have_sens) {
            for (DevCsr* A : {&ctx->S, &ctx->G, &ctx->GT}) {
                dfree(ctx, A->rowptr);
                dfree(ctx, A->col);
                dfree(ctx, A->val);
            }
            dfree(ctx, ctx->wpair);
        }
        ctx->S = upload_csr(ctx, *S);
        ctx->G = upload_csr(ctx, *G);
        ctx->GT = upload_transpose(ctx, *G);
        ctx->wpair = dalloc<double>(ctx, K0.nnz);
        ctx->have_sens = true;
        return PHMG_OK;
    });
}

phmg_status phmg_forcing_rhs(phmg_ctx ctx, int nrhs, const double* F, double* B) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !F || !B) fail(PHMG_EINVAL, "null argument");
        if (!ctx->have_sens) fail(PHMG_ESTATE, "phmg_set_sensitivities has not been called");
        if (nrhs < 1) fail(PHMG_EINVAL, "nrhs must be >= 1");
        const int64_t nf = ctx->G.ncols, n0 = ctx->L[0].n;
        for (int c = 0; c < nrhs; ++c) launch_spmv(ctx->stream, ctx->G, F + c * nf, 1.0, nullptr, 0.0, B + c * n0);
        hipcheck(hipGetLastError(), "kernel launch");
        return PHMG_OK;
    });
}

phmg_status phmg_gradients(phmg_ctx ctx, int nrhs, const double* X, const double* Lam, double* grad_theta,
                           double* grad_f) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !X || !Lam || !grad_theta) fail(PHMG_EINVAL, "null argument");
        if (!ctx->have_sens) fail(PHMG_ESTATE, "phmg_set_sensitivities has not been called");
        if (nrhs < 1) fail(PHMG_EINVAL, "nrhs must be >= 1");
        hipStream_t s = ctx->stream;
        launch_pair_products(s, ctx->L[0].K, nrhs, X, Lam, ctx->wpair);
        launch_spmv(s, ctx->S, ctx->wpair, -1.0, nullptr, 0.0, grad_theta);
        if (grad_f) {
            const int64_t nf = ctx->G.ncols, n0 = ctx->L[0].n;
            for (int c = 0; c < nrhs; ++c)
                launch_spmv(s, ctx->GT, Lam + c * n0, 1.0, nullptr, 0.0, grad_f + c * nf);
        }
        hipcheck(hipGetLastError(), "kernel launch");
        return PHMG_OK;
    });
}

// ---------------------------------------------------------------------------
// Full block factorisation (Section 3.3, eq. "eq:fbf"):
// P^{-1} = [I -A~^{-1}B^T; 0 I] [A~^{-1} 0; 0 S~^{-1}] [I 0; -B A~^{-1} I],
// A~^{-1} one cycle of the velocity-block hierarchy, S~^{-1} a given matrix
// (the inverse block-diagonal pressure mass matrix, with the sign of the
// Schur complement -B A^{-1} B^T).
// ---------------------------------------------------------------------------

phmg_status phmg_fbf_create(phmg_ctx velocity, const phmg_csr* K, const phmg_csr* B, const phmg_csr* S_inv,
                            phmg_fbf* out) {
    return guarded([&]() -> phmg_status {
        if (!velocity || !K || !B || !S_inv || !out) fail(PHMG_EINVAL, "null argument");
        *out = nullptr;
        const int64_t nu = velocity->L[0].n;
        check_csr(*K, "fbf K: ");
        check_csr(*B, "fbf B: ");
        check_csr(*S_inv, "fbf S_inv: ");
        if (K->nrows != K->ncols) fail(PHMG_EINVAL, "fbf K: not square");
        const int64_t np = K->nrows - nu;
        if (np <= 0) fail(PHMG_EINVAL, "fbf K: not larger than the velocity block");
        if (B->nrows != np || B->ncols != nu) fail(PHMG_EINVAL, "fbf B: must be n_p x n_u");
        if (S_inv->nrows != np || S_inv->ncols != np) fail(PHMG_EINVAL, "fbf S_inv: must be n_p x n_p");
        auto* F = new phmg_fbf_s();
        try {
            F->A = velocity;
            F->mem.stream = velocity->stream;
            F->n = K->nrows;
            F->nu = nu;
            F->np = np;
            F->K = upload_csr(&F->mem, *K);
            F->B = upload_csr(&F->mem, *B);
            F->BT = upload_transpose(&F->mem, *B);
            F->Sinv = upload_csr(&F->mem, *S_inv);
            F->yu = dalloc<double>(&F->mem, nu);
            F->t = dalloc<double>(&F->mem, np);
            F->wu = dalloc<double>(&F->mem, nu);
            F->qu = dalloc<double>(&F->mem, nu);
        } catch (...) {
            for (void* p : F->mem.allocs) (void)hipFree(p);
            delete F;
            throw;
        }
        *out = F;
        return PHMG_OK;
    });
}

namespace {
void fbf_apply(phmg_fbf F, const double* r, double* z) {
    hipStream_t s = F->A->stream;
    const double* rp = r + F->nu;
    double* zp = z + F->nu;
    precond(F->A, r, F->yu, false);                             // y_u = A~^{-1} r_u
    launch_spmv(s, F->B, F->yu, -1.0, rp, 1.0, F->t);           // t = r_p - B y_u
    launch_spmv(s, F->Sinv, F->t, 1.0, nullptr, 0.0, zp);        // z_p = S~^{-1} t
    launch_spmv(s, F->BT, zp, 1.0, nullptr, 0.0, F->wu);         // w = B^T z_p
    precond(F->A, F->wu, F->qu, false);                         // q = A~^{-1} w
    launch_axpby(s, F->nu, 1.0, F->yu, -1.0, F->qu, z);          // z_u = y_u - q
}
}  // namespace

phmg_status phmg_fbf_apply(phmg_fbf fbf, const double* r, double* z) {
    return guarded([&]() -> phmg_status {
        if (!fbf || !r || !z) fail(PHMG_EINVAL, "null argument");
        require_ready(fbf->A);
        fbf_apply(fbf, r, z);
        hipcheck(hipGetLastError(), "kernel launch");
        return PHMG_OK;
    });
}

phmg_status phmg_fbf_fgmres_solve(phmg_fbf fbf, const double* b, double* x, double rtol, int restart, int maxit,
                                  int* iters, double* relres) {
    return guarded([&]() -> phmg_status {
        if (!fbf || !b || !x || !iters || !relres) fail(PHMG_EINVAL, "null argument");
        if (restart < 1 || maxit < 1 || !(rtol >= 0.0)) fail(PHMG_EINVAL, "invalid rtol / restart / maxit");
        require_ready(fbf->A);
        hipStream_t s = fbf->A->stream;
        fbf->mem.stream = s;
        ensure_krylov(&fbf->mem, fbf->kry, fbf->n, restart);
        auto matvec = [&](const double* xx, double alpha, const double* zz, double beta, double* y) {
            launch_spmv(s, fbf->K, xx, alpha, zz, beta, y);
        };
        auto prec = [&](const double* v, double* z) { fbf_apply(fbf, v, z); };
        const phmg_status st = fgmres_core(s, fbf->kry, fbf->n, matvec, prec, b, x, rtol, restart, maxit, iters,
                                           relres);
        hipcheck(hipGetLastError(), "kernel launch");
        if (st == PHMG_ENOCONV) g_last_error = "FGMRES (FBF) reached maxit without converging";
        return st;
    });
}

phmg_status phmg_fbf_destroy(phmg_fbf fbf) {
    if (!fbf) return PHMG_OK;
    for (void* p : fbf->mem.allocs) (void)hipFree(p);
    if (fbf->kry.hhost) (void)hipHostFree(fbf->kry.hhost);
    for (auto e : fbf->kry.ev)
        if (e) (void)hipEventDestroy(e);
    delete fbf;
    return PHMG_OK;
}

phmg_status phmg_set_kernel_vector(phmg_ctx ctx, const double* z) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        const int64_t n = ctx->L[0].n;
        if (!z) {
            dfree(ctx, ctx->z0);
            ctx->z0 = nullptr;
            ctx->z0z0 = 0.0;
            return PHMG_OK;
        }
        double zz = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!std::isfinite(z[i])) fail(PHMG_EINVAL, "kernel vector holds a NaN or Inf");
            zz += z[i] * z[i];
        }
        if (!(zz > 0.0)) fail(PHMG_EINVAL, "kernel vector is zero");
        if (!ctx->z0) ctx->z0 = dalloc<double>(ctx, n);
        if (!ctx->zpartial) {
            ctx->zpartial = dalloc<double>(ctx, (int64_t)kRedBlocks * kBS);
            ctx->zdots = dalloc<double>(ctx, kBS);
        }
        hipcheck(hipMemcpy(ctx->z0, z, sizeof(double) * (size_t)n, hipMemcpyHostToDevice), "hipMemcpy H2D");
        ctx->z0z0 = zz;
        return PHMG_OK;
    });
}

phmg_status phmg_project_kernel(phmg_ctx ctx, int nrhs, double* X) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !X) fail(PHMG_EINVAL, "null argument");
        if (nrhs < 1 || nrhs > PHMG_MAX_RHS) fail(PHMG_EINVAL, "nrhs must be in [1, 16]");
        if (!ctx->z0) fail(PHMG_ESTATE, "no kernel vector set (phmg_set_kernel_vector)");
        launch_project_off(ctx->stream, ctx->L[0].n, nrhs, X, ctx->z0, ctx->z0z0, ctx->zpartial, ctx->zdots);
        hipcheck(hipGetLastError(), "kernel launch");
        return PHMG_OK;
    });
}

phmg_status phmg_residual(phmg_ctx ctx, int level, const double* b, const double* x, double* r) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !b || !x || !r) fail(PHMG_EINVAL, "null argument");
        if (level < 0 || level >= (int)ctx->L.size()) fail(PHMG_EINVAL, "level out of range");
        launch_spmv(ctx->stream, ctx->L[level].K, x, -1.0, b, 1.0, r);
        hipcheck(hipGetLastError(), "kernel launch");
        return PHMG_OK;
    });
}

phmg_status phmg_get_level_info(phmg_ctx ctx, int level, phmg_level_info* info) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !info) fail(PHMG_EINVAL, "null argument");
        if (level < 0 || level >= (int)ctx->L.size()) fail(PHMG_EINVAL, "level out of range");
        const Level& L = ctx->L[level];
        info->n = L.n;
        info->npatch = L.npatch;
        info->max_m = L.max_m;
        info->precision = L.prec;
        info->nnz = L.K.nnz;
        info->sum_m = L.sum_m;
        info->sum_m2 = L.sum_m2;
        info->lambda_max = L.lmax;
        info->apply_variant = L.apply_variant;
        info->apply_variants = apply_variant_count(L);
        info->symmetric_storage = L.sym ? 1 : 0;
        info->spmv_variant = spmv_variant_of(L.K);
        info->stored_elements = L.npatch == 0 ? 0 : (L.sym ? L.sum_ls[L.prec] : L.sum_lp[L.prec]);
        const bool btuned = L.npatch > 0 && L.block_tuned_for == L.prec + (L.sym ? 3 : 0);
        info->block_variant = btuned ? L.block_variant : -1;
        info->block_variants = L.npatch > 0 ? block_variant_count(L) : 0;
        return PHMG_OK;
    });
}

phmg_status phmg_set_apply_variant(phmg_ctx ctx, int level, int variant) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        if (level < 0 || level >= (int)ctx->L.size() - 1) fail(PHMG_EINVAL, "level out of range");
        Level& L = ctx->L[level];
        if (variant < 0 || variant >= apply_variant_count(L)) fail(PHMG_EINVAL, "variant out of range");
        L.apply_variant = variant;
        L.tuned_for = tune_key(L);
        invalidate_graph(ctx);
        return PHMG_OK;
    });
}

phmg_status phmg_set_block_variant(phmg_ctx ctx, int level, int variant) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        if (level < 0 || level >= (int)ctx->L.size() - 1) fail(PHMG_EINVAL, "level out of range");
        Level& L = ctx->L[level];
        if (L.npatch == 0 || variant < 0 || variant >= block_variant_count(L))
            fail(PHMG_EINVAL, "variant out of range");
        L.block_variant = variant;
        L.block_tuned_for = L.prec + (L.sym ? 3 : 0);
        invalidate_block_graph(ctx);
        return PHMG_OK;
    });
}

phmg_status phmg_set_spmv_variant(phmg_ctx ctx, int level, int matrix, int variant) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        const int last = (int)ctx->L.size() - 1;
        if (level < 0 || level > last) fail(PHMG_EINVAL, "level out of range");
        if (matrix < 0 || matrix > 3 || (matrix > 0 && level == last)) fail(PHMG_EINVAL, "matrix out of range");
        Level& L = ctx->L[level];
        if (matrix == 3) {
            // the restricted residual: 0 two-step, 1-6 fused R b - (R K) x with 2 .. 64 lanes per row
            if (variant < 0 || variant > 6 || (variant > 0 && L.RK.nrows == 0)) fail(PHMG_EINVAL, "variant out of range");
            L.fuse_restrict = variant > 0;
            if (variant > 0) L.RK.group = 1 << variant;
            L.RK.tuned = true;
            invalidate_graph(ctx);
            return PHMG_OK;
        }
        DevCsr& A = matrix == 0 ? L.K : (matrix == 1 ? L.P : L.R);
        if (!spmv_variant_ok(A, variant)) fail(PHMG_EINVAL, "variant out of range");
        set_spmv_variant(A, variant);
        A.tuned = true;
        invalidate_graph(ctx);
        return PHMG_OK;
    });
}

phmg_status phmg_set_spmm_variant(phmg_ctx ctx, int level, int matrix, int variant) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        const int last = (int)ctx->L.size() - 1;
        if (level < 0 || level > last) fail(PHMG_EINVAL, "level out of range");
        if (matrix < 0 || matrix > 2 || (matrix > 0 && level == last)) fail(PHMG_EINVAL, "matrix out of range");
        if (variant < 0 || variant > 9) fail(PHMG_EINVAL, "variant out of range");
        Level& L = ctx->L[level];
        DevCsr& A = matrix == 0 ? L.K : (matrix == 1 ? L.P : L.R);
        if (variant < 6) {
            A.bquad = 0;
            A.bgroup = 1 << (variant % 3);
            A.bxcd = variant >= 3;
        } else {
            A.bquad = (variant - 6) % 2 == 0 ? 4 : 2;
            A.bxcd = variant >= 8;
        }
        A.btuned = true;
        invalidate_graph(ctx);
        return PHMG_OK;
    });
}

phmg_status phmg_profile_enable(phmg_ctx ctx, unsigned kernel_mask) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        ctx->prof.mask = kernel_mask & ((1u << PHMG_K_COUNT) - 1);
        return PHMG_OK;
    });
}

phmg_status phmg_profile_read(phmg_ctx ctx, int kernel, int level, double* total_ms, int64_t* launches) {
    return guarded([&]() -> phmg_status {
        if (!ctx || !total_ms || !launches) fail(PHMG_EINVAL, "null argument");
        if (kernel < 0 || kernel >= PHMG_K_COUNT) fail(PHMG_EINVAL, "unknown kernel id");
        if (level >= (int)ctx->L.size() || level >= PHMG_MAX_LEVELS) fail(PHMG_EINVAL, "level out of range");
        drain_profile(ctx);
        double ms = 0.0;
        int64_t cnt = 0;
        for (int l = 0; l < PHMG_MAX_LEVELS; ++l) {
            if (level >= 0 && l != level) continue;
            ms += ctx->prof.ms[kernel][l];
            cnt += ctx->prof.count[kernel][l];
        }
        *total_ms = ms;
        *launches = cnt;
        return PHMG_OK;
    });
}

phmg_status phmg_profile_reset(phmg_ctx ctx) {
    return guarded([&]() -> phmg_status {
        if (!ctx) fail(PHMG_EINVAL, "null context");
        drain_profile(ctx);
        for (int k = 0; k < PHMG_K_COUNT; ++k)
            for (int l = 0; l < PHMG_MAX_LEVELS; ++l) {
                ctx->prof.ms[k][l] = 0.0;
                ctx->prof.count[k][l] = 0;
            }
        return PHMG_OK;
    });
}

}  // extern "C"
