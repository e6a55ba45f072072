// Host runtime of the multi-right-hand-side (block) path: up to kBS systems
// K x_c = b_c relaxed, cycled and solved by FGMRES together.
//
// Every column runs exactly the single-system method (eq. "eq:ASM" sweeps,
// the cycles of Sections 3.1-3.2, FGMRES(30) of Section 4): the kernels never
// mix columns, and the block FGMRES keeps one Hessenberg matrix, Givens
// sequence and stopping test per column.  Sharing the sweeps is what pays:
// the patch inverses and the matrix entries are streamed once per sweep for
// all columns, so the patch solve becomes a dense product on MFMA.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "host_util.h"
#include "phmg_internal.h"

namespace phmg {

void invalidate_block_graph(phmg_ctx ctx) {
    for (int t = 0; t < 2; ++t) {
        if (ctx->bexec[t]) (void)hipGraphExecDestroy(ctx->bexec[t]);
        if (ctx->bgraph[t]) (void)hipGraphDestroy(ctx->bgraph[t]);
        ctx->bexec[t] = nullptr;
        ctx->bgraph[t] = nullptr;
    }
}

namespace {

// layout of ctx->bh (device) and ctx->bhhost (pinned host mirror)
constexpr int kHB = 32;                       // basis vectors the Gram-Schmidt kernels handle
constexpr int kOffH1 = 0;
constexpr int kOffH2 = kHB * kBS;
constexpr int kOffHN = 2 * kHB * kBS;
constexpr int kOffCS = 2 * kHB * kBS + kBS;   // column scales: den[kBS], active[kBS]
constexpr int kOffY = kOffCS + 2 * kBS;       // FGMRES update coefficients y[j * kBS + c]
constexpr int kBhLen = kOffY + kHB * kBS;

void ensure_block(phmg_ctx ctx) {
    if (ctx->block_ready) return;
    for (auto& L : ctx->L) {
        const int64_t nb = (int64_t)L.n * kBS;
        L.rb = dalloc<double>(ctx, nb);
        L.bb = dalloc<double>(ctx, nb);
        L.xb = dalloc<double>(ctx, nb);
        L.db = dalloc<double>(ctx, nb);
        if (L.npatch > 0) L.Yb = dalloc<double>(ctx, L.sum_m * kBS);
    }
    if (block_gs_max_basis() != kHB) fail(PHMG_EINVAL, "block Gram-Schmidt basis limit mismatch");
    ctx->bpartial = dalloc<double>(ctx, (int64_t)kBlockGsBlocks * kHB * kBS);
    ctx->bh = dalloc<double>(ctx, kBhLen);
    hipcheck(hipHostMalloc((void**)&ctx->bhhost, sizeof(double) * kBhLen), "hipHostMalloc");
    ctx->block_ready = true;
}

void ensure_block_krylov(phmg_ctx ctx, int restart) {
    if (ctx->brestart_cap >= restart) return;
    const int64_t nb = (int64_t)ctx->L[0].n * kBS;
    dfree(ctx, ctx->Vb);
    dfree(ctx, ctx->Zb);
    ctx->Vb = dalloc<double>(ctx, nb * (restart + 1));
    ctx->Zb = dalloc<double>(ctx, nb * restart);
    if (!ctx->wb) ctx->wb = dalloc<double>(ctx, nb);
    if (!ctx->rvb) ctx->rvb = dalloc<double>(ctx, nb);
    ctx->brestart_cap = restart;
}

float time_launch(hipStream_t s, hipEvent_t e0, hipEvent_t e1, const std::function<void()>& go) {
    go();                                                     // warm-up
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        hipcheck(hipEventRecord(e0, s), "hipEventRecord");
        go();
        hipcheck(hipEventRecord(e1, s), "hipEventRecord");
        hipcheck(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        hipcheck(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        best = std::min(best, ms);
    }
    return best;
}

// First-use autotuner of the block path: the shape of every block SpMM (groups
// of 16 lanes per row with 1, 2 or 4 entries in flight, or 2 / 4 lanes per row
// with 8 / 4 columns each; row ranges plain or XCD-contiguous), and the block
// patch-solve shape of every level for the level's precision (HIP events, best
// of three launches per candidate).
void tune_block(phmg_ctx ctx) {
    hipStream_t s = ctx->stream;
    hipEvent_t e0, e1;
    hipcheck(hipEventCreate(&e0), "hipEventCreate");
    hipcheck(hipEventCreate(&e1), "hipEventCreate");
    auto tune_csr = [&](DevCsr& A, const double* X, double* Y) {
        if (A.btuned || A.nrows == 0) return;
        int best = 1;
        bool best_x = false;
        int best_q = 0;
        float best_ms = 1e30f;
        A.bquad = 0;
        for (int xm = 0; xm < 2; ++xm)
            for (int g = 1; g <= 4; g *= 2) {
                A.bgroup = g;
                A.bxcd = xm != 0;
                const float ms = time_launch(s, e0, e1, [&] { launch_spmm(s, A, X, 1.0, nullptr, 0.0, Y); });
                if (ms < best_ms) {
                    best_ms = ms;
                    best = g;
                    best_x = xm != 0;
                }
            }
        A.bgroup = best;
        A.bxcd = best_x;
        for (int q = 2; q <= 4; q += 2)
            for (int xm = 0; xm < 2; ++xm) {
                A.bquad = q;
                A.bxcd = xm != 0;
                const float ms = time_launch(s, e0, e1, [&] { launch_spmm(s, A, X, 1.0, nullptr, 0.0, Y); });
                A.bquad = 0;
                if (ms < best_ms) {
                    best_ms = ms;
                    best_q = q;
                    best_x = xm != 0;
                }
            }
        A.bquad = best_q;
        A.bxcd = best_x;
        A.btuned = true;
    };
    const int last = (int)ctx->L.size() - 1;
    for (int l = 0; l < last; ++l) {
        Level& L = ctx->L[l];
        Level& C = ctx->L[l + 1];
        launch_fill(s, (int64_t)L.n * kBS, L.db, 1.0);
        launch_fill(s, (int64_t)C.n * kBS, C.xb, 1.0);
        tune_csr(L.K, L.db, L.rb);
        if (L.KT.rowptr != L.K.rowptr) tune_csr(L.KT, L.db, L.rb);
        tune_csr(L.R, L.db, C.bb);
        tune_csr(L.P, C.xb, L.rb);
        if (L.npatch > 0 && L.block_tuned_for != L.prec + (L.sym ? 3 : 0)) {
            int best = 0;
            float best_ms = 1e30f;
            for (int v = 0; v < block_variant_count(L); ++v) {
                L.block_variant = v;
                const float ms = time_launch(s, e0, e1, [&] { launch_block_apply(s, L, L.db); });
                if (ms < best_ms) {
                    best_ms = ms;
                    best = v;
                }
            }
            L.block_variant = best;
            L.block_tuned_for = L.prec + (L.sym ? 3 : 0);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hipcheck(hipGetLastError(), "block autotune launch");
}

// the block path is ready to run: set-up done, buffers allocated, shapes tuned
void prepare_block(phmg_ctx ctx) {
    require_ready(ctx);
    ensure_block(ctx);
    // general copies of the inverses of symmetric levels whose patches are too large
    // for the symmetric-layout block solve, converted from the f64 set-up buffer once
    // per set-up
    for (size_t l = 0; l + 1 < ctx->L.size(); ++l) {
        Level& L = ctx->L[l];
        if (!L.sym || L.npatch == 0 || block_sym_blocks(L) > 0 || L.bconv_count == L.setup_count) continue;
        const int V = factor_pad_of(L.prec);
        const size_t es = L.prec == PHMG_PREC_F64 ? 8 : (L.prec == PHMG_PREC_F32 ? 4 : 2);
        std::vector<int64_t> off(L.npatch);
        int64_t acc = 0;
        for (int32_t i = 0; i < L.npatch; ++i) {
            const int64_t m = L.hptr[i + 1] - L.hptr[i];
            off[i] = acc;
            acc += (m + V - 1) / V * V * m;
        }
        if (!L.bfoff) L.bfoff = dalloc<int64_t>(ctx, L.npatch);
        hipcheck(hipMemcpy(L.bfoff, off.data(), sizeof(int64_t) * (size_t)L.npatch, hipMemcpyHostToDevice),
                 "hipMemcpy H2D");
        const size_t bytes = es * (size_t)std::max<int64_t>(acc, 1);
        if (!L.bfactors || L.bfactor_bytes < bytes) {
            dfree(ctx, L.bfactors);
            L.bfactors = nullptr;
            L.bfactor_bytes = 0;
            L.bfactors = dalloc<char>(ctx, (int64_t)bytes);
            L.bfactor_bytes = bytes;
        }
        launch_convert_general(ctx->stream, L, L.work64, L.bfactors, L.bfoff);
        hipcheck(hipGetLastError(), "convert launch");
        L.bconv_count = L.setup_count;
    }
    bool stale = false;
    for (size_t l = 0; l + 1 < ctx->L.size(); ++l) {
        const Level& L = ctx->L[l];
        stale = stale || !L.K.btuned || (L.npatch > 0 && L.block_tuned_for != L.prec + (L.sym ? 3 : 0)) ||
                (L.KT.rowptr != L.K.rowptr && !L.KT.btuned);
    }
    if (stale) {
        invalidate_block_graph(ctx);
        tune_block(ctx);
    }
}

// nu smoothing steps on level l for all columns (the single-system relax with
// block kernels; the Chebyshev coefficients are shared by all columns).
void relax_block(phmg_ctx ctx, int l, const double* B, double* X, int nu, bool x_zero, bool transpose = false) {
    Level& L = ctx->L[l];
    hipStream_t s = ctx->stream;
    const int64_t nb = (int64_t)L.n * kBS;
    if (nu == 0) {
        if (x_zero) launch_fill(s, nb, X, 0.0);
        return;
    }
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
        const double* R = B;
        if (!(it == 0 && x_zero)) {
            Timed t(ctx, PHMG_K_SPMV, l);
            launch_spmm(s, transpose ? L.KT : L.K, X, -1.0, B, 1.0, L.rb);
            R = L.rb;
        }
        {
            Timed t(ctx, PHMG_K_PATCH_APPLY, l);
            launch_block_apply(s, L, R, transpose);
        }
        Timed t(ctx, PHMG_K_SCATTER, l);
        const bool xz = it == 0 && x_zero;
        if (!cheb) {
            launch_block_scatter(s, L, ctx->opts.omega, 0.0, nullptr, false, X, xz, transpose);
        } else if (it == 0) {
            launch_block_scatter(s, L, 1.0 / theta, 0.0, L.db, nu > 1, X, xz, transpose);
        } else {
            const double rho = 1.0 / (2.0 * sigma - rho_prev);
            launch_block_scatter(s, L, 2.0 * rho / delta, rho * rho_prev, L.db, it + 1 < nu, X, false, transpose);
            rho_prev = rho;
        }
    }
}

void cycle_block(phmg_ctx ctx, int l, const double* B, double* X, bool x_zero, bool transpose = false) {
    const int last = (int)ctx->L.size() - 1;
    hipStream_t s = ctx->stream;
    if (l == last) {
        launch_block_coarse_solve(s, ctx->L[l], B, X, transpose);
        return;
    }
    Level& L = ctx->L[l];
    Level& C = ctx->L[l + 1];
    const int np = ctx->opts.n_plevels;
    const int nu = l < np ? ctx->opts.nu_p : ctx->opts.nu_h;
    relax_block(ctx, l, B, X, nu, x_zero, transpose);
    {
        Timed t(ctx, PHMG_K_SPMV, l);
        launch_spmm(s, transpose ? L.KT : L.K, X, -1.0, B, 1.0, L.rb);
        launch_spmm(s, L.R, L.rb, 1.0, nullptr, 0.0, C.bb);
    }
    if (l + 1 < np || l + 1 == last || l >= np) {
        cycle_block(ctx, l + 1, C.bb, C.xb, true, transpose);
    } else {
        for (int t = 0; t < ctx->opts.n_v; ++t) cycle_block(ctx, l + 1, C.bb, C.xb, t == 0, transpose);
    }
    {
        Timed t(ctx, PHMG_K_SPMV, l);
        launch_spmm(s, L.P, C.xb, 1.0, X, 1.0, X);
    }
    relax_block(ctx, l, B, X, nu, false, transpose);
}

void vcycle_block(phmg_ctx ctx, const double* B, double* X, bool transpose = false) {
    if (ctx->opts.n_plevels == 0) {
        for (int t = 0; t < ctx->opts.n_v; ++t) cycle_block(ctx, 0, B, X, t == 0, transpose);
    } else {
        cycle_block(ctx, 0, B, X, true, transpose);
    }
}

// One block V-cycle (bgin -> bgout) captured on the private stream; kernels
// only, so a replay is exact.  Rebuilt whenever graph_signature() changes.
void build_block_graph(phmg_ctx ctx, bool transpose) {
    const int64_t nb = (int64_t)ctx->L[0].n * kBS;
    if (!ctx->cap_stream) hipcheck(hipStreamCreate(&ctx->cap_stream), "hipStreamCreate");
    if (!ctx->bgin) {
        ctx->bgin = dalloc<double>(ctx, nb);
        ctx->bgout = dalloc<double>(ctx, nb);
    }
    hipStream_t saved = ctx->stream;
    hipcheck(hipStreamSynchronize(saved), "hipStreamSynchronize");
    ctx->stream = ctx->cap_stream;
    hipcheck(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
        vcycle_block(ctx, ctx->bgin, ctx->bgout, transpose);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(ctx->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        ctx->stream = saved;
        throw;
    }
    ctx->stream = saved;
    const int t = transpose ? 1 : 0;
    hipcheck(hipStreamEndCapture(ctx->cap_stream, &ctx->bgraph[t]), "hipStreamEndCapture");
    hipcheck(hipGraphInstantiate(&ctx->bexec[t], ctx->bgraph[t], nullptr, nullptr, 0), "hipGraphInstantiate");
    ctx->bsig[t] = graph_signature(ctx);
}

void precond_block(phmg_ctx ctx, const double* B, double* X, bool transpose = false) {
    if (!ctx->use_graphs || ctx->prof.mask) {
        vcycle_block(ctx, B, X, transpose);
        return;
    }
    const int t = transpose ? 1 : 0;
    if (ctx->bexec[t] && ctx->bsig[t] != graph_signature(ctx)) {
        (void)hipGraphExecDestroy(ctx->bexec[t]);
        (void)hipGraphDestroy(ctx->bgraph[t]);
        ctx->bexec[t] = nullptr;
        ctx->bgraph[t] = nullptr;
    }
    if (!ctx->bexec[t]) build_block_graph(ctx, transpose);
    const int64_t nb = (int64_t)ctx->L[0].n * kBS;
    launch_copy(ctx->stream, nb, B, ctx->bgin);
    hipcheck(hipGraphLaunch(ctx->bexec[t], ctx->stream), "hipGraphLaunch");
    launch_copy(ctx->stream, nb, ctx->bgout, X);
}

// per-column ||v||^2 of a block vector into bhhost[kOffHN ...] (synchronises)
void block_norms(phmg_ctx ctx, double* v, double* out) {
    hipStream_t s = ctx->stream;
    const int64_t n = ctx->L[0].n;
    launch_block_gs(s, 2, n, 0, nullptr, 0, v, nullptr, ctx->bpartial, ctx->bh + kOffHN);
    hipcheck(hipMemcpyAsync(ctx->bhhost + kOffHN, ctx->bh + kOffHN, sizeof(double) * kBS, hipMemcpyDeviceToHost, s),
             "D2H");
    hipcheck(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int c = 0; c < kBS; ++c) out[c] = std::sqrt(ctx->bhhost[kOffHN + c]);
}

void upload_scales(phmg_ctx ctx, const double* den, const bool* act) {
    for (int c = 0; c < kBS; ++c) {
        ctx->bhhost[kOffCS + c] = den[c];
        ctx->bhhost[kOffCS + kBS + c] = act[c] ? 1.0 : 0.0;
    }
    hipcheck(hipMemcpyAsync(ctx->bh + kOffCS, ctx->bhhost + kOffCS, sizeof(double) * 2 * kBS, hipMemcpyHostToDevice,
                            ctx->stream),
             "H2D");
}

// Restarted FGMRES for the columns c < nrhs of the block B (X in/out), run in
// lockstep.  A column leaves the current cycle when its own Givens estimate
// reaches rtol ||r_0,c||, on an exact breakdown, or at maxit; it idles (zero
// basis column, so the shared preconditioner maps it to zero) until every
// column has left or the cycle is exhausted.  Then each column takes its own
// update and true residual and either stops or restarts: the iterates and
// counts of a column are those of the single-system FGMRES.
phmg_status fgmres_block(phmg_ctx ctx, int nrhs, const double* B, double* X, double rtol, int restart, int maxit,
                         int32_t* iters_out, double* relres_out, bool transpose = false) {
    Level& L0 = ctx->L[0];
    const int64_t n = L0.n;
    const int64_t nb = n * kBS;
    hipStream_t s = ctx->stream;
    ensure_block_krylov(ctx, restart);
    double* V = ctx->Vb;
    double* Z = ctx->Zb;
    double* w = ctx->wb;
    double* r = ctx->rvb;
    double* dh = ctx->bh;
    double* hh = ctx->bhhost;

    const DevCsr& A = transpose ? L0.KT : L0.K;
    launch_spmm(s, A, X, -1.0, B, 1.0, r);
    std::vector<double> beta(kBS), r0(kBS), target(kBS);
    block_norms(ctx, r, beta.data());
    std::vector<int> iters(kBS, 0);
    std::vector<bool> done(kBS, true), conv(kBS, false);
    for (int c = 0; c < nrhs; ++c)
        if (!std::isfinite(beta[c]))
            fail(PHMG_EINVAL, "system " + std::to_string(c) + ": b or the initial x holds a NaN or Inf "
                              "(||b - K x_0|| is not finite)");
    for (int c = 0; c < nrhs; ++c) {
        r0[c] = beta[c];
        target[c] = rtol * r0[c];
        if (r0[c] == 0.0 || beta[c] <= target[c]) {
            conv[c] = true;
        } else {
            done[c] = false;
        }
    }
    const int R1 = restart + 1;
    std::vector<double> H((size_t)kBS * R1 * restart), cs((size_t)kBS * restart), sn((size_t)kBS * restart),
        g((size_t)kBS * R1), y((size_t)kBS * restart);
    auto Hij = [&](int c, int i, int j) -> double& { return H[((size_t)c * restart + j) * R1 + i]; };
    std::vector<bool> act(kBS);
    std::vector<int> ncols(kBS);
    std::vector<double> den(kBS);
    for (;;) {
        bool any = false;
        for (int c = 0; c < kBS; ++c) {
            act[c] = !done[c];
            any = any || act[c];
            ncols[c] = 0;
            den[c] = act[c] ? beta[c] : 1.0;
        }
        if (!any) break;
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        for (int c = 0; c < kBS; ++c) g[(size_t)c * R1] = act[c] ? beta[c] : 0.0;
        {
            bool a[kBS];
            for (int c = 0; c < kBS; ++c) a[c] = act[c];
            upload_scales(ctx, den.data(), a);
        }
        launch_block_scale(s, n, r, dh + kOffCS, V);
        for (int j = 0; j < restart; ++j) {
            double* vj = V + (int64_t)j * nb;
            double* zj = Z + (int64_t)j * nb;
            precond_block(ctx, vj, zj, transpose);
            launch_spmm(s, A, zj, 1.0, nullptr, 0.0, w);
            launch_block_gs(s, 0, n, j + 1, V, nb, w, nullptr, ctx->bpartial, dh + kOffH1);
            launch_block_gs(s, 1, n, j + 1, V, nb, w, dh + kOffH1, ctx->bpartial, dh + kOffH2);
            launch_block_gs(s, 2, n, j + 1, V, nb, w, dh + kOffH2, ctx->bpartial, dh + kOffHN);
            hipcheck(hipMemcpyAsync(hh, dh, sizeof(double) * (kOffHN + kBS), hipMemcpyDeviceToHost, s), "D2H");
            hipcheck(hipStreamSynchronize(s), "hipStreamSynchronize");
            bool still = false;
            for (int c = 0; c < kBS; ++c) {
                if (!act[c]) continue;
                double* gc = &g[(size_t)c * R1];
                double* csc = &cs[(size_t)c * restart];
                double* snc = &sn[(size_t)c * restart];
                const double hn = std::sqrt(hh[kOffHN + c]);
                for (int i = 0; i <= j; ++i) Hij(c, i, j) = hh[kOffH1 + i * kBS + c] + hh[kOffH2 + i * kBS + c];
                Hij(c, j + 1, j) = hn;
                for (int i = 0; i < j; ++i) {
                    const double a = Hij(c, i, j), b = Hij(c, i + 1, j);
                    Hij(c, i, j) = csc[i] * a + snc[i] * b;
                    Hij(c, i + 1, j) = -snc[i] * a + csc[i] * b;
                }
                const double a = Hij(c, j, j), b = Hij(c, j + 1, j);
                const double rho = std::hypot(a, b);
                csc[j] = a / rho;
                snc[j] = b / rho;
                Hij(c, j, j) = rho;
                Hij(c, j + 1, j) = 0.0;
                gc[j + 1] = -snc[j] * gc[j];
                gc[j] = csc[j] * gc[j];
                ++iters[c];
                ncols[c] = j + 1;
                if (std::fabs(gc[j + 1]) <= target[c] || hn == 0.0 || iters[c] >= maxit) {
                    act[c] = false;
                } else {
                    den[c] = hn;
                    still = true;
                }
            }
            if (!still || j + 1 == restart) break;
            {
                bool a[kBS];
                for (int c = 0; c < kBS; ++c) a[c] = act[c];
                upload_scales(ctx, den.data(), a);
            }
            launch_block_scale(s, n, w, dh + kOffCS, V + (int64_t)(j + 1) * nb);
        }
        int nmax = 0;
        for (int c = 0; c < kBS; ++c) {
            double* yc = &y[(size_t)c * restart];
            std::fill(yc, yc + restart, 0.0);
            const double* gc = &g[(size_t)c * R1];
            for (int i = ncols[c] - 1; i >= 0; --i) {
                double acc = gc[i];
                for (int k = i + 1; k < ncols[c]; ++k) acc -= Hij(c, i, k) * yc[k];
                yc[i] = acc / Hij(c, i, i);
            }
            nmax = std::max(nmax, ncols[c]);
        }
        for (int j = 0; j < nmax; ++j)
            for (int c = 0; c < kBS; ++c) hh[kOffY + j * kBS + c] = y[(size_t)c * restart + j];
        hipcheck(hipMemcpyAsync(dh + kOffY, hh + kOffY, sizeof(double) * nmax * kBS, hipMemcpyHostToDevice, s),
                 "H2D");
        launch_block_gemv_add(s, n, nmax, Z, nb, dh + kOffY, X);
        launch_spmm(s, A, X, -1.0, B, 1.0, r);
        block_norms(ctx, r, beta.data());
        for (int c = 0; c < kBS; ++c) {
            if (done[c]) continue;
            if (beta[c] <= target[c]) {
                done[c] = true;
                conv[c] = true;
            } else if (iters[c] >= maxit) {
                done[c] = true;
            }
        }
    }
    bool all = true;
    for (int c = 0; c < nrhs; ++c) {
        iters_out[c] = iters[c];
        relres_out[c] = r0[c] == 0.0 ? 0.0 : beta[c] / r0[c];
        all = all && conv[c];
    }
    return all ? PHMG_OK : PHMG_ENOCONV;
}

// the batched adjoint applies K_i^{-1} as K_i^{-T}: every relaxed level must be
// symmetric to rounding (after set-up in the default layout)
void check_block_adjoint(phmg_ctx ctx) {
    for (size_t l = 0; l + 1 < ctx->L.size(); ++l)
        if (ctx->L[l].npatch > 0 && !ctx->L[l].sym)
            fail(PHMG_EINVAL, lvl((int)l) + "the batched adjoint needs symmetric levels in the symmetric layout; "
                                           "use phmg_fgmres_solve_transposed per system");
}

void check_block_args(phmg_ctx ctx, int level, int nrhs, const void* B, const void* X) {
    if (!ctx) fail(PHMG_EINVAL, "null context");
    if (level < 0 || level >= (int)ctx->L.size()) fail(PHMG_EINVAL, "level out of range");
    if (nrhs < 1 || nrhs > kBS) fail(PHMG_EINVAL, "nrhs must be in [1, " + std::to_string(kBS) + "]");
    if (!B || !X) fail(PHMG_EINVAL, "null vector");
    if (B == X) fail(PHMG_EINVAL, "B and X must not alias");
}

}  // namespace
}  // namespace phmg

using namespace phmg;

extern "C" {

phmg_status phmg_relax_apply_batched(phmg_ctx ctx, int level, int nrhs, const double* B, double* X, int nu) {
    return guarded([&] {
        check_block_args(ctx, level, nrhs, B, X);
        if (level == (int)ctx->L.size() - 1) fail(PHMG_EINVAL, lvl(level) + "the coarsest level has no patches");
        if (nu < 0) fail(PHMG_EINVAL, "nu must be >= 0");
        prepare_block(ctx);
        Level& L = ctx->L[level];
        hipStream_t s = ctx->stream;
        launch_interleave(s, L.n, nrhs, B, L.bb);
        launch_interleave(s, L.n, nrhs, X, L.xb);
        relax_block(ctx, level, L.bb, L.xb, nu, false);
        launch_deinterleave(s, L.n, nrhs, L.xb, X);
        hipcheck(hipGetLastError(), "relax_apply_batched launch");
        return PHMG_OK;
    });
}

phmg_status phmg_vcycle_batched(phmg_ctx ctx, int nrhs, const double* B, double* X) {
    return guarded([&] {
        check_block_args(ctx, 0, nrhs, B, X);
        prepare_block(ctx);
        Level& L = ctx->L[0];
        hipStream_t s = ctx->stream;
        launch_interleave(s, L.n, nrhs, B, L.bb);
        precond_block(ctx, L.bb, L.xb);
        launch_deinterleave(s, L.n, nrhs, L.xb, X);
        hipcheck(hipGetLastError(), "vcycle_batched launch");
        return PHMG_OK;
    });
}

namespace {
phmg_status fgmres_batched_entry(phmg_ctx ctx, int nrhs, const double* B, double* X, double rtol, int restart,
                                 int maxit, int32_t* iters, double* relres, bool transpose) {
    return guarded([&] {
        check_block_args(ctx, 0, nrhs, B, X);
        if (!iters || !relres) fail(PHMG_EINVAL, "null output");
        if (!(rtol > 0.0) || restart < 1 || restart >= kHB || maxit < 1)
            fail(PHMG_EINVAL, "need rtol > 0, 1 <= restart <= " + std::to_string(kHB - 1) + ", maxit >= 1");
        prepare_block(ctx);
        if (transpose) check_block_adjoint(ctx);
        Level& L = ctx->L[0];
        hipStream_t s = ctx->stream;
        launch_interleave(s, L.n, nrhs, B, L.bb);
        launch_interleave(s, L.n, nrhs, X, L.xb);
        const phmg_status st = fgmres_block(ctx, nrhs, L.bb, L.xb, rtol, restart, maxit, iters, relres, transpose);
        launch_deinterleave(s, L.n, nrhs, L.xb, X);
        hipcheck(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (st == PHMG_ENOCONV) g_last_error = "fgmres_solve_batched: maxit reached before rtol in some column";
        return st;
    });
}
}  // namespace

phmg_status phmg_fgmres_solve_batched(phmg_ctx ctx, int nrhs, const double* B, double* X, double rtol, int restart,
                                      int maxit, int32_t* iters, double* relres) {
    return fgmres_batched_entry(ctx, nrhs, B, X, rtol, restart, maxit, iters, relres, false);
}

phmg_status phmg_fgmres_solve_batched_transposed(phmg_ctx ctx, int nrhs, const double* B, double* X, double rtol,
                                                 int restart, int maxit, int32_t* iters, double* relres) {
    return fgmres_batched_entry(ctx, nrhs, B, X, rtol, restart, maxit, iters, relres, true);
}

phmg_status phmg_vcycle_batched_transposed(phmg_ctx ctx, int nrhs, const double* B, double* X) {
    return guarded([&] {
        check_block_args(ctx, 0, nrhs, B, X);
        prepare_block(ctx);
        check_block_adjoint(ctx);
        Level& L = ctx->L[0];
        hipStream_t s = ctx->stream;
        launch_interleave(s, L.n, nrhs, B, L.bb);
        precond_block(ctx, L.bb, L.xb, true);
        launch_deinterleave(s, L.n, nrhs, L.xb, X);
        hipcheck(hipGetLastError(), "vcycle_batched_transposed launch");
        return PHMG_OK;
    });
}

}  // extern "C"
