// Launch-configuration autotuner: times the candidate configurations of the
// projector kernels on the device for one loaded system matrix and keeps the
// fastest.
//
//  - B = 1 kernels: lanes per matrix row G in {4, 8, 16, 32, 64} for the
//    forward projection and for the back projection (+ update) kernel;
//  - B > 1 kernels (one 64-lane chunk): workgroups of the row-strided forward
//    grid, and the XCD-compact tile order of the step kernel.
//
// Each candidate runs once to warm up and is then timed three times with HIP
// events on the context's stream; the smallest time counts.  Environment
// overrides (APPGA_GROUP_FWD, APPGA_GROUP_BACK, APPGA_FWD_WGS, APPGA_XCD_REMAP)
// pin a parameter and take it out of the search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <functional>
#include <vector>

#include "appga.h"
#include "appga_impl.h"

using namespace appga;

namespace {

bool pinned(const char *name) {
    const char *s = std::getenv(name);
    return s && *s;
}

// Smallest of three timed runs of `launch` (after one warm-up), in microseconds.
hipError_t time_us(hipStream_t st, const std::function<hipError_t()> &launch, double *us) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = launch();
    double best = 1e30;
    for (int r = 0; r < 3 && e == hipSuccess; ++r) {
        e = hipEventRecord(a, st);
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) e = hipEventRecord(b, st);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        best = std::min(best, 1e3 * static_cast<double>(ms));
    }
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    *us = best;
    return e;
}

}  // namespace

namespace appga {

appga_status tune_matrix(appga_ctx *ctx, appga_matrix *mat, int flags, appga_tuning *out) {
    const int m = mat->A.n_rows, d = mat->A.n_cols, n = mat->geom.n;
    hipStream_t st = ctx->stream;
    appga_tuning res{};
    res.group_fwd = mat->group_fwd;
    res.group_back = mat->group_back;
    res.fwd_wgs = mat->fwd_wgs;
    res.xcd_remap = mat->xcd_remap;
    const int lanes = (flags & APPGA_TUNE_BATCH) ? 64 : 1;
    // vectors for the timed launches: x (d x lanes) and y (m x lanes), f~ and
    // the output of the back projection (d x lanes), per-lane parameters
    float *buf = nullptr;
    const size_t nfl = static_cast<size_t>(lanes) * (3 * static_cast<size_t>(d) + m) + 64;
    HIP_TRY(hipMalloc(&buf, sizeof(float) * nfl + sizeof(LaneParams) * 64));
    float *x = buf, *y = x + static_cast<size_t>(d) * lanes, *ft = y + static_cast<size_t>(m) * lanes,
          *outb = ft + static_cast<size_t>(d) * lanes, *theta = outb + static_cast<size_t>(d) * lanes;
    auto *lp = reinterpret_cast<LaneParams *>(buf + nfl);
    hipError_t e = launch_fill(buf, nfl, 1.0f, st);
    std::vector<LaneParams> hlp(64, LaneParams{0.01f, 0.01f, 1e-3f, 1.0f, 0.f, 0.f, 0.f, 0.f});
    if (e == hipSuccess) e = hipMemcpyAsync(lp, hlp.data(), sizeof(LaneParams) * 64, hipMemcpyHostToDevice, st);
    auto fwd_args = [&](int B) {
        FwdArgs fa{};
        fa.row_ptr = mat->A.row_ptr;
        fa.col = mat->A.col;
        fa.col32 = mat->A.col32;
        fa.nnz_padded = mat->A.nnz_padded;
        fa.val = mat->A.val;
        fa.row_scale = mat->A.row_scale;
        fa.m = m;
        fa.n_x = d;
        fa.B = B;
        fa.Bp = B == 1 ? 1 : 64;
        fa.x = x;
        fa.out = y;
        fa.mode = FM_PROJ;
        fa.fwd_wgs = mat->fwd_wgs;
        return fa;
    };
    auto back_args = [&](int B) {
        StepArgs sa{};
        sa.row_ptr = mat->AT.row_ptr;
        sa.col = mat->AT.col;
        sa.col32 = mat->AT.col32;
        sa.nnz_padded = mat->AT.nnz_padded;
        sa.val = mat->AT.val;
        sa.row_scale = mat->AT.row_scale;
        sa.n = n;
        sa.m = m;
        sa.B = B;
        sa.Bp = B == 1 ? 1 : 64;
        sa.e = y;
        sa.ft = ft;
        sa.f = x;
        sa.ft_next = ft;
        sa.lam = x;
        sa.lp = lp;
        sa.theta_next = theta;
        sa.pmode = PM_EM;
        sa.out_mode = SO_BACK;
        sa.out = outb;
        sa.tiles_x = (n + 3) / 4;
        sa.xcd_remap = mat->xcd_remap;
        return sa;
    };
    const int groups[] = {4, 8, 16, 32, 64};
    if (e == hipSuccess && (flags & APPGA_TUNE_SINGLE)) {
        if (!pinned("APPGA_GROUP_FWD")) {
            double best = 1e30;
            const FwdArgs fa = fwd_args(1);
            for (int g : groups) {
                double us = 0.0;
                e = time_us(st, [&] { return launch_forward_single(mat, fa, g, st); }, &us);
                if (e != hipSuccess) break;
                if (us < best) {
                    best = us;
                    res.group_fwd = g;
                }
            }
            res.us_fwd_single = best;
        }
        if (e == hipSuccess && !pinned("APPGA_GROUP_BACK")) {
            double best = 1e30;
            const StepArgs sa = back_args(1);
            for (int g : groups) {
                double us = 0.0;
                e = time_us(st, [&] { return launch_step_mat(mat, sa, g, st); }, &us);
                if (e != hipSuccess) break;
                if (us < best) {
                    best = us;
                    res.group_back = g;
                }
            }
            res.us_back_single = best;
        }
    }
    if (e == hipSuccess && (flags & APPGA_TUNE_BATCH)) {
        if (!pinned("APPGA_FWD_WGS")) {
            double best = 1e30;
            FwdArgs fa = fwd_args(64);
            for (int wgs : {1024, 2048, 4096, 8192}) {
                fa.fwd_wgs = wgs;
                double us = 0.0;
                e = time_us(st, [&] { return launch_forward(mat->A, fa, mat->group_fwd, st); }, &us);
                if (e != hipSuccess) break;
                if (us < best) {
                    best = us;
                    res.fwd_wgs = wgs;
                }
            }
            res.us_fwd_batch = best;
        }
        if (e == hipSuccess && !pinned("APPGA_XCD_REMAP") && mat->remap_ok) {
            double best = 1e30;
            StepArgs sa = back_args(64);
            for (int remap : {1, 0}) {
                sa.xcd_remap = remap;
                double us = 0.0;
                e = time_us(st, [&] { return launch_step(mat->AT, sa, mat->group_back, st); }, &us);
                if (e != hipSuccess) break;
                if (us < best) {
                    best = us;
                    res.xcd_remap = remap;
                }
            }
            res.us_step_batch = best;
        }
    }
    const hipError_t es = hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return fail(APPGA_E_DEVICE, "tuning launch failed: %s", hipGetErrorString(e));
    mat->group_fwd = res.group_fwd;
    mat->group_back = res.group_back;
    mat->fwd_wgs = res.fwd_wgs;
    mat->xcd_remap = res.xcd_remap;
    if (out) *out = res;
    return APPGA_OK;
}

}  // namespace appga

extern "C" appga_status appga_tune(appga_ctx *ctx, appga_matrix *mat, int32_t flags, appga_tuning *out) {
    clear_error();
    if (!ctx || !mat) return fail(APPGA_E_INVALID_ARG, "NULL ctx or matrix");
    if (mat->ctx != ctx) return fail(APPGA_E_INVALID_ARG, "matrix belongs to another context");
    if (flags & ~(APPGA_TUNE_SINGLE | APPGA_TUNE_BATCH)) return fail(APPGA_E_INVALID_ARG, "unknown tuning flags");
    if (mat->inflight.load() > 0) return fail(APPGA_E_BUSY, "matrix is used by in-flight server requests");
    HIP_TRY(hipSetDevice(ctx->device));
    return tune_matrix(ctx, mat, flags, out);
}
