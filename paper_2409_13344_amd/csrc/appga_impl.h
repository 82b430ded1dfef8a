// Definitions of the opaque ABI handles and the session helpers shared by
// appga_api.cpp and server.cpp.
#pragma once

#include <atomic>
#include <chrono>
#include <functional>
#include <string>
#include <vector>

#include "appga.h"
#include "appga_internal.h"

struct appga_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // kernel timing (appga_set_kernel_timing)
    bool timing = false;
    struct Pending {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<std::string> knames;
    std::vector<int64_t> kcount;
    std::vector<double> kms;
};

struct appga_matrix {
    appga_ctx *ctx = nullptr;
    appga_geometry geom{};
    int64_t nnz = 0;
    int storage = 0;
    appga::DevCsr A, AT;
    appga::DevGatherTiles bt;          // B > 1 back projection over pixel tiles (bt.valid = 0: none)
    appga::DevGatherTiles ft;          // B > 1 forward projection over ray tiles (ft.valid = 0: none)
    // B = 1 with quarter-turn symmetry: the first half of A's rows (angles below
    // 90 degrees) and their transpose; the other half is the first turned by 90
    // degrees (sym = 0: not used)
    int sym = 0;
    appga::DevCsr A_half, AT_half;
    float *lam = nullptr;              // Lambda (d), device
    std::vector<double> deq;           // dequantised values in the caller's CSR order
    std::vector<int64_t> user_row_ptr; // caller's CSR structure (for reports)
    std::vector<int32_t> user_col;
    int group_fwd = 16, group_back = 16;
    int xcd_remap = 0;
    int remap_ok = 0;                  // the 4 x 4 tile grid splits into 2 x 4 XCD blocks
    int bt_remap = 0;                  // XCD remap of the 8 x 8 tile grid
    int bt_split = 1;                  // workgroups (partial sums) per tile of the back projection
    int fwd_wgs = 2048;                // batched forward: workgroups of the row-strided grid
    mutable std::atomic<int> inflight{0};
    uint64_t serial = 0;               // unique per load (servers key their pools by it)
    // factored model (Section 4.1 physics): A = diag(row factors) G H with H a
    // Gaussian PSF of 2 psf_R + 1 taps per axis (psf_R < 0: no PSF)
    double psf_fwhm = 0.0;
    int psf_R = -1;
    float *psf_taps = nullptr;         // device, 2 psf_R + 1 floats
    bool has_row_factors = false;
};

struct appga_solve {
    appga_ctx *ctx = nullptr;
    const appga_matrix *mat = nullptr;
    int B = 0;
    int Bp = 1;  // padded lane count (1 for B = 1, else a multiple of 64)
    hipStream_t st = nullptr;
    std::vector<appga_params> prm;
    bool has_gamma = false, need_pbuf = false;
    void *arena = nullptr;
    float *g = nullptr, *gamma = nullptr, *gamma_lane = nullptr, *f = nullptr, *ft[2] = {nullptr, nullptr},
          *e = nullptr, *pbuf = nullptr, *theta = nullptr;
    float *gf = nullptr;   // A^T e from the tile kernel (B > 1 with tiles), else null
    float *tile_part = nullptr;  // partial sums of split forward tiles (B > 1), else null
    appga::LaneParams *lp = nullptr;
    double *part = nullptr, *red = nullptr, *tmc = nullptr;
    unsigned long long *clamps = nullptr;
    size_t part_len = 0;
    int theta_cap = 0, theta_base = 0;
    int k = 1, cur = 0;
    bool re_valid = false;
    std::vector<double> obj0;
    // objective monitor (monitor_every > 0): its own reduction buffers, and the
    // history of (k, Phi(f^k)) per solve, f^1 first
    int monitor_every = 0;
    double *mpart = nullptr, *mred = nullptr;
    std::vector<int32_t> hist_k;
    std::vector<double> hist_obj;   // [entry][B]
    std::chrono::steady_clock::time_point t0;
    // AFPPA sessions (Section 4.3): w = 2 f^{k+1} - f~, the duals (b, c) and their
    // extrapolation as 6 components per pixel, and three rotating sets of
    // per-solve accumulators of max P (kAfppaPmSlots each, FP32 bits)
    bool afppa = false;
    float *w = nullptr, *ydual = nullptr, *ybar = nullptr;
    // PSF sessions: H f~ (the forward's input), the blur's intermediate pass, and H A^T e
    float *xb = nullptr, *tb = nullptr, *gfb = nullptr;
    unsigned *pm = nullptr;
    int gf_split = 1;
    int re_blocks = 0;   // workgroups that wrote the RE partial sums of the last step
};

// Returns APPGA_E_DEVICE (with the failing call in the message) when a HIP
// call fails, and propagates a failed appga_status.
#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::appga::fail(APPGA_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define ST_TRY(expr)                        \
    do {                                    \
        appga_status s_ = (expr);           \
        if (s_ != APPGA_OK) return s_;      \
    } while (0)

namespace appga {

appga_status fail(appga_status st, const char *fmt, ...);
void clear_error();
// afppa: the nonsmooth model (Section 4.3): eps is unused, Nesterov momentum is
// allowed, the frozen EM preconditioner is not.
appga_status validate_params(const appga_params *p, bool afppa = false);
appga_status validate_data(const float *v, int64_t n, const char *what);
double theta_of(const appga_params &p, int k);
hipError_t timed_launch(appga_ctx *ctx, const char *name, hipStream_t st,
                        const std::function<hipError_t()> &fn);

appga_status sess_begin(appga_ctx *ctx, const appga_matrix *mat, int B, const float *d_g,
                        const float *d_gamma, const appga_params *params, const float *d_f_init,
                        hipStream_t st, appga_solve **out, bool afppa = false);
appga_status sess_step(appga_solve *s, int n_iters);
appga_status sess_end(appga_solve *s, float *d_out, appga_stats *stats, bool free_session);
appga_status tune_matrix(appga_ctx *ctx, appga_matrix *mat, int flags, appga_tuning *out);

// Forward projection: over the ray tiles when the matrix has them and the
// batch fills 64-lane chunks, else the row kernels.  *name (optional)
// receives the kernel timing name.
hipError_t launch_forward_mat(const appga_matrix *mat, const appga::FwdArgs &fa, hipStream_t st);
// B = 1 forward row kernel with `group` lanes per row on the stored matrix (the
// half-stored one with quarter-turn symmetry).
hipError_t launch_forward_single(const appga_matrix *mat, const appga::FwdArgs &fa, int group, hipStream_t st);
// The back-projection / step kernel on the matrix's stored transpose (the half-stored
// one for B = 1 with quarter-turn symmetry); `group` lanes per pixel row for B = 1.
hipError_t launch_step_mat(const appga_matrix *mat, const appga::StepArgs &sa, int group, hipStream_t st);
inline bool forward_uses_tiles(const appga_matrix *mat, const appga::FwdArgs &fa) {
    return mat->ft.valid && fa.Bp >= 64;
}
void sess_free(appga_solve *s);
// out = H in for a matrix with a PSF (in: n_parts partial sums; tmp: d * Bp floats).
hipError_t psf_blur(const appga_matrix *mat, const float *in, int n_parts, float *tmp, float *out, int B,
                    int Bp, hipStream_t st);

}  // namespace appga
