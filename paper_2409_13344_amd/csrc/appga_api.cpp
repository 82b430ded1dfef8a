// Host side of libappga: validation, system-matrix packing, solve sessions and
// the C ABI declared in include/appga.h.  Every step of the iteration runs in
// the HIP kernels of kernels.hip; this file only prepares data, launches and
// reduces the per-solve FP64 scalars.
#include "appga.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "appga_internal.h"
#include "appga_impl.h"
#include "gather_tiles.h"

using namespace appga;

// ---------------------------------------------------------------- errors ---

namespace appga {

static thread_local std::string g_last_error;

appga_status fail(appga_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

void clear_error() { g_last_error.clear(); }

}  // namespace appga

extern "C" const char *appga_last_error(void) { return g_last_error.c_str(); }

// --------------------------------------------------------- value coding ---

namespace {

uint16_t f32_to_bf16(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;  // round to nearest even (inputs are finite)
    return static_cast<uint16_t>(u >> 16);
}

float bf16_to_f32_host(uint16_t h) {
    const uint32_t u = static_cast<uint32_t>(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

uint16_t f32_to_f16(float x) {
    const _Float16 h = static_cast<_Float16>(x);
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}

float f16_to_f32_host(uint16_t u) {
    _Float16 h;
    std::memcpy(&h, &u, 2);
    return static_cast<float>(h);
}

// OCP FP8 E4M3 (bias 7, max 448, no infinities), round to nearest even, saturating.
uint8_t f32_to_e4m3(double x) {
    uint8_t sign = 0;
    if (x < 0) {
        sign = 0x80;
        x = -x;
    }
    if (x == 0.0) return sign;
    if (x >= 448.0) return sign | 0x7E;
    int e;
    const double fr = std::frexp(x, &e);  // x = fr 2^e, fr in [0.5, 1)
    int E = e - 1;                        // x = (2 fr) 2^E
    if (E < -6) {                         // subnormal: m 2^-9
        const double m = std::nearbyint(x * 512.0);
        if (m >= 8.0) return sign | 0x08;
        return sign | static_cast<uint8_t>(m);
    }
    double mant = std::nearbyint((2.0 * fr - 1.0) * 8.0);
    if (mant >= 8.0) {
        mant = 0.0;
        ++E;
    }
    if (E > 8 || (E == 8 && mant > 6.0)) return sign | 0x7E;
    return sign | static_cast<uint8_t>(((E + 7) << 3) | static_cast<int>(mant));
}

double e4m3_to_f64(uint8_t q) {
    const int s = q & 0x80 ? -1 : 1;
    const int e = (q >> 3) & 0xF, m = q & 7;
    if (e == 0) return s * m * std::ldexp(1.0, -9);
    return s * (1.0 + m / 8.0) * std::ldexp(1.0, e - 7);
}

int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

// -------------------------------------------------------------- context ---

namespace appga {

int kernel_id(appga_ctx *ctx, const char *name) {
    for (size_t i = 0; i < ctx->knames.size(); ++i)
        if (ctx->knames[i] == name) return static_cast<int>(i);
    ctx->knames.push_back(name);
    ctx->kcount.push_back(0);
    ctx->kms.push_back(0.0);
    return static_cast<int>(ctx->knames.size() - 1);
}

hipError_t timed_launch(appga_ctx *ctx, const char *name, hipStream_t st,
                        const std::function<hipError_t()> &fn) {
    if (!ctx->timing) return fn();
    hipEvent_t a, b;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) return e;
    if ((e = hipEventRecord(a, st)) != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(b, st)) != hipSuccess) return e;
    ctx->pending.push_back({kernel_id(ctx, name), a, b});
    return hipSuccess;
}

}  // namespace appga

extern "C" appga_status appga_params_default(appga_params *p) {
    if (!p) return fail(APPGA_E_INVALID_ARG, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->lambda1 = 0.0;
    p->lambda2 = 0.0;
    p->eps = 1e-3;
    p->omega = 1.0;
    p->a = 0.125;
    p->b = 1.0;
    p->beta = 1.0;
    p->iterations = 100;
    p->momentum = APPGA_MOMENTUM_GN;
    p->precond = APPGA_PRECOND_EM;
    p->precond_freeze_iter = 0;
    p->monitor_every = 0;
    p->fixed_p = 0.0;
    p->gamma_scalar = 0.0;
    return APPGA_OK;
}

extern "C" appga_status appga_create(appga_ctx **out, int device) {
    clear_error();
    if (!out) return fail(APPGA_E_INVALID_ARG, "ctx output pointer is NULL");
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(APPGA_E_INVALID_ARG, "device %d out of range (have %d)", device, ndev);
    HIP_TRY(hipSetDevice(device));
    appga_ctx *ctx = new appga_ctx();
    ctx->device = device;
    hipError_t e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete ctx;
        return fail(APPGA_E_DEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return APPGA_OK;
}

extern "C" appga_status appga_destroy(appga_ctx *ctx) {
    clear_error();
    if (!ctx) return fail(APPGA_E_INVALID_ARG, "ctx is NULL");
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    for (auto &p : ctx->pending) {
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    hipStreamDestroy(ctx->stream);
    delete ctx;
    return APPGA_OK;
}

extern "C" appga_status appga_set_kernel_timing(appga_ctx *ctx, int32_t enable) {
    clear_error();
    if (!ctx) return fail(APPGA_E_INVALID_ARG, "ctx is NULL");
    ctx->timing = enable != 0;
    return APPGA_OK;
}

extern "C" appga_status appga_kernel_times(appga_ctx *ctx, int32_t cap, char *names_out,
                                           int32_t names_cap, int64_t *counts, double *total_ms,
                                           int32_t *n_kernels) {
    clear_error();
    if (!ctx) return fail(APPGA_E_INVALID_ARG, "ctx is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    for (auto &p : ctx->pending) {
        HIP_TRY(hipEventSynchronize(p.b));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, p.a, p.b));
        ctx->kms[p.kernel] += ms;
        ctx->kcount[p.kernel] += 1;
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    ctx->pending.clear();
    const int nk = static_cast<int>(ctx->knames.size());
    if (n_kernels) *n_kernels = nk;
    int pos = 0;
    for (int i = 0; i < nk && i < cap; ++i) {
        if (counts) counts[i] = ctx->kcount[i];
        if (total_ms) total_ms[i] = ctx->kms[i];
        if (names_out) {
            const std::string &s = ctx->knames[i];
            if (pos + static_cast<int>(s.size()) + 1 <= names_cap) {
                std::memcpy(names_out + pos, s.c_str(), s.size() + 1);
                pos += static_cast<int>(s.size()) + 1;
            }
        }
    }
    return APPGA_OK;
}

// ------------------------------------------------------------- matrices ---

namespace {

struct HostPacked {
    std::vector<int32_t> row_ptr;
    std::vector<uint16_t> col16;
    std::vector<uint32_t> col32;
    std::vector<uint32_t> col32u;   // col * 256: byte offset of a column's 64-lane record (B > 1)
    std::vector<uint8_t> val;  // raw bytes of the stored values
    std::vector<float> scale;
    int max_len = 0;
};

// Packs CSR rows (original order within each row) into the padded stored
// form; `deq` (optional) receives the dequantised value of each original entry.
// FP8: per-row scale s_i = max_k |a_ik| / 448 (rounded to FP32) and the code of
// each entry, e4m3(a_ik / s_i), in the caller's CSR order.
void fp8_quantize(int64_t nrows, const int64_t *rp, const double *val, std::vector<uint8_t> &codes,
                  std::vector<float> &scales) {
    codes.assign(rp[nrows], 0);
    scales.assign(nrows, 1.0f);
    for (int64_t i = 0; i < nrows; ++i) {
        double mx = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) mx = std::max(mx, std::fabs(val[k]));
        const double sc = mx > 0.0 ? static_cast<double>(static_cast<float>(mx / 448.0)) : 1.0;
        scales[i] = static_cast<float>(sc);
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) codes[k] = f32_to_e4m3(val[k] / sc);
    }
}

// For FP8 `codes` holds one code per entry (CSR order of this operator) and
// `scales` the per-row scales, or NULL when the rows carry no scale (the
// transpose: its codes are A's, and A's row scales are applied to the residual
// the back projection reads, so A and A^T stay exact adjoints).
appga_status pack_rows(int64_t nrows, int64_t ncols, const int64_t *rp, const int32_t *col,
                       const double *val, int vtype, HostPacked &hp, double *deq,
                       const uint8_t *codes = nullptr, const float *scales = nullptr) {
    hp.row_ptr.assign(nrows + 1, 0);
    int64_t total = 0;
    for (int64_t i = 0; i < nrows; ++i) {
        const int64_t len = rp[i + 1] - rp[i];
        hp.max_len = std::max<int64_t>(hp.max_len, len);
        total += (len + kRowPad - 1) / kRowPad * kRowPad;
        if (total > 0x7FFFFFF0LL) return fail(APPGA_E_SHAPE, "too many stored entries (>= 2^31)");
        hp.row_ptr[i + 1] = static_cast<int32_t>(total);
    }
    const bool idx16 = ncols <= 65536;
    if (ncols > (1LL << 24)) return fail(APPGA_E_SHAPE, "too many columns for 32-bit lane offsets");
    if (idx16)
        hp.col16.assign(total, 0);
    else
        hp.col32.assign(total, 0);
    hp.col32u.assign(total, 0);
    const size_t vsz = vtype == VT_F32 ? 4 : (vtype == VT_FP8 ? 1 : 2);
    hp.val.assign(total * vsz, 0);
    if (vtype == VT_FP8 && scales) hp.scale.assign(scales, scales + nrows);
    for (int64_t i = 0; i < nrows; ++i) {
        const int64_t a = rp[i], b = rp[i + 1];
        const int64_t o = hp.row_ptr[i], oe = hp.row_ptr[i + 1];
        const double sc = (vtype == VT_FP8 && scales) ? static_cast<double>(scales[i]) : 1.0;
        const uint32_t padcol = b > a ? static_cast<uint32_t>(col[b - 1]) : 0u;
        for (int64_t t = 0; t < oe - o; ++t) {
            const bool real = t < b - a;
            const uint32_t c = real ? static_cast<uint32_t>(col[a + t]) : padcol;
            const double v = real ? val[a + t] : 0.0;
            if (idx16)
                hp.col16[o + t] = static_cast<uint16_t>(c);
            else
                hp.col32[o + t] = c;
            hp.col32u[o + t] = c * 256u;
            double dq = 0.0;
            uint8_t *dst = hp.val.data() + (o + t) * vsz;
            switch (vtype) {
                case VT_F32: {
                    const float f = static_cast<float>(v);
                    std::memcpy(dst, &f, 4);
                    dq = f;
                    break;
                }
                case VT_BF16: {
                    const uint16_t h = f32_to_bf16(static_cast<float>(v));
                    std::memcpy(dst, &h, 2);
                    dq = bf16_to_f32_host(h);
                    break;
                }
                case VT_F16: {
                    const uint16_t h = f32_to_f16(static_cast<float>(v));
                    std::memcpy(dst, &h, 2);
                    dq = f16_to_f32_host(h);
                    break;
                }
                case VT_FP8: {
                    const uint8_t q = real ? codes[a + t] : 0;
                    *dst = q;
                    dq = sc * e4m3_to_f64(q);
                    break;
                }
            }
            if (real && deq) deq[a + t] = dq;
        }
    }
    return APPGA_OK;
}

template <typename T>
appga_status upload(const std::vector<T> &h, void **d, int64_t &bytes) {
    *d = nullptr;
    if (h.empty()) return APPGA_OK;
    HIP_TRY(hipMalloc(d, h.size() * sizeof(T)));
    HIP_TRY(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    bytes += static_cast<int64_t>(h.size() * sizeof(T));
    return APPGA_OK;
}

appga_status to_device(const HostPacked &hp, int64_t nrows, int64_t ncols, int64_t nnz, int vtype,
                       DevCsr &dc) {
    dc.n_rows = static_cast<int32_t>(nrows);
    dc.n_cols = static_cast<int32_t>(ncols);
    dc.nnz = nnz;
    dc.nnz_padded = hp.row_ptr.back();
    dc.idx16 = ncols <= 65536;
    dc.vtype = vtype;
    dc.max_row_len = hp.max_len;
    dc.mean_row_len = nrows > 0 ? static_cast<double>(nnz) / nrows : 0.0;
    dc.bytes = 0;
    ST_TRY(upload(hp.row_ptr, reinterpret_cast<void **>(&dc.row_ptr), dc.bytes));
    if (dc.idx16)
        ST_TRY(upload(hp.col16, &dc.col, dc.bytes));
    else
        ST_TRY(upload(hp.col32, &dc.col, dc.bytes));
    ST_TRY(upload(hp.val, &dc.val, dc.bytes));
    int64_t off_bytes = 0;  // the lane-record offsets are a second index array, counted apart
    ST_TRY(upload(hp.col32u, reinterpret_cast<void **>(&dc.col32), off_bytes));
    ST_TRY(upload(hp.scale, reinterpret_cast<void **>(&dc.row_scale), dc.bytes));
    return APPGA_OK;
}

appga_status gather_tiles_to_device(const HostGatherTiles &h, DevGatherTiles &d) {
    d = DevGatherTiles();
    d.n_tiles = h.n_tiles;
    d.tiles_x = h.tiles_x;
    d.n_groups = h.n_groups;
    d.group_angles = h.group_angles;
    d.max_windows = h.max_windows;
    d.n_windows = static_cast<int64_t>(h.rec_off.size()) - 1;
    d.n_records = static_cast<int64_t>(h.records.size());
    d.n_words = static_cast<int64_t>(h.word.size());
    ST_TRY(upload(h.win_off, reinterpret_cast<void **>(&d.win_off), d.bytes));
    ST_TRY(upload(h.rec_off, reinterpret_cast<void **>(&d.rec_off), d.bytes));
    ST_TRY(upload(h.records, reinterpret_cast<void **>(&d.records), d.bytes));
    ST_TRY(upload(h.rp, reinterpret_cast<void **>(&d.rp), d.bytes));
    ST_TRY(upload(h.word, reinterpret_cast<void **>(&d.word), d.bytes));
    ST_TRY(upload(h.outs, reinterpret_cast<void **>(&d.outs), d.bytes));
    ST_TRY(upload(h.parts, reinterpret_cast<void **>(&d.parts), d.bytes));
    ST_TRY(upload(h.reds, reinterpret_cast<void **>(&d.reds), d.bytes));
    d.n_parts = static_cast<int>(h.parts.size() / 4);
    d.n_reds = static_cast<int>(h.reds.size() / 4);
    d.n_pslots = h.n_pslots;
    d.valid = 1;
    return APPGA_OK;
}

void free_gather_tiles(DevGatherTiles &d) {
    hipFree(d.win_off);
    hipFree(d.rec_off);
    hipFree(d.records);
    hipFree(d.rp);
    hipFree(d.word);
    hipFree(d.outs);
    hipFree(d.parts);
    hipFree(d.reds);
    d = DevGatherTiles();
}

void free_csr(DevCsr &dc) {
    hipFree(dc.row_ptr);
    hipFree(dc.col);
    hipFree(dc.col32);
    hipFree(dc.val);
    hipFree(dc.row_scale);
    dc = DevCsr();
}

// Launch group (lanes per row) for the B = 1 kernels: enough lanes that each
// covers about one 8-entry chunk of a mean-length row.
int plan_group(double mean_len) {
    const int chunks = static_cast<int>(std::ceil(mean_len / kChunk));
    return std::min(64, std::max(4, next_pow2(std::max(1, chunks))));
}

int env_int(const char *name, int dflt) {
    const char *s = std::getenv(name);
    return s && *s ? std::atoi(s) : dflt;
}

}  // namespace

namespace {

appga_status check_matrix(const appga_geometry *geom, int64_t nnz, const int64_t *row_ptr,
                          const int32_t *col_idx, const double *values) {
    if (!geom) return fail(APPGA_E_INVALID_ARG, "geometry is NULL");
    if (!row_ptr || (nnz > 0 && (!col_idx || !values)))
        return fail(APPGA_E_INVALID_ARG, "NULL CSR array");
    if (geom->n <= 0 || geom->n_angles <= 0 || geom->n_bins <= 0)
        return fail(APPGA_E_SHAPE, "geometry sizes must be positive");
    if (static_cast<int64_t>(geom->n) * geom->n > (1LL << 30) ||
        static_cast<int64_t>(geom->n_angles) * geom->n_bins > (1LL << 30))
        return fail(APPGA_E_SHAPE, "geometry too large");
    if (nnz < 0 || nnz >= (1LL << 31)) return fail(APPGA_E_SHAPE, "nnz out of range");
    const int64_t m = static_cast<int64_t>(geom->n_angles) * geom->n_bins;
    const int64_t d = static_cast<int64_t>(geom->n) * geom->n;
    if (row_ptr[0] != 0) return fail(APPGA_E_SHAPE, "row_ptr[0] must be 0");
    for (int64_t i = 0; i < m; ++i)
        if (row_ptr[i + 1] < row_ptr[i])
            return fail(APPGA_E_SHAPE, "row_ptr decreases at row %lld", (long long)i);
    if (row_ptr[m] != nnz) return fail(APPGA_E_SHAPE, "row_ptr[m] != nnz");
    for (int64_t k = 0; k < nnz; ++k) {
        if (col_idx[k] < 0 || col_idx[k] >= d)
            return fail(APPGA_E_SHAPE, "column index %d out of range at entry %lld", col_idx[k],
                        (long long)k);
        if (!std::isfinite(values[k]))
            return fail(APPGA_E_NONFINITE, "non-finite value at entry %lld", (long long)k);
        if (values[k] < 0.0)
            return fail(APPGA_E_DOMAIN, "negative value at entry %lld (A must be >= 0)",
                        (long long)k);
    }
    return APPGA_OK;
}

}  // namespace

extern "C" appga_status appga_validate_system_matrix(const appga_geometry *geom, int64_t nnz,
                                                     const int64_t *row_ptr,
                                                     const int32_t *col_idx,
                                                     const double *values) {
    clear_error();
    return check_matrix(geom, nnz, row_ptr, col_idx, values);
}

extern "C" appga_status appga_validate_params(const appga_params *p) {
    clear_error();
    return validate_params(p);
}

// Gaussian PSF taps (Section 4.1): FWHM in pixels, sigma = FWHM / (2 sqrt(2 ln 2)),
// offsets -R..R with R = ceil(3 sigma), normalised to sum 1.
static std::vector<double> psf_taps_host(double fwhm, int &R) {
    const double sigma = fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    R = static_cast<int>(std::ceil(3.0 * sigma));
    std::vector<double> w(2 * R + 1);
    double sum = 0.0;
    for (int t = -R; t <= R; ++t) sum += (w[t + R] = std::exp(-static_cast<double>(t) * t / (2.0 * sigma * sigma)));
    for (double &v : w) v /= sum;
    return w;
}

// One FP64 pass of H on the host along axis 0 (columns c) or 1 (rows r), zero outside.
static void psf_pass_host(int n, const std::vector<double> &w, int axis, const std::vector<double> &in,
                          std::vector<double> &out) {
    const int R = (static_cast<int>(w.size()) - 1) / 2;
    out.assign(static_cast<size_t>(n) * n, 0.0);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            double acc = 0.0;
            for (int k = 0; k <= 2 * R; ++k) {
                const int q = (axis == 0 ? c : r) + k - R;
                if (q < 0 || q >= n) continue;
                acc += w[k] * in[axis == 0 ? static_cast<size_t>(r) * n + q : static_cast<size_t>(q) * n + c];
            }
            out[static_cast<size_t>(r) * n + c] = acc;
        }
}

static appga_status load_impl(appga_ctx *ctx, const appga_geometry *geom, int64_t nnz, const int64_t *row_ptr,
                              const int32_t *col_idx, const double *values_in, appga_dtype storage,
                              const double *row_factors, double psf_fwhm, appga_matrix **out) {
    if (!ctx || !geom || !out) return fail(APPGA_E_INVALID_ARG, "NULL ctx, geometry or output");
    if (storage != APPGA_F32 && storage != APPGA_BF16 && storage != APPGA_F16 &&
        storage != APPGA_FP8_E4M3_ROWSCALE)
        return fail(APPGA_E_INVALID_ARG, "unknown storage type %d", static_cast<int>(storage));
    ST_TRY(check_matrix(geom, nnz, row_ptr, col_idx, values_in));
    const int64_t m = static_cast<int64_t>(geom->n_angles) * geom->n_bins;
    const int64_t d = static_cast<int64_t>(geom->n) * geom->n;
    if (!std::isfinite(psf_fwhm) || psf_fwhm < 0.0) return fail(APPGA_E_DOMAIN, "psf_fwhm_px must be >= 0");
    int psf_R = -1;
    std::vector<double> taps;
    if (psf_fwhm > 0.0) {
        if (psf_fwhm > 24.0) return fail(APPGA_E_DOMAIN, "psf_fwhm_px must be <= 24 pixels");
        taps = psf_taps_host(psf_fwhm, psf_R);
        if (2 * psf_R + 1 > kPsfMaxTaps) return fail(APPGA_E_DOMAIN, "PSF too wide");
    }
    // A = diag(row factors) G: the factors are folded into the stored values
    std::vector<double> scaled;
    const double *values = values_in;
    if (row_factors) {
        for (int64_t i = 0; i < m; ++i)
            if (!std::isfinite(row_factors[i]) || row_factors[i] < 0.0)
                return fail(APPGA_E_DOMAIN, "row factor %lld is negative or not finite", (long long)i);
        scaled.resize(nnz);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) scaled[k] = values_in[k] * row_factors[i];
        values = scaled.data();
    }
    HIP_TRY(hipSetDevice(ctx->device));
    const int vtype = static_cast<int>(storage);

    static std::atomic<uint64_t> next_serial{1};
    auto *mat = new appga_matrix();
    mat->ctx = ctx;
    mat->serial = next_serial.fetch_add(1);
    mat->geom = *geom;
    mat->nnz = nnz;
    mat->storage = vtype;
    mat->deq.assign(nnz, 0.0);
    mat->user_row_ptr.assign(row_ptr, row_ptr + m + 1);
    mat->user_col.assign(col_idx, col_idx + nnz);
    mat->has_row_factors = row_factors != nullptr;
    mat->psf_fwhm = psf_fwhm;
    mat->psf_R = psf_R;

    // stored transpose: rows = pixels, entries ordered by detector row
    std::vector<int64_t> trp(d + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) trp[col_idx[k] + 1] += 1;
    for (int64_t j = 0; j < d; ++j) trp[j + 1] += trp[j];
    std::vector<uint8_t> codes, tcodes;
    std::vector<float> scales;
    if (vtype == VT_FP8) {
        fp8_quantize(m, row_ptr, values, codes, scales);
        tcodes.resize(nnz);
    }
    std::vector<int32_t> tcol(nnz);
    std::vector<double> tval(nnz);
    {
        std::vector<int64_t> pos(trp.begin(), trp.end() - 1);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                const int64_t p = pos[col_idx[k]]++;
                tcol[p] = static_cast<int32_t>(i);
                tval[p] = values[k];
                if (vtype == VT_FP8) tcodes[p] = codes[k];
            }
    }
    appga_status st = APPGA_OK;
    {
        HostPacked ha, ht;
        st = pack_rows(m, d, row_ptr, col_idx, values, vtype, ha, mat->deq.data(), codes.data(),
                       scales.data());
        if (st == APPGA_OK)
            st = pack_rows(d, m, trp.data(), tcol.data(), tval.data(), vtype, ht, nullptr,
                           tcodes.data(), nullptr);
        if (st == APPGA_OK) st = to_device(ha, m, d, nnz, vtype, mat->A);
        if (st == APPGA_OK) st = to_device(ht, d, m, nnz, vtype, mat->AT);
    }
    // quarter-turn symmetry (B = 1, opt-in with APPGA_SYMMETRY=1): row (a + A/2, b) is
    // row (a, b) with pixel j moved to rho(j), rho(r, c) = (c, N - 1 - r), when the
    // angles are even in number and every such pair agrees to 1e-9 of the row's largest
    // entry; then the B = 1 kernels read only the first half of the rows and of the
    // transpose.  It halves their matrix bytes and memory; it does not make them faster
    // (they are bound by the rate of per-entry gathers of x, not by matrix bytes), hence
    // off by default
    if (st == APPGA_OK && env_int("APPGA_SYMMETRY", 0) && geom->n_angles % 2 == 0 && vtype != VT_FP8 &&
        mat->A.idx16 && mat->AT.idx16) {
        const int64_t half = m / 2;
        const int N = geom->n;
        bool ok = true;
        std::vector<std::pair<int32_t, double>> ra, rb;
        for (int64_t i = 0; i < half && ok; ++i) {
            ra.clear();
            rb.clear();
            double big = 0.0;
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                const int32_t r = col_idx[k] / N, c = col_idx[k] % N;
                ra.emplace_back(c * N + (N - 1 - r), values[k]);
                big = std::max(big, std::fabs(values[k]));
            }
            for (int64_t k = row_ptr[i + half]; k < row_ptr[i + half + 1]; ++k) {
                rb.emplace_back(col_idx[k], values[k]);
                big = std::max(big, std::fabs(values[k]));
            }
            std::sort(ra.begin(), ra.end());
            std::sort(rb.begin(), rb.end());
            const double tol = 1e-9 * std::max(big, 1e-300);
            size_t p = 0, q = 0;
            while (ok && (p < ra.size() || q < rb.size())) {
                if (q == rb.size() || (p < ra.size() && ra[p].first < rb[q].first)) {
                    ok = std::fabs(ra[p++].second) <= tol;
                } else if (p == ra.size() || rb[q].first < ra[p].first) {
                    ok = std::fabs(rb[q++].second) <= tol;
                } else {
                    ok = std::fabs(ra[p++].second - rb[q++].second) <= tol;
                }
            }
        }
        if (ok && half > 0) {
            // the transpose of the first half: rows = pixels, entries = base rays in order
            std::vector<int64_t> hrp(d + 1, 0);
            for (int64_t k = 0; k < row_ptr[half]; ++k) hrp[col_idx[k] + 1] += 1;
            for (int64_t j = 0; j < d; ++j) hrp[j + 1] += hrp[j];
            const int64_t hnnz = row_ptr[half];
            std::vector<int32_t> hcol(hnnz);
            std::vector<double> hval(hnnz);
            std::vector<int64_t> pos(hrp.begin(), hrp.end() - 1);
            for (int64_t i = 0; i < half; ++i)
                for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                    const int64_t p2 = pos[col_idx[k]]++;
                    hcol[p2] = static_cast<int32_t>(i);
                    hval[p2] = values[k];
                }
            HostPacked hh, hth;
            st = pack_rows(half, d, row_ptr, col_idx, values, vtype, hh, nullptr);
            if (st == APPGA_OK) st = pack_rows(d, half, hrp.data(), hcol.data(), hval.data(), vtype, hth, nullptr);
            if (st == APPGA_OK) st = to_device(hh, half, d, hnnz, vtype, mat->A_half);
            if (st == APPGA_OK) st = to_device(hth, d, half, hnnz, vtype, mat->AT_half);
            if (st == APPGA_OK) mat->sym = (mat->A_half.idx16 && mat->AT_half.idx16) ? 1 : 0;
        }
    }
    // tile forms for batches (B > 1); without them the row kernels serve
    if (st == APPGA_OK && env_int("APPGA_BACK_TILES", 1)) {
        // value of each transpose entry as the stored transpose decodes it
        std::vector<float> tv32(nnz);
        for (int64_t k = 0; k < nnz; ++k) {
            const float v = static_cast<float>(tval[k]);
            switch (vtype) {
                case VT_F32: tv32[k] = v; break;
                case VT_BF16: tv32[k] = bf16_to_f32_host(f32_to_bf16(v)); break;
                case VT_F16: tv32[k] = f16_to_f32_host(f32_to_f16(v)); break;
                default: tv32[k] = static_cast<float>(e4m3_to_f64(tcodes[k])); break;
            }
        }
        HostGatherTiles hb;
        if (build_back_tiles(geom->n, geom->n_angles, geom->n_bins, trp.data(), tcol.data(), tv32.data(), hb))
            st = gather_tiles_to_device(hb, mat->bt);
    }
    if (st == APPGA_OK && env_int("APPGA_FWD_TILES", 1)) {
        // value of each entry of A as the stored matrix decodes it (FP8: the
        // code without its row scale)
        std::vector<float> v32(nnz);
        for (int64_t k = 0; k < nnz; ++k)
            v32[k] = vtype == VT_FP8 ? static_cast<float>(e4m3_to_f64(codes[k])) : static_cast<float>(mat->deq[k]);
        HostGatherTiles hf;
        if (build_fwd_tiles(geom->n, geom->n_angles, geom->n_bins, row_ptr, col_idx, v32.data(), hf,
                            env_int("APPGA_FWD_PART_WINDOWS", 0)))
            st = gather_tiles_to_device(hf, mat->ft);
    }
    if (st == APPGA_OK && psf_R >= 0) {
        std::vector<float> tf(taps.begin(), taps.end());
        int64_t dummy = 0;
        st = upload(tf, reinterpret_cast<void **>(&mat->psf_taps), dummy);
    }
    if (st == APPGA_OK) {
        // Lambda = A^T 1 of the stored (dequantised) values, zeros -> 1 (eq. EM);
        // with a PSF, A^T 1 = H (G^T n) (H is symmetric)
        std::vector<double> lam(d, 0.0);
        for (int64_t k = 0; k < nnz; ++k) lam[col_idx[k]] += mat->deq[k];
        if (psf_R >= 0) {
            std::vector<double> t1;
            psf_pass_host(geom->n, taps, 0, lam, t1);
            psf_pass_host(geom->n, taps, 1, t1, lam);
        }
        std::vector<float> lamf(d);
        for (int64_t j = 0; j < d; ++j) lamf[j] = lam[j] > 0.0 ? static_cast<float>(lam[j]) : 1.0f;
        int64_t dummy = 0;
        st = upload(lamf, reinterpret_cast<void **>(&mat->lam), dummy);
    }
    if (st != APPGA_OK) {
        free_csr(mat->A);
        free_csr(mat->AT);
        free_csr(mat->A_half);
        free_csr(mat->AT_half);
        free_gather_tiles(mat->bt);
        free_gather_tiles(mat->ft);
        hipFree(mat->lam);
        hipFree(mat->psf_taps);
        delete mat;
        return st;
    }
    mat->group_fwd = env_int("APPGA_GROUP_FWD", plan_group(mat->A.mean_row_len));
    mat->group_back = env_int("APPGA_GROUP_BACK", plan_group(mat->AT.mean_row_len));
    mat->fwd_wgs = env_int("APPGA_FWD_WGS", 2048);
    // the remap needs the tile grid (tx x tx) to split into 2 x 4 equal blocks
    const int tx = (geom->n + 3) / 4;
    const bool remap_ok = tx % 4 == 0;
    mat->remap_ok = remap_ok ? 1 : 0;
    mat->xcd_remap = (remap_ok && env_int("APPGA_XCD_REMAP", 1)) ? 1 : 0;
    mat->bt_remap = (mat->bt.valid && mat->bt.tiles_x % 4 == 0 && env_int("APPGA_XCD_REMAP", 1)) ? 1 : 0;
    mat->bt_split = mat->bt.valid ? std::max(1, std::min(mat->bt.n_groups,
                                                         env_int("APPGA_BACK_SPLIT", back_tiles_split(mat->bt))))
                                  : 1;
    if (env_int("APPGA_AUTOTUNE", 1)) {
        const appga_status ts = tune_matrix(ctx, mat, APPGA_TUNE_SINGLE | APPGA_TUNE_BATCH, nullptr);
        if (ts != APPGA_OK) {
            free_csr(mat->A);
            free_csr(mat->AT);
            free_csr(mat->A_half);
            free_csr(mat->AT_half);
            free_gather_tiles(mat->bt);
            free_gather_tiles(mat->ft);
            hipFree(mat->lam);
            hipFree(mat->psf_taps);
            delete mat;
            return ts;
        }
    }
    *out = mat;
    return APPGA_OK;
}

extern "C" appga_status appga_free_system_matrix(appga_ctx *ctx, appga_matrix *mat) {
    clear_error();
    if (!ctx || !mat) return fail(APPGA_E_INVALID_ARG, "NULL ctx or matrix");
    if (mat->inflight.load() > 0)
        return fail(APPGA_E_BUSY, "matrix is used by %d in-flight requests", mat->inflight.load());
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    free_csr(mat->A);
    free_csr(mat->AT);
    free_csr(mat->A_half);
    free_csr(mat->AT_half);
    free_gather_tiles(mat->bt);
    free_gather_tiles(mat->ft);
    hipFree(mat->lam);
    hipFree(mat->psf_taps);
    delete mat;
    return APPGA_OK;
}

extern "C" appga_status appga_load_system_matrix(appga_ctx *ctx, const appga_geometry *geom, int64_t nnz,
                                                 const int64_t *row_ptr, const int32_t *col_idx,
                                                 const double *values, appga_dtype storage, appga_matrix **out) {
    clear_error();
    return load_impl(ctx, geom, nnz, row_ptr, col_idx, values, storage, nullptr, 0.0, out);
}

extern "C" appga_status appga_load_system_matrix_factored(appga_ctx *ctx, const appga_geometry *geom,
                                                          int64_t nnz, const int64_t *row_ptr,
                                                          const int32_t *col_idx, const double *values,
                                                          appga_dtype storage, const double *row_factors,
                                                          double psf_fwhm_px, appga_matrix **out) {
    clear_error();
    return load_impl(ctx, geom, nnz, row_ptr, col_idx, values, storage, row_factors, psf_fwhm_px, out);
}

extern "C" appga_status appga_matrix_symmetry(const appga_matrix *mat, int32_t *folds, int64_t *stored_bytes) {
    clear_error();
    if (!mat || !folds) return fail(APPGA_E_INVALID_ARG, "NULL argument");
    *folds = mat->sym ? 2 : 1;
    if (stored_bytes) *stored_bytes = mat->sym ? mat->A_half.bytes + mat->AT_half.bytes : mat->A.bytes + mat->AT.bytes;
    return APPGA_OK;
}

extern "C" appga_status appga_matrix_psf(const appga_matrix *mat, double *fwhm_px, int32_t *radius) {
    clear_error();
    if (!mat || !fwhm_px || !radius) return fail(APPGA_E_INVALID_ARG, "NULL argument");
    *fwhm_px = mat->psf_R >= 0 ? mat->psf_fwhm : 0.0;
    *radius = mat->psf_R;
    return APPGA_OK;
}

extern "C" appga_status appga_matrix_info(const appga_matrix *mat, int64_t *nnz, int64_t *bytes_a,
                                          int64_t *bytes_at, int32_t *storage) {
    clear_error();
    if (!mat) return fail(APPGA_E_INVALID_ARG, "matrix is NULL");
    if (nnz) *nnz = mat->nnz;
    if (bytes_a) *bytes_a = mat->A.bytes;
    if (bytes_at) *bytes_at = mat->AT.bytes;
    if (storage) *storage = mat->storage;
    return APPGA_OK;
}

extern "C" appga_status appga_matrix_tiles(const appga_matrix *mat, int32_t which, appga_tile_info *out) {
    clear_error();
    if (!mat || !out) return fail(APPGA_E_INVALID_ARG, "NULL matrix or output");
    if (which != APPGA_TILES_FORWARD && which != APPGA_TILES_BACK)
        return fail(APPGA_E_INVALID_ARG, "which must be APPGA_TILES_FORWARD or APPGA_TILES_BACK");
    const DevGatherTiles &t = which == APPGA_TILES_FORWARD ? mat->ft : mat->bt;
    *out = appga_tile_info{};
    out->valid = t.valid;
    out->tiles = t.n_tiles;
    out->split = which == APPGA_TILES_BACK ? mat->bt_split : 1;
    out->windows = t.n_windows;
    out->records = t.n_records;
    out->entries = t.n_words / 2;
    out->bytes = t.bytes;
    return APPGA_OK;
}

extern "C" appga_status appga_tiles_emulate(const appga_geometry *geom, int64_t nnz, const int64_t *row_ptr,
                                           const int32_t *col_idx, const double *values, appga_dtype storage,
                                           int32_t which, int32_t split, const float *in, float *out,
                                           appga_tile_info *info) {
    clear_error();
    if (!geom || !in || !out) return fail(APPGA_E_INVALID_ARG, "NULL geometry, input or output");
    if (storage != APPGA_F32 && storage != APPGA_BF16 && storage != APPGA_F16)
        return fail(APPGA_E_INVALID_ARG, "emulation supports F32, BF16 and F16 storage");
    if (which != APPGA_TILES_FORWARD && which != APPGA_TILES_BACK)
        return fail(APPGA_E_INVALID_ARG, "which must be APPGA_TILES_FORWARD or APPGA_TILES_BACK");
    ST_TRY(check_matrix(geom, nnz, row_ptr, col_idx, values));
    const int n = geom->n;
    const int64_t m = static_cast<int64_t>(geom->n_angles) * geom->n_bins, d = static_cast<int64_t>(n) * n;
    std::vector<float> v32(nnz);
    for (int64_t k = 0; k < nnz; ++k) {
        const float v = static_cast<float>(values[k]);
        v32[k] = storage == APPGA_F32 ? v
                 : storage == APPGA_BF16 ? bf16_to_f32_host(f32_to_bf16(v))
                                         : f16_to_f32_host(f32_to_f16(v));
    }
    HostGatherTiles t;
    bool ok = false;
    if (which == APPGA_TILES_FORWARD) {
        ok = build_fwd_tiles(n, geom->n_angles, geom->n_bins, row_ptr, col_idx, v32.data(), t, split);
    } else {
        std::vector<int64_t> trp(d + 1, 0);
        for (int64_t k = 0; k < nnz; ++k) trp[col_idx[k] + 1] += 1;
        for (int64_t j = 0; j < d; ++j) trp[j + 1] += trp[j];
        std::vector<int32_t> tcol(nnz);
        std::vector<float> tv(nnz);
        std::vector<int64_t> pos(trp.begin(), trp.end() - 1);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                const int64_t q = pos[col_idx[k]]++;
                tcol[q] = static_cast<int32_t>(i);
                tv[q] = v32[k];
            }
        ok = build_back_tiles(n, geom->n_angles, geom->n_bins, trp.data(), tcol.data(), tv.data(), t);
        if (ok && (split < 1 || split > std::max(1, t.n_groups)))
            return fail(APPGA_E_INVALID_ARG, "split must be in [1, %d]", std::max(1, t.n_groups));
    }
    if (info) {
        *info = appga_tile_info{};
        info->valid = ok ? 1 : 0;
    }
    if (!ok) return APPGA_OK;
    const int64_t n_in = which == APPGA_TILES_FORWARD ? d : m, n_out = which == APPGA_TILES_FORWARD ? m : d;
    std::fill(out, out + n_out, 0.0f);
    // the sums of windows [w0, w1) of tile tt, as a workgroup forms them
    std::vector<float> acc(64);
    auto sum_windows = [&](int64_t w0, int64_t w1) -> bool {
        std::fill(acc.begin(), acc.end(), 0.0f);
        for (int64_t w = w0; w < w1; ++w) {
            const uint32_t r0 = t.rec_off[w], S = t.rec_off[w + 1] - r0;
            if (S > static_cast<uint32_t>(kBackSlots)) return false;
            for (int o = 0; o < 64; ++o)
                for (uint32_t k = t.rp[w * 64 + o]; k < t.rp[w * 64 + o + 1]; k += 2) {
                    const uint32_t slot = t.word[k] / 256;
                    if (t.word[k] % 256 || (slot >= S && slot != static_cast<uint32_t>(kBackSlots))) return false;
                    float v;
                    std::memcpy(&v, &t.word[k + 1], 4);
                    const float x = slot == static_cast<uint32_t>(kBackSlots) ? 0.0f : in[t.records[r0 + slot]];
                    acc[o] = std::fmaf(v, x, acc[o]);
                }
        }
        return true;
    };
    for (uint32_t r : t.records)
        if (r >= static_cast<uint64_t>(n_in)) return fail(APPGA_E_SHAPE, "tile form names input %u", r);
    if (which == APPGA_TILES_FORWARD) {
        std::vector<float> part(static_cast<size_t>(t.n_pslots) * 64);
        for (size_t p = 0; p < t.parts.size() / 4; ++p) {
            const uint32_t tt = t.parts[4 * p], slot = t.parts[4 * p + 3];
            if (!sum_windows(t.parts[4 * p + 1], t.parts[4 * p + 2])) return fail(APPGA_E_SHAPE, "bad tile form");
            for (int o = 0; o < 64; ++o) {
                if (slot != kNoSlot) part[slot * 64 + o] = acc[o];
                else if (t.outs[tt * 64 + o] >= 0) out[t.outs[tt * 64 + o]] = acc[o];
            }
        }
        for (size_t r = 0; r < t.reds.size() / 4; ++r) {
            const uint32_t tt = t.reds[4 * r], s0 = t.reds[4 * r + 1], np = t.reds[4 * r + 2];
            for (int o = 0; o < 64; ++o) {
                float sum = part[s0 * 64 + o];
                for (uint32_t q = 1; q < np; ++q) sum += part[(s0 + q) * 64 + o];
                if (t.outs[tt * 64 + o] >= 0) out[t.outs[tt * 64 + o]] = sum;
            }
        }
    } else {
        std::vector<float> tot(64);
        for (int tt = 0; tt < t.n_tiles; ++tt) {
            const int64_t wt0 = t.win_off[tt], nwt = t.win_off[tt + 1] - wt0;
            std::fill(tot.begin(), tot.end(), 0.0f);
            for (int q = 0; q < split; ++q) {   // the step kernel adds the partial sums in order
                if (!sum_windows(wt0 + q * nwt / split, wt0 + (q + 1) * nwt / split))
                    return fail(APPGA_E_SHAPE, "bad tile form");
                for (int o = 0; o < 64; ++o) tot[o] += acc[o];
            }
            for (int o = 0; o < 64; ++o)
                if (t.outs[tt * 64 + o] >= 0) out[t.outs[tt * 64 + o]] = tot[o];
        }
    }
    if (info) {
        info->tiles = t.n_tiles;
        info->split = which == APPGA_TILES_BACK ? split : 1;
        info->windows = static_cast<int64_t>(t.rec_off.size()) - 1;
        info->records = static_cast<int64_t>(t.records.size());
        info->entries = static_cast<int64_t>(t.word.size() / 2);
        info->bytes = 4 * static_cast<int64_t>(t.win_off.size() + t.rec_off.size() + t.records.size() +
                                               t.rp.size() + t.word.size() + t.outs.size() + t.parts.size() +
                                               t.reds.size());
    }
    return APPGA_OK;
}

extern "C" appga_status appga_matrix_dequantized(const appga_matrix *mat, double *values_out) {
    clear_error();
    if (!mat || (!values_out && mat->nnz > 0)) return fail(APPGA_E_INVALID_ARG, "NULL argument");
    std::memcpy(values_out, mat->deq.data(), sizeof(double) * mat->nnz);
    return APPGA_OK;
}

// ------------------------------------------------------------ validation ---

namespace appga {

appga_status validate_params(const appga_params *p, bool afppa) {
    if (!p) return fail(APPGA_E_INVALID_ARG, "params is NULL");
    const double vals[] = {p->lambda1, p->lambda2, p->eps, p->omega, p->a, p->b, p->beta,
                           p->fixed_p, p->gamma_scalar};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(APPGA_E_DOMAIN, "non-finite parameter");
    if (p->lambda1 < 0 || p->lambda2 < 0) return fail(APPGA_E_DOMAIN, "lambda must be >= 0");
    if (!afppa && !(p->eps > 0)) return fail(APPGA_E_DOMAIN, "eps must be > 0");
    if (!(p->omega > 0) || p->omega > 1) return fail(APPGA_E_DOMAIN, "omega must be in (0, 1]");
    if (!(p->a > 0)) return fail(APPGA_E_DOMAIN, "a must be > 0");
    if (p->omega == 1.0 && p->a >= 0.5) return fail(APPGA_E_DOMAIN, "omega = 1 needs a < 1/2");
    if (p->b < 0) {  // t_k = a k^omega + b must not vanish
        const double k = std::pow(-p->b / p->a, 1.0 / p->omega);
        if (k >= 0.5 && std::fabs(k - std::nearbyint(k)) < 1e-9)
            return fail(APPGA_E_DOMAIN, "b = -a k^omega for k = %.0f", k);
    }
    if (!(p->beta > 0)) return fail(APPGA_E_DOMAIN, "beta must be > 0");
    if (p->iterations < 0) return fail(APPGA_E_DOMAIN, "iterations must be >= 0");
    if (p->momentum != APPGA_MOMENTUM_GN && p->momentum != APPGA_MOMENTUM_NONE &&
        !(afppa && p->momentum == APPGA_MOMENTUM_NESTEROV))
        return fail(APPGA_E_INVALID_ARG, "unknown momentum %d", p->momentum);
    if (p->precond != APPGA_PRECOND_EM && p->precond != APPGA_PRECOND_EM_FROZEN &&
        p->precond != APPGA_PRECOND_FIXED)
        return fail(APPGA_E_INVALID_ARG, "unknown preconditioner %d", p->precond);
    if (afppa && p->precond == APPGA_PRECOND_EM_FROZEN)
        return fail(APPGA_E_INVALID_ARG, "AFPPA takes the EM or the fixed preconditioner");
    if (p->precond == APPGA_PRECOND_FIXED && !(p->fixed_p > 0))
        return fail(APPGA_E_DOMAIN, "fixed_p must be > 0");
    if (p->gamma_scalar < 0) return fail(APPGA_E_DOMAIN, "gamma_scalar must be >= 0");
    if (p->monitor_every < 0) return fail(APPGA_E_DOMAIN, "monitor_every must be >= 0");
    return APPGA_OK;
}

appga_status validate_data(const float *v, int64_t n, const char *what) {
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(v[i])) return fail(APPGA_E_NONFINITE, "non-finite %s[%lld]", what, (long long)i);
        if (v[i] < 0) return fail(APPGA_E_DOMAIN, "negative %s[%lld]", what, (long long)i);
    }
    return APPGA_OK;
}

double theta_of(const appga_params &p, int k) {
    if (p.momentum == APPGA_MOMENTUM_NONE || k < 1) return 0.0;
    if (p.momentum == APPGA_MOMENTUM_NESTEROV) {
        // t_0 = 1, t_k = (1 + sqrt(1 + 4 t_{k-1}^2)) / 2; theta_k = (t_{k-1} - 1) / t_k
        double tp = 1.0, t = 1.0;
        for (int i = 1; i <= k; ++i) {
            tp = t;
            t = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
        }
        return (tp - 1.0) / t;
    }
    const double tkm1 = p.a * std::pow(static_cast<double>(k - 1), p.omega) + p.b;
    const double tk = p.a * std::pow(static_cast<double>(k), p.omega) + p.b;
    return (tkm1 - 1.0) / tk;
}

}  // namespace appga

// --------------------------------------------------------------- sessions ---

namespace appga {

hipError_t psf_blur(const appga_matrix *mat, const float *in, int n_parts, float *tmp, float *out, int B, int Bp,
                    hipStream_t st) {
    return launch_psf_blur(in, n_parts, tmp, out, mat->geom.n, B, Bp, mat->psf_taps, mat->psf_R, st);
}

static appga_status sess_alloc(appga_solve *s) {
    const int B = s->B;
    const int64_t m = s->mat->A.n_rows, d = s->mat->A.n_cols;
    const int sb = step_blocks(s->mat->geom.n, B);
    const int nb = std::max({fidelity_blocks(static_cast<int>(m)), reg_value_blocks(s->mat->geom.n),
                             sum_blocks(static_cast<int>(m)), sb});
    const int Bp = pad_lanes(B);
    s->Bp = Bp;
    s->part_len = static_cast<size_t>(std::max(nb, afppa_blocks(s->mat->geom.n, Bp))) * Bp * 2;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_g = take(sizeof(float) * m * Bp);
    const size_t o_gam = s->has_gamma ? take(sizeof(float) * m * Bp) : 0;
    const size_t o_gl = take(sizeof(float) * Bp);
    const size_t o_f = take(sizeof(float) * d * Bp);
    const size_t o_ft0 = take(sizeof(float) * d * Bp);
    const size_t o_ft1 = take(sizeof(float) * d * Bp);
    const size_t o_e = take(sizeof(float) * m * Bp);
    const size_t o_pb = s->need_pbuf ? take(sizeof(float) * d * Bp) : 0;
    const bool tiles = B > 1 && s->mat->bt.valid;
    // AFPPA takes A^T e as its own pass in every layout (split partial sums with tiles)
    s->gf_split = tiles ? s->mat->bt_split : 1;
    const bool psf = s->mat->psf_R >= 0;
    const bool need_gf = tiles || s->afppa || psf;
    const size_t o_xb = psf ? take(sizeof(float) * d * Bp) : 0;
    const size_t o_tb = psf ? take(sizeof(float) * d * Bp) : 0;
    const size_t o_gfb = psf ? take(sizeof(float) * d * Bp) : 0;
    const size_t o_gf = need_gf ? take(sizeof(float) * d * Bp * s->gf_split) : 0;
    const size_t o_w = s->afppa ? take(sizeof(float) * d * Bp) : 0;
    const size_t o_y = s->afppa ? take(sizeof(float) * 6 * d * Bp) : 0;
    const size_t o_yb = s->afppa ? take(sizeof(float) * 6 * d * Bp) : 0;
    const size_t o_pm = s->afppa ? take(sizeof(unsigned) * 3 * kAfppaPmSlots * Bp) : 0;
    const size_t n_tp = B > 1 && s->mat->ft.valid ? fwd_tile_part_floats(s->mat->ft, Bp) : 0;
    const size_t o_tp = n_tp ? take(sizeof(float) * n_tp) : 0;
    const size_t o_lp = take(sizeof(LaneParams) * Bp);
    s->theta_cap = 1024;
    const size_t o_th = take(sizeof(float) * (s->theta_cap + 2) * Bp);
    const size_t o_part = take(sizeof(double) * s->part_len);
    const size_t o_red = take(sizeof(double) * 4 * Bp);
    const bool mon = s->monitor_every > 0;
    const size_t o_mpart = mon ? take(sizeof(double) * s->part_len) : 0;
    const size_t o_mred = mon ? take(sizeof(double) * 4 * Bp) : 0;
    const size_t o_cl = take(sizeof(unsigned long long) * Bp);
    const size_t o_tmc = take(sizeof(double) * Bp);
    HIP_TRY(hipMalloc(&s->arena, off));
    char *base = static_cast<char *>(s->arena);
    s->g = reinterpret_cast<float *>(base + o_g);
    s->gamma = s->has_gamma ? reinterpret_cast<float *>(base + o_gam) : nullptr;
    s->gamma_lane = reinterpret_cast<float *>(base + o_gl);
    s->f = reinterpret_cast<float *>(base + o_f);
    s->ft[0] = reinterpret_cast<float *>(base + o_ft0);
    s->ft[1] = reinterpret_cast<float *>(base + o_ft1);
    s->e = reinterpret_cast<float *>(base + o_e);
    s->pbuf = s->need_pbuf ? reinterpret_cast<float *>(base + o_pb) : nullptr;
    s->gf = need_gf ? reinterpret_cast<float *>(base + o_gf) : nullptr;
    if (psf) {
        s->xb = reinterpret_cast<float *>(base + o_xb);
        s->tb = reinterpret_cast<float *>(base + o_tb);
        s->gfb = reinterpret_cast<float *>(base + o_gfb);
    }
    if (s->afppa) {
        s->w = reinterpret_cast<float *>(base + o_w);
        s->ydual = reinterpret_cast<float *>(base + o_y);
        s->ybar = reinterpret_cast<float *>(base + o_yb);
        s->pm = reinterpret_cast<unsigned *>(base + o_pm);
    }
    s->tile_part = n_tp ? reinterpret_cast<float *>(base + o_tp) : nullptr;
    s->lp = reinterpret_cast<LaneParams *>(base + o_lp);
    s->theta = reinterpret_cast<float *>(base + o_th);
    s->part = reinterpret_cast<double *>(base + o_part);
    s->red = reinterpret_cast<double *>(base + o_red);
    s->mpart = mon ? reinterpret_cast<double *>(base + o_mpart) : nullptr;
    s->mred = mon ? reinterpret_cast<double *>(base + o_mred) : nullptr;
    s->clamps = reinterpret_cast<unsigned long long *>(base + o_cl);
    s->tmc = reinterpret_cast<double *>(base + o_tmc);
    return APPGA_OK;
}

// Uploads theta_k for k in [k0, k0 + theta_cap] (lane-major within k).
static appga_status sess_theta(appga_solve *s, int k0) {
    const int B = s->B, Bp = s->Bp;
    std::vector<float> th(static_cast<size_t>(s->theta_cap + 2) * Bp, 0.0f);
    for (int kk = 0; kk < s->theta_cap + 2; ++kk)
        for (int b = 0; b < B; ++b)
            th[static_cast<size_t>(kk) * Bp + b] = static_cast<float>(theta_of(s->prm[b], k0 + kk));
    HIP_TRY(hipMemcpyAsync(s->theta, th.data(), th.size() * sizeof(float), hipMemcpyHostToDevice,
                           s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    s->theta_base = k0;
    return APPGA_OK;
}

// FP64 objective Phi(x) per solve (Section 2.1) into host vector out.
hipError_t launch_forward_single(const appga_matrix *mat, const FwdArgs &fa, int group, hipStream_t st) {
    if (fa.B == 1 && mat->sym) {
        FwdArgs h = fa;
        h.row_ptr = mat->A_half.row_ptr;
        h.col = mat->A_half.col;
        h.col32 = mat->A_half.col32;
        h.nnz_padded = mat->A_half.nnz_padded;
        h.val = mat->A_half.val;
        h.sym_half = mat->A.n_rows / 2;
        h.img_n = mat->geom.n;
        return launch_forward(mat->A_half, h, group, st);
    }
    return launch_forward(mat->A, fa, group, st);
}

hipError_t launch_forward_mat(const appga_matrix *mat, const FwdArgs &fa, hipStream_t st) {
    if (forward_uses_tiles(mat, fa)) return launch_fwd_tiles(mat->ft, mat->A.vtype, fa, st);
    return launch_forward_single(mat, fa, mat->group_fwd, st);
}

hipError_t launch_step_mat(const appga_matrix *mat, const StepArgs &sa, int group, hipStream_t st) {
    if (sa.B == 1 && mat->sym) {
        StepArgs h = sa;
        h.row_ptr = mat->AT_half.row_ptr;
        h.col = mat->AT_half.col;
        h.col32 = mat->AT_half.col32;
        h.nnz_padded = mat->AT_half.nnz_padded;
        h.val = mat->AT_half.val;
        h.sym_half = mat->A.n_rows / 2;
        return launch_step(mat->AT_half, h, group, st);
    }
    return launch_step(mat->AT, sa, group, st);
}

appga_status sess_objective(appga_solve *s, const float *x, std::vector<double> &out,
                            double *part = nullptr, double *red = nullptr) {
    if (!part) part = s->part;
    if (!red) red = s->red;
    const appga_matrix *mat = s->mat;
    const int B = s->B;
    const int m = mat->A.n_rows, n = mat->geom.n;
    FwdArgs fa{};
    fa.row_ptr = mat->A.row_ptr;
    fa.col = mat->A.col;
    fa.val = mat->A.val;
    fa.row_scale = mat->A.row_scale;
    fa.col32 = mat->A.col32;
    fa.nnz_padded = mat->A.nnz_padded;
    fa.m = m;
    fa.n_x = mat->A.n_cols;
    fa.B = B;
    fa.Bp = s->Bp;
    fa.x = x;
    if (mat->psf_R >= 0) {   // A x = G (H x)
        HIP_TRY(psf_blur(mat, x, 1, s->tb, s->xb, B, s->Bp, s->st));
        fa.x = s->xb;
    }
    fa.g = s->g;
    fa.gamma = s->gamma;
    fa.gamma_lane = s->gamma_lane;
    fa.out = s->e;
    fa.mode = FM_PROJ;
    fa.tile_part = s->tile_part;
    HIP_TRY(timed_launch(s->ctx, forward_uses_tiles(mat, fa) ? "forward_proj_tiles" : "forward_proj", s->st,
                         [&] { return launch_forward_mat(mat, fa, s->st); }));
    HIP_TRY(launch_fidelity_terms(m, B, s->e, s->g, s->gamma, s->gamma_lane, part, s->st));
    HIP_TRY(launch_reduce_partials(part, fidelity_blocks(m), B, 1, red, s->st));
    HIP_TRY(launch_reg_value(n, B, x, s->lp, part, s->st));
    HIP_TRY(launch_reduce_partials(part, reg_value_blocks(n), B, 1, red + B, s->st));
    std::vector<double> h(2 * B);
    HIP_TRY(hipMemcpyAsync(h.data(), red, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    out.resize(B);
    for (int b = 0; b < B; ++b) out[b] = h[b] + h[B + b];
    return APPGA_OK;
}

appga_status sess_begin(appga_ctx *ctx, const appga_matrix *mat, int B, const float *d_g,
                        const float *d_gamma, const appga_params *params, const float *d_f_init,
                        hipStream_t st, appga_solve **out, bool afppa) {
    if (!ctx || !mat || !params || !d_g || !out)
        return fail(APPGA_E_INVALID_ARG, "NULL ctx, matrix, params, data or output");
    if (B <= 0) return fail(APPGA_E_INVALID_ARG, "B must be >= 1");
    if (mat->ctx != ctx) return fail(APPGA_E_INVALID_ARG, "matrix belongs to another context");
    for (int b = 0; b < B; ++b) ST_TRY(validate_params(&params[b], afppa));
    for (int b = 1; b < B; ++b)
        if (params[b].precond != params[0].precond ||
            params[b].precond_freeze_iter != params[0].precond_freeze_iter)
            return fail(APPGA_E_INVALID_ARG, "all solves of a batch need the same preconditioner mode");
    HIP_TRY(hipSetDevice(ctx->device));
    auto s = new appga_solve();
    s->ctx = ctx;
    s->mat = mat;
    s->B = B;
    s->st = st ? st : ctx->stream;
    s->prm.assign(params, params + B);
    s->afppa = afppa;
    s->has_gamma = d_gamma != nullptr;
    s->need_pbuf = params[0].precond == APPGA_PRECOND_EM_FROZEN;
    s->monitor_every = params[0].monitor_every;
    s->t0 = std::chrono::steady_clock::now();
    appga_status rs = sess_alloc(s);
    if (rs != APPGA_OK) {
        delete s;
        return rs;
    }
    auto bail = [&](appga_status code) {
        hipStreamSynchronize(s->st);
        hipFree(s->arena);
        delete s;
        return code;
    };
    const int64_t m = mat->A.n_rows, d = mat->A.n_cols;
    const int n = mat->geom.n;
    hipError_t he = hipSuccess;
    // inputs in the [index][B] layout
    if (B == 1) {
        he = hipMemcpyAsync(s->g, d_g, sizeof(float) * m, hipMemcpyDeviceToDevice, s->st);
        if (he == hipSuccess && d_gamma)
            he = hipMemcpyAsync(s->gamma, d_gamma, sizeof(float) * m, hipMemcpyDeviceToDevice, s->st);
    } else {
        he = launch_to_lanes(d_g, s->g, static_cast<int>(m), B, s->st);
        if (he == hipSuccess && d_gamma)
            he = launch_to_lanes(d_gamma, s->gamma, static_cast<int>(m), B, s->st);
    }
    // padding lanes get benign parameters (no regulariser, beta = 1, eps = 1)
    const int Bp = s->Bp;
    std::vector<LaneParams> lp(Bp, LaneParams{0.f, 0.f, 1.f, 1.f, 0.f, 0.f, 0.f, 0.f});
    std::vector<float> gl(Bp, 0.0f);
    for (int b = 0; b < B; ++b) {
        const appga_params &p = params[b];
        // eps = 0 makes the objective kernels evaluate the nonsmooth HOITV model
        lp[b] = LaneParams{static_cast<float>(p.lambda1), static_cast<float>(p.lambda2),
                           afppa ? 0.0f : static_cast<float>(p.eps), static_cast<float>(p.beta),
                           static_cast<float>(p.fixed_p), 0.f, 0.f, 0.f};
        gl[b] = static_cast<float>(p.gamma_scalar);
    }
    if (he == hipSuccess)
        he = hipMemcpyAsync(s->lp, lp.data(), sizeof(LaneParams) * Bp, hipMemcpyHostToDevice, s->st);
    if (he == hipSuccess)
        he = hipMemcpyAsync(s->gamma_lane, gl.data(), sizeof(float) * Bp, hipMemcpyHostToDevice, s->st);
    if (he == hipSuccess)
        he = launch_fill(reinterpret_cast<float *>(s->clamps), 2 * static_cast<size_t>(Bp), 0.0f, s->st);
    // AFPPA: b^0 = b^1 = 0, c^0 = c^1 = 0, max accumulators at 0 (the bits of +0.0f)
    if (he == hipSuccess && afppa)
        he = launch_fill(s->ydual, static_cast<size_t>(6) * d * Bp, 0.0f, s->st);
    if (he == hipSuccess && afppa)
        he = launch_fill(s->ybar, static_cast<size_t>(6) * d * Bp, 0.0f, s->st);
    if (he == hipSuccess && afppa)
        he = launch_fill(reinterpret_cast<float *>(s->pm), static_cast<size_t>(3) * kAfppaPmSlots * Bp, 0.0f,
                         s->st);
    // initial image f^0 = f^1
    if (he == hipSuccess) {
        if (d_f_init) {
            if (B == 1)
                he = hipMemcpyAsync(s->f, d_f_init, sizeof(float) * d, hipMemcpyDeviceToDevice, s->st);
            else
                he = launch_to_lanes(d_f_init, s->f, static_cast<int>(d), B, s->st);
            if (he == hipSuccess) he = launch_copy(s->ft[0], s->f, static_cast<size_t>(d) * Bp, s->st);
        } else {
            // ACTc = sum g - sum gamma per solve (FP64), TMC = ACTc / (NPFOV * NPA)
            he = launch_sum_g_minus_gamma(static_cast<int>(m), B, s->g, s->gamma, s->gamma_lane,
                                          s->part, s->st);
            if (he == hipSuccess)
                he = launch_reduce_partials(s->part, sum_blocks(static_cast<int>(m)), B, 1, s->red, s->st);
            std::vector<double> actc(B);
            if (he == hipSuccess)
                he = hipMemcpyAsync(actc.data(), s->red, sizeof(double) * B, hipMemcpyDeviceToHost, s->st);
            if (he == hipSuccess) he = hipStreamSynchronize(s->st);
            if (he == hipSuccess) {
                const double ctr = (n - 1) / 2.0, rad2 = (n / 2.0) * (n / 2.0);
                int64_t npfov = 0;
                for (int r = 0; r < n; ++r)
                    for (int c = 0; c < n; ++c)
                        npfov += (c - ctr) * (c - ctr) + (r - ctr) * (r - ctr) <= rad2;
                std::vector<double> tmc(Bp, 0.0);
                for (int b = 0; b < B; ++b) {
                    if (!std::isfinite(actc[b])) {
                        fail(APPGA_E_NONFINITE, "non-finite sum of the data of solve %d", b);
                        return bail(APPGA_E_NONFINITE);
                    }
                    if (!(actc[b] > 0)) {
                        fail(APPGA_E_DOMAIN, "ACTc = sum(g) - sum(gamma) <= 0 for solve %d", b);
                        return bail(APPGA_E_DOMAIN);
                    }
                    tmc[b] = actc[b] / (static_cast<double>(npfov) * mat->geom.n_angles);
                }
                he = hipMemcpyAsync(s->tmc, tmc.data(), sizeof(double) * Bp, hipMemcpyHostToDevice, s->st);
                if (he == hipSuccess) he = launch_disk_init(n, B, s->tmc, s->f, s->ft[0], s->st);
            }
        }
    }
    if (he != hipSuccess) {
        fail(APPGA_E_DEVICE, "session setup failed: %s", hipGetErrorString(he));
        return bail(APPGA_E_DEVICE);
    }
    s->cur = 0;
    s->k = 1;
    rs = sess_theta(s, 0);
    if (rs == APPGA_OK) rs = sess_objective(s, s->f, s->obj0);
    if (rs == APPGA_OK && s->monitor_every > 0) {
        s->hist_k.push_back(1);
        s->hist_obj.insert(s->hist_obj.end(), s->obj0.begin(), s->obj0.end());
    }
    if (rs != APPGA_OK) return bail(rs);
    *out = s;
    return APPGA_OK;
}

// One AFPPA iteration per pass (Section 4.3): the ratio forward projection at
// f~^k, the back projection A^T e (tile partial sums for batches with tiles,
// else the step kernel's gather), then the primal and the dual kernels.
static appga_status afppa_step(appga_solve *s, int n_iters) {
    const appga_matrix *mat = s->mat;
    const int B = s->B, Bp = s->Bp;
    const appga_params &p0 = s->prm[0];
    for (int it = 0; it < n_iters; ++it) {
        const int k = s->k;
        if (k + 1 > s->theta_base + s->theta_cap) ST_TRY(sess_theta(s, k));
        FwdArgs fa{};
        fa.row_ptr = mat->A.row_ptr;
        fa.col = mat->A.col;
        fa.val = mat->A.val;
        fa.row_scale = mat->A.row_scale;
        fa.col32 = mat->A.col32;
        fa.nnz_padded = mat->A.nnz_padded;
        fa.m = mat->A.n_rows;
        fa.n_x = mat->A.n_cols;
        fa.B = B;
        fa.Bp = Bp;
        fa.x = s->ft[s->cur];
        if (mat->psf_R >= 0) {   // the forward takes H f~
            HIP_TRY(timed_launch(s->ctx, "psf_fwd", s->st, [&] {
                return psf_blur(mat, s->ft[s->cur], 1, s->tb, s->xb, B, Bp, s->st);
            }));
            fa.x = s->xb;
        }
        fa.g = s->g;
        fa.gamma = s->gamma;
        fa.gamma_lane = s->gamma_lane;
        fa.out = s->e;
        fa.mode = FM_RATIO;
        fa.scale_out = 1;
        fa.fwd_wgs = mat->fwd_wgs;
        fa.clamps = s->clamps;
        fa.tile_part = s->tile_part;
        const char *fname = B == 1 ? "forward_single" : (forward_uses_tiles(mat, fa) ? "fwd_tiles" : "forward_batch");
        HIP_TRY(timed_launch(s->ctx, fname, s->st, [&] { return launch_forward_mat(mat, fa, s->st); }));
        if (B > 1 && mat->bt.valid) {
            HIP_TRY(timed_launch(s->ctx, "back_tiles", s->st, [&] {
                return launch_back_tiles(mat->bt, mat->AT.vtype, mat->geom.n, mat->A.n_rows, Bp,
                                         mat->bt_remap, mat->bt_split, s->e, s->gf, s->st);
            }));
        } else {
            StepArgs sa{};
            sa.row_ptr = mat->AT.row_ptr;
            sa.col = mat->AT.col;
            sa.val = mat->AT.val;
            sa.row_scale = mat->AT.row_scale;
            sa.col32 = mat->AT.col32;
            sa.nnz_padded = mat->AT.nnz_padded;
            sa.n = mat->geom.n;
            sa.m = mat->A.n_rows;
            sa.B = B;
            sa.Bp = Bp;
            sa.e = s->e;
            sa.ft = s->ft[s->cur];
            sa.f = s->f;
            sa.ft_next = s->ft[s->cur ^ 1];
            sa.lam = mat->lam;
            sa.lp = s->lp;
            sa.theta_next = s->theta;
            sa.pmode = PM_EM;
            sa.out_mode = SO_BACK;
            sa.out = s->gf;
            sa.tiles_x = (mat->geom.n + 3) / 4;
            sa.xcd_remap = mat->xcd_remap;
            HIP_TRY(timed_launch(s->ctx, B == 1 ? "back_single" : "back_batch", s->st,
                                 [&] { return launch_step_mat(mat, sa, mat->group_back, s->st); }));
        }
        AfppaArgs aa{};
        aa.n = mat->geom.n;
        aa.B = B;
        aa.Bp = Bp;
        aa.gf = s->gf;
        aa.gf_split = s->gf_split;
        if (mat->psf_R >= 0) {   // grad F = H (A^T e)
            HIP_TRY(timed_launch(s->ctx, "psf_back", s->st, [&] {
                return psf_blur(mat, s->gf, s->gf_split, s->tb, s->gfb, B, Bp, s->st);
            }));
            aa.gf = s->gfb;
            aa.gf_split = 1;
        }
        aa.f = s->f;
        aa.ft = s->ft[s->cur];
        aa.ft_next = s->ft[s->cur ^ 1];
        aa.w = s->w;
        aa.y = s->ydual;
        aa.ybar = s->ybar;
        aa.lam = mat->lam;
        aa.lp = s->lp;
        aa.theta_next = s->theta + static_cast<size_t>(k + 1 - s->theta_base) * Bp;
        aa.pmode = p0.precond == APPGA_PRECOND_FIXED ? PM_FIXED : PM_EM;
        const size_t pm_set = static_cast<size_t>(kAfppaPmSlots) * Bp;
        aa.pmax_acc = s->pm + static_cast<size_t>(k % 3) * pm_set;
        aa.pmax_in = aa.pmax_acc;
        aa.pmax_clear = s->pm + static_cast<size_t>((k + 1) % 3) * pm_set;
        aa.re_part = (it == n_iters - 1) ? s->part : nullptr;
        HIP_TRY(timed_launch(s->ctx, "afppa_primal", s->st, [&] { return launch_afppa_primal(aa, s->st); }));
        HIP_TRY(timed_launch(s->ctx, "afppa_dual", s->st, [&] { return launch_afppa_dual(aa, s->st); }));
        s->cur ^= 1;
        s->k += 1;
        s->re_valid = (it == n_iters - 1);
        s->re_blocks = afppa_blocks(mat->geom.n, Bp);
        if (s->monitor_every > 0 && (s->k - 1) % s->monitor_every == 0) {
            std::vector<double> obj;
            ST_TRY(sess_objective(s, s->f, obj, s->mpart, s->mred));
            s->hist_k.push_back(s->k);
            s->hist_obj.insert(s->hist_obj.end(), obj.begin(), obj.end());
        }
    }
    return APPGA_OK;
}

appga_status sess_step(appga_solve *s, int n_iters) {
    if (!s) return fail(APPGA_E_INVALID_ARG, "session is NULL");
    if (n_iters < 0) return fail(APPGA_E_INVALID_ARG, "n_iters must be >= 0");
    if (s->afppa) return afppa_step(s, n_iters);
    const appga_matrix *mat = s->mat;
    const int B = s->B;
    const appga_params &p0 = s->prm[0];
    for (int it = 0; it < n_iters; ++it) {
        const int k = s->k;
        if (k + 1 > s->theta_base + s->theta_cap) ST_TRY(sess_theta(s, k));
        FwdArgs fa{};
        fa.row_ptr = mat->A.row_ptr;
        fa.col = mat->A.col;
        fa.val = mat->A.val;
        fa.row_scale = mat->A.row_scale;
        fa.col32 = mat->A.col32;
        fa.nnz_padded = mat->A.nnz_padded;
        fa.m = mat->A.n_rows;
        fa.n_x = mat->A.n_cols;
        fa.B = B;
        fa.Bp = s->Bp;
        fa.x = s->ft[s->cur];
        if (mat->psf_R >= 0) {   // the forward takes H f~
            HIP_TRY(timed_launch(s->ctx, "psf_fwd", s->st, [&] {
                return psf_blur(mat, s->ft[s->cur], 1, s->tb, s->xb, B, s->Bp, s->st);
            }));
            fa.x = s->xb;
        }
        fa.g = s->g;
        fa.gamma = s->gamma;
        fa.gamma_lane = s->gamma_lane;
        fa.out = s->e;
        fa.mode = FM_RATIO;
        fa.scale_out = 1;
        fa.fwd_wgs = mat->fwd_wgs;
        fa.clamps = s->clamps;
        fa.tile_part = s->tile_part;
        const char *fname = B == 1 ? "forward_single" : (forward_uses_tiles(mat, fa) ? "fwd_tiles" : "forward_batch");
        HIP_TRY(timed_launch(s->ctx, fname, s->st, [&] { return launch_forward_mat(mat, fa, s->st); }));
        StepArgs sa{};
        sa.row_ptr = mat->AT.row_ptr;
        sa.col = mat->AT.col;
        sa.val = mat->AT.val;
        sa.row_scale = mat->AT.row_scale;
        sa.col32 = mat->AT.col32;
        sa.nnz_padded = mat->AT.nnz_padded;
        sa.n = mat->geom.n;
        sa.m = mat->A.n_rows;
        sa.B = B;
        sa.Bp = s->Bp;
        sa.e = s->e;
        sa.ft = s->ft[s->cur];
        sa.f = s->f;
        sa.ft_next = s->ft[s->cur ^ 1];
        sa.lam = mat->lam;
        sa.lp = s->lp;
        sa.theta_next = s->theta + static_cast<size_t>(k + 1 - s->theta_base) * s->Bp;
        sa.pbuf = s->pbuf;
        if (p0.precond == APPGA_PRECOND_FIXED)
            sa.pmode = PM_FIXED;
        else if (p0.precond == APPGA_PRECOND_EM_FROZEN)
            sa.pmode = (k == 1 || k <= p0.precond_freeze_iter) ? PM_EM_STORE : PM_STORED;
        else
            sa.pmode = PM_EM;
        sa.out_mode = SO_STEP;
        sa.re_part = (it == n_iters - 1) ? s->part : nullptr;
        sa.tiles_x = (mat->geom.n + 3) / 4;
        sa.xcd_remap = mat->xcd_remap;
        if (mat->psf_R >= 0) {
            // grad F = H (A^T e): the back projection on its own (tiles, or the step
            // kernel's gather), then the blur; the step takes the result
            if (B > 1 && mat->bt.valid) {
                HIP_TRY(timed_launch(s->ctx, "back_tiles", s->st, [&] {
                    return launch_back_tiles(mat->bt, mat->AT.vtype, mat->geom.n, mat->A.n_rows, s->Bp,
                                             mat->bt_remap, mat->bt_split, s->e, s->gf, s->st);
                }));
            } else {
                StepArgs sb = sa;
                sb.out_mode = SO_BACK;
                sb.out = s->gf;
                sb.re_part = nullptr;
                HIP_TRY(timed_launch(s->ctx, B == 1 ? "back_single" : "back_batch", s->st,
                                     [&] { return launch_step_mat(mat, sb, mat->group_back, s->st); }));
            }
            HIP_TRY(timed_launch(s->ctx, "psf_back", s->st, [&] {
                return psf_blur(mat, s->gf, s->gf_split, s->tb, s->gfb, B, s->Bp, s->st);
            }));
            sa.gf_in = s->gfb;
            sa.gf_split = 1;
        } else if (s->gf) {
            HIP_TRY(timed_launch(s->ctx, "back_tiles", s->st, [&] {
                return launch_back_tiles(mat->bt, mat->AT.vtype, mat->geom.n, mat->A.n_rows, s->Bp,
                                         mat->bt_remap, mat->bt_split, s->e, s->gf, s->st);
            }));
            sa.gf_in = s->gf;
            sa.gf_split = mat->bt_split;
        }
        HIP_TRY(timed_launch(s->ctx, B == 1 ? "step_single" : "step_batch", s->st,
                             [&] { return launch_step_mat(mat, sa, mat->group_back, s->st); }));
        s->cur ^= 1;
        s->k += 1;
        s->re_valid = (it == n_iters - 1);
        s->re_blocks = step_blocks(mat->geom.n, B);
        if (s->monitor_every > 0 && (s->k - 1) % s->monitor_every == 0) {
            std::vector<double> obj;
            ST_TRY(sess_objective(s, s->f, obj, s->mpart, s->mred));
            s->hist_k.push_back(s->k);
            s->hist_obj.insert(s->hist_obj.end(), obj.begin(), obj.end());
        }
    }
    return APPGA_OK;
}

appga_status sess_end(appga_solve *s, float *d_out, appga_stats *stats, bool free_session) {
    if (!s) return fail(APPGA_E_INVALID_ARG, "session is NULL");
    const int B = s->B;
    const int64_t d = s->mat->A.n_cols;
    const int n = s->mat->geom.n;
    appga_status rs = APPGA_OK;
    std::vector<double> re(2 * B, 0.0);
    if (s->re_valid) {
        HIP_TRY(launch_reduce_partials(s->part, s->re_blocks, B, 2, s->red + 2 * B, s->st));
        HIP_TRY(hipMemcpyAsync(re.data(), s->red + 2 * B, sizeof(double) * 2 * B,
                               hipMemcpyDeviceToHost, s->st));
    }
    std::vector<double> obj;
    rs = sess_objective(s, s->f, obj);
    if (rs != APPGA_OK) return rs;
    std::vector<unsigned long long> cl(B);
    HIP_TRY(hipMemcpyAsync(cl.data(), s->clamps, sizeof(unsigned long long) * B,
                           hipMemcpyDeviceToHost, s->st));
    if (d_out) {
        if (B == 1)
            HIP_TRY(hipMemcpyAsync(d_out, s->f, sizeof(float) * d, hipMemcpyDeviceToDevice, s->st));
        else
            HIP_TRY(launch_from_lanes(s->f, d_out, static_cast<int>(d), B, s->st));
    }
    HIP_TRY(hipStreamSynchronize(s->st));
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
    bool nonfinite = false;
    for (int b = 0; b < B; ++b) {
        if (!std::isfinite(obj[b])) nonfinite = true;
        if (stats) {
            stats[b].iterations_done = s->k - 1;
            stats[b].objective0 = s->obj0[b];
            stats[b].objective = obj[b];
            stats[b].re = (s->re_valid && re[2 * b + 1] > 0) ? std::sqrt(re[2 * b] / re[2 * b + 1]) : 0.0;
            stats[b].guard_clamps = static_cast<int64_t>(cl[b]);
            stats[b].seconds = secs;
        }
    }
    if (free_session) {
        hipFree(s->arena);
        delete s;
    }
    if (nonfinite) return fail(APPGA_E_NONFINITE, "non-finite objective: the iterates diverged");
    return APPGA_OK;
}

void sess_free(appga_solve *s) {
    if (!s) return;
    hipStreamSynchronize(s->st);
    hipFree(s->arena);
    delete s;
}

}  // namespace appga

extern "C" appga_status appga_solve_begin(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                          const float *d_g, const float *d_gamma,
                                          const appga_params *params, const float *d_f_init,
                                          void *hip_stream, appga_solve **out) {
    clear_error();
    return sess_begin(ctx, mat, B, d_g, d_gamma, params, d_f_init,
                      static_cast<hipStream_t>(hip_stream), out);
}

extern "C" appga_status appga_solve_step(appga_solve *s, int32_t n_iters) {
    clear_error();
    return sess_step(s, n_iters);
}

extern "C" appga_status appga_solve_history(const appga_solve *s, int32_t solve, int32_t cap,
                                            int32_t *iters_out, double *obj_out, int32_t *count) {
    clear_error();
    if (!s || !count) return fail(APPGA_E_INVALID_ARG, "NULL session or count");
    if (solve < 0 || solve >= s->B) return fail(APPGA_E_INVALID_ARG, "solve index %d out of range", solve);
    const int32_t n = static_cast<int32_t>(s->hist_k.size());
    *count = n;
    if (cap > 0 && (!iters_out || !obj_out)) return fail(APPGA_E_INVALID_ARG, "NULL output arrays");
    for (int32_t i = 0; i < std::min(n, cap); ++i) {
        iters_out[i] = s->hist_k[i];
        obj_out[i] = s->hist_obj[static_cast<size_t>(i) * s->B + solve];
    }
    return APPGA_OK;
}

extern "C" appga_status appga_solve_end(appga_solve *s, float *d_out, appga_stats *stats) {
    clear_error();
    if (!s) return fail(APPGA_E_INVALID_ARG, "session is NULL");
    appga_status st = sess_end(s, d_out, stats, false);
    sess_free(s);
    return st;
}

// ------------------------------------------------------------ solvers ---

namespace {

// The duals (b, c) of an AFPPA session, solve-major [B][6 d] (b: 2 d, then c: 4 d).
appga_status sess_duals(const appga_solve *s, float *d_duals) {
    if (!s) return fail(APPGA_E_INVALID_ARG, "session is NULL");
    if (!s->afppa) return fail(APPGA_E_INVALID_ARG, "not an AFPPA session");
    if (!d_duals) return fail(APPGA_E_INVALID_ARG, "NULL output");
    const int64_t len = 6 * s->mat->A.n_cols;
    if (s->Bp == 1)
        HIP_TRY(hipMemcpyAsync(d_duals, s->ydual, sizeof(float) * len, hipMemcpyDeviceToDevice, s->st));
    else
        HIP_TRY(launch_from_lanes(s->ydual, d_duals, static_cast<int>(len), s->B, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    return APPGA_OK;
}

// The current image f^k of a session, solve-major [B][d].
appga_status sess_image(const appga_solve *s, float *d_out) {
    if (!s) return fail(APPGA_E_INVALID_ARG, "session is NULL");
    if (!d_out) return fail(APPGA_E_INVALID_ARG, "NULL output");
    const int64_t d = s->mat->A.n_cols;
    if (s->Bp == 1)
        HIP_TRY(hipMemcpyAsync(d_out, s->f, sizeof(float) * d, hipMemcpyDeviceToDevice, s->st));
    else
        HIP_TRY(launch_from_lanes(s->f, d_out, static_cast<int>(d), s->B, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    return APPGA_OK;
}

appga_status run_batch_device(appga_ctx *ctx, const appga_matrix *mat, int B, const float *d_g,
                              const float *d_gamma, const appga_params *params,
                              const float *d_f_init, float *d_out, hipStream_t st,
                              appga_stats *stats, bool afppa = false, float *d_duals = nullptr) {
    for (int b = 0; b < B; ++b) ST_TRY(validate_params(&params[b], afppa));
    for (int b = 1; b < B; ++b)
        if (params[b].iterations != params[0].iterations)
            return fail(APPGA_E_INVALID_ARG, "all solves of a batch need the same iteration count");
    appga_solve *s = nullptr;
    ST_TRY(sess_begin(ctx, mat, B, d_g, d_gamma, params, d_f_init, st, &s, afppa));
    appga_status rs = sess_step(s, params[0].iterations);
    if (rs == APPGA_OK && d_duals) rs = sess_duals(s, d_duals);
    if (rs == APPGA_OK) rs = sess_end(s, d_out, stats, false);
    sess_free(s);
    return rs;
}

appga_status run_batch_host(appga_ctx *ctx, const appga_matrix *mat, int B, const float *g,
                            const float *gamma, const appga_params *params, const float *f_init,
                            float *f_out, appga_stats *stats, bool afppa = false,
                            float *duals_out = nullptr) {
    if (!ctx || !mat || !g || !params || !f_out)
        return fail(APPGA_E_INVALID_ARG, "NULL ctx, matrix, data, params or output");
    if (B <= 0) return fail(APPGA_E_INVALID_ARG, "B must be >= 1");
    const int64_t m = mat->A.n_rows, d = mat->A.n_cols;
    for (int b = 0; b < B; ++b) ST_TRY(validate_params(&params[b], afppa));
    ST_TRY(validate_data(g, m * B, "sinogram"));
    if (gamma) ST_TRY(validate_data(gamma, m * B, "background"));
    if (f_init) ST_TRY(validate_data(f_init, d * B, "f_init"));
    HIP_TRY(hipSetDevice(ctx->device));
    float *buf = nullptr;
    const size_t ndual = duals_out ? static_cast<size_t>(6) * d * B : 0;
    const size_t nf = static_cast<size_t>(m) * B * (gamma ? 2 : 1) + static_cast<size_t>(d) * B * (f_init ? 2 : 1) +
                      ndual;
    HIP_TRY(hipMalloc(&buf, sizeof(float) * nf));
    float *dg = buf, *dgam = gamma ? buf + m * B : nullptr;
    float *dfi = f_init ? buf + m * B * (gamma ? 2 : 1) : nullptr;
    float *dout = buf + m * B * (gamma ? 2 : 1) + (f_init ? d * B : 0);
    float *ddual = duals_out ? dout + d * B : nullptr;
    hipStream_t st = ctx->stream;
    appga_status rs = APPGA_OK;
    hipError_t he = hipMemcpyAsync(dg, g, sizeof(float) * m * B, hipMemcpyHostToDevice, st);
    if (he == hipSuccess && gamma)
        he = hipMemcpyAsync(dgam, gamma, sizeof(float) * m * B, hipMemcpyHostToDevice, st);
    if (he == hipSuccess && f_init)
        he = hipMemcpyAsync(dfi, f_init, sizeof(float) * d * B, hipMemcpyHostToDevice, st);
    if (he != hipSuccess) {
        rs = fail(APPGA_E_DEVICE, "upload failed: %s", hipGetErrorString(he));
    } else {
        std::vector<appga_stats> tmp(B);
        rs = run_batch_device(ctx, mat, B, dg, dgam, params, dfi, dout, st, tmp.data(), afppa, ddual);
        if (rs == APPGA_OK || rs == APPGA_E_NONFINITE) {
            if (stats) std::memcpy(stats, tmp.data(), sizeof(appga_stats) * B);
        }
        if (rs == APPGA_OK) {
            he = hipMemcpy(f_out, dout, sizeof(float) * d * B, hipMemcpyDeviceToHost);
            if (he == hipSuccess && duals_out)
                he = hipMemcpy(duals_out, ddual, sizeof(float) * ndual, hipMemcpyDeviceToHost);
            if (he != hipSuccess) rs = fail(APPGA_E_DEVICE, "download failed: %s", hipGetErrorString(he));
        }
    }
    hipStreamSynchronize(st);
    hipFree(buf);
    return rs;
}

}  // namespace

extern "C" appga_status appga_reconstruct(appga_ctx *ctx, const appga_matrix *mat,
                                          const float *sinogram, const float *background,
                                          const appga_params *params, const float *f_init,
                                          float *f_out, appga_stats *stats) {
    clear_error();
    return run_batch_host(ctx, mat, 1, sinogram, background, params, f_init, f_out, stats);
}

extern "C" appga_status appga_reconstruct_simple(appga_ctx *ctx, const appga_matrix *mat,
                                                 const float *g, const float *gamma, double lambda,
                                                 double eps, double omega, int32_t iterations,
                                                 float *f_out) {
    clear_error();
    appga_params p;
    appga_params_default(&p);
    p.lambda1 = p.lambda2 = lambda;
    p.eps = eps;
    p.omega = omega;
    p.iterations = iterations;
    return run_batch_host(ctx, mat, 1, g, gamma, &p, nullptr, f_out, nullptr);
}

extern "C" appga_status appga_reconstruct_batch(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                                const float *g, const float *gamma,
                                                const appga_params *params, const float *f_init,
                                                float *f_out, appga_stats *stats) {
    clear_error();
    return run_batch_host(ctx, mat, B, g, gamma, params, f_init, f_out, stats);
}

extern "C" appga_status appga_reconstruct_batch_device(appga_ctx *ctx, const appga_matrix *mat,
                                                       int32_t B, const float *d_g,
                                                       const float *d_gamma,
                                                       const appga_params *params,
                                                       const float *d_f_init, float *d_out,
                                                       void *hip_stream) {
    clear_error();
    if (!ctx || !mat || !d_g || !params || !d_out)
        return fail(APPGA_E_INVALID_ARG, "NULL ctx, matrix, data, params or output");
    if (B <= 0) return fail(APPGA_E_INVALID_ARG, "B must be >= 1");
    return run_batch_device(ctx, mat, B, d_g, d_gamma, params, d_f_init, d_out,
                            static_cast<hipStream_t>(hip_stream), nullptr);
}

extern "C" appga_status appga_afppa_batch(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                          const float *g, const float *gamma, const appga_params *params,
                                          const float *f_init, float *f_out, float *duals_out,
                                          appga_stats *stats) {
    clear_error();
    return run_batch_host(ctx, mat, B, g, gamma, params, f_init, f_out, stats, true, duals_out);
}

extern "C" appga_status appga_afppa_batch_device(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                                 const float *d_g, const float *d_gamma,
                                                 const appga_params *params, const float *d_f_init,
                                                 float *d_out, float *d_duals_out, void *hip_stream) {
    clear_error();
    if (!ctx || !mat || !d_g || !params || !d_out)
        return fail(APPGA_E_INVALID_ARG, "NULL ctx, matrix, data, params or output");
    if (B <= 0) return fail(APPGA_E_INVALID_ARG, "B must be >= 1");
    return run_batch_device(ctx, mat, B, d_g, d_gamma, params, d_f_init, d_out,
                            static_cast<hipStream_t>(hip_stream), nullptr, true, d_duals_out);
}

extern "C" appga_status appga_afppa_begin(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                          const float *d_g, const float *d_gamma,
                                          const appga_params *params, const float *d_f_init,
                                          void *hip_stream, appga_solve **out) {
    clear_error();
    return sess_begin(ctx, mat, B, d_g, d_gamma, params, d_f_init, static_cast<hipStream_t>(hip_stream),
                      out, true);
}

extern "C" appga_status appga_solve_duals(const appga_solve *s, float *d_duals) {
    clear_error();
    return sess_duals(s, d_duals);
}

extern "C" appga_status appga_solve_image(const appga_solve *s, float *d_out) {
    clear_error();
    return sess_image(s, d_out);
}

// ------------------------------------------------------------ operators ---

namespace {

// Temporary buffers of the operator entry points, in the layout of B.
struct OpBufs {
    void *mem = nullptr;
    ~OpBufs() { hipFree(mem); }
};

hipStream_t pick_stream(appga_ctx *ctx, void *s) {
    return s ? static_cast<hipStream_t>(s) : ctx->stream;
}

appga_status to_internal(const float *src, float *dst, int B, int64_t len, hipStream_t st) {
    if (B == 1)
        HIP_TRY(hipMemcpyAsync(dst, src, sizeof(float) * len, hipMemcpyDeviceToDevice, st));
    else
        HIP_TRY(launch_to_lanes(src, dst, static_cast<int>(len), B, st));
    return APPGA_OK;
}

appga_status from_internal(const float *src, float *dst, int B, int64_t len, hipStream_t st) {
    if (B == 1)
        HIP_TRY(hipMemcpyAsync(dst, src, sizeof(float) * len, hipMemcpyDeviceToDevice, st));
    else
        HIP_TRY(launch_from_lanes(src, dst, static_cast<int>(len), B, st));
    return APPGA_OK;
}

appga_status op_forward_impl(appga_ctx *ctx, const appga_matrix *mat, int B, const float *d_x,
                             const float *d_g, const float *d_gamma, float *d_y, int mode,
                             void *stream, int scale_out = 0) {
    if (!ctx || !mat || !d_x || !d_y || (mode == FM_RATIO && !d_g))
        return fail(APPGA_E_INVALID_ARG, "NULL argument");
    if (B <= 0) return fail(APPGA_E_INVALID_ARG, "B must be >= 1");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = pick_stream(ctx, stream);
    const int64_t m = mat->A.n_rows, d = mat->A.n_cols;
    const int Bp = pad_lanes(B);
    OpBufs ob;
    const size_t ntp = B > 1 && mat->ft.valid ? fwd_tile_part_floats(mat->ft, Bp) : 0;
    const bool psf = mat->psf_R >= 0;
    const size_t nf = static_cast<size_t>(d) * Bp * (psf ? 3 : 1) + 3 * static_cast<size_t>(m) * Bp + ntp;
    HIP_TRY(hipMalloc(&ob.mem, sizeof(float) * nf));
    float *x = static_cast<float *>(ob.mem), *g = x + d * Bp, *gam = g + m * Bp, *y = gam + m * Bp;
    float *tp = ntp ? y + m * Bp : nullptr;
    float *xb = psf ? y + m * Bp + ntp : nullptr, *tb = psf ? xb + d * Bp : nullptr;
    ST_TRY(to_internal(d_x, x, B, d, st));
    if (psf) {   // A x = diag(n) G (H x)
        HIP_TRY(timed_launch(ctx, "op_psf", st, [&] { return psf_blur(mat, x, 1, tb, xb, B, Bp, st); }));
        x = xb;
    }
    if (d_g) ST_TRY(to_internal(d_g, g, B, m, st));
    if (d_gamma) ST_TRY(to_internal(d_gamma, gam, B, m, st));
    FwdArgs fa{};
    fa.row_ptr = mat->A.row_ptr;
    fa.col = mat->A.col;
    fa.col32 = mat->A.col32;
        fa.nnz_padded = mat->A.nnz_padded;
    fa.val = mat->A.val;
    fa.row_scale = mat->A.row_scale;
    fa.m = static_cast<int>(m);
    fa.n_x = static_cast<int>(d);
    fa.B = B;
    fa.Bp = Bp;
    fa.x = x;
    fa.g = g;
    fa.gamma = d_gamma ? gam : nullptr;
    fa.gamma_lane = nullptr;
    fa.out = y;
    fa.mode = mode;
    fa.scale_out = scale_out;
    fa.fwd_wgs = mat->fwd_wgs;
    fa.tile_part = tp;
    const char *fname = B == 1 ? "op_forward_single" : (forward_uses_tiles(mat, fa) ? "op_fwd_tiles" : "op_forward_batch");
    HIP_TRY(timed_launch(ctx, fname, st, [&] { return launch_forward_mat(mat, fa, st); }));
    ST_TRY(from_internal(y, d_y, B, m, st));
    HIP_TRY(hipStreamSynchronize(st));
    return APPGA_OK;
}

appga_status op_step_impl(appga_ctx *ctx, const appga_matrix *mat, int n, int B, const float *d_e,
                          const double *lambda1, const double *lambda2, const double *eps,
                          const double *beta, const double *theta_next, float *d_f,
                          const float *d_ft, float *d_ft_next, float *d_out, int out_mode,
                          void *stream, int scale_rows = 0) {
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = pick_stream(ctx, stream);
    const int64_t d = static_cast<int64_t>(n) * n;
    const int64_t m = mat ? mat->A.n_rows : 0;
    const int Bp = pad_lanes(B);
    const bool psf = mat && mat->psf_R >= 0 && out_mode != SO_REG;
    if (psf && out_mode != SO_BACK)
        return fail(APPGA_E_INVALID_ARG, "appga_op_step does not model a PSF; use a session");
    OpBufs ob;
    const int split = mat ? mat->bt_split : 1;
    const size_t nfl = static_cast<size_t>(d) * Bp * (4 + split) + static_cast<size_t>(m) * Bp + Bp;
    const size_t lp_off = (sizeof(float) * nfl + 255) / 256 * 256;
    HIP_TRY(hipMalloc(&ob.mem, lp_off + sizeof(LaneParams) * Bp));
    float *e = static_cast<float *>(ob.mem);
    float *ft = e + m * Bp, *f = ft + d * Bp, *ftn = f + d * Bp, *out = ftn + d * Bp, *gf = out + d * Bp,
          *th = gf + d * Bp * split;
    LaneParams *lp = reinterpret_cast<LaneParams *>(static_cast<char *>(ob.mem) + lp_off);
    if (d_e) ST_TRY(to_internal(d_e, e, B, m, st));
    if (d_e && scale_rows && mat && mat->A.row_scale)
        HIP_TRY(launch_scale_rows(e, mat->A.row_scale, static_cast<int>(m), B, st));
    if (d_ft)
        ST_TRY(to_internal(d_ft, ft, B, d, st));
    else
        HIP_TRY(launch_fill(ft, static_cast<size_t>(d) * Bp, 0.0f, st));
    if (d_f)
        ST_TRY(to_internal(d_f, f, B, d, st));
    else
        HIP_TRY(launch_fill(f, static_cast<size_t>(d) * Bp, 0.0f, st));
    std::vector<LaneParams> hlp(Bp, LaneParams{0.f, 0.f, 1.f, 1.f, 0.f, 0.f, 0.f, 0.f});
    std::vector<float> hth(Bp, 0.0f);
    for (int b = 0; b < B; ++b) {
        hlp[b] = LaneParams{static_cast<float>(lambda1[b]), static_cast<float>(lambda2[b]),
                            static_cast<float>(eps[b]), beta ? static_cast<float>(beta[b]) : 1.0f,
                            0.f, 0.f, 0.f, 0.f};
        if (theta_next) hth[b] = static_cast<float>(theta_next[b]);
    }
    HIP_TRY(hipMemcpyAsync(lp, hlp.data(), sizeof(LaneParams) * Bp, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(th, hth.data(), sizeof(float) * Bp, hipMemcpyHostToDevice, st));
    StepArgs sa{};
    DevCsr dummy;
    const DevCsr &AT = mat ? mat->AT : dummy;
    sa.row_ptr = AT.row_ptr;
    sa.col = AT.col;
    sa.col32 = AT.col32;
    sa.nnz_padded = AT.nnz_padded;
    sa.val = AT.val;
    sa.row_scale = AT.row_scale;
    sa.n = n;
    sa.m = static_cast<int>(m);
    sa.B = B;
    sa.Bp = Bp;
    sa.e = e;
    sa.ft = ft;
    sa.f = f;
    sa.ft_next = ftn;
    sa.lam = mat ? mat->lam : nullptr;
    sa.lp = lp;
    sa.theta_next = th;
    sa.pbuf = nullptr;
    sa.pmode = PM_EM;
    sa.out_mode = out_mode;
    sa.out = out;
    sa.re_part = nullptr;
    sa.tiles_x = (n + 3) / 4;
    sa.xcd_remap = mat ? mat->xcd_remap : 0;
    const int group = mat ? mat->group_back : 16;
    const char *name = out_mode == SO_REG ? "op_grad_reg" : (out_mode == SO_BACK ? "op_back" : "op_step");
    const bool tiles = mat && B > 1 && mat->bt.valid && out_mode != SO_REG;
    if (tiles) {
        HIP_TRY(timed_launch(ctx, "op_back_tiles", st, [&] {
            return launch_back_tiles(mat->bt, AT.vtype, n, static_cast<int>(m), Bp, mat->bt_remap, split, e,
                                     gf, st);
        }));
        sa.gf_in = gf;
        sa.gf_split = split;
    }
    HIP_TRY(timed_launch(ctx, name, st, [&] {
        return mat ? launch_step_mat(mat, sa, group, st) : launch_step(AT, sa, group, st);
    }));
    if (psf) {   // A^T e = H (G^T diag(n) e): blur the back projection (f and ft_next serve as scratch)
        HIP_TRY(timed_launch(ctx, "op_psf", st, [&] { return psf_blur(mat, out, 1, f, ftn, B, Bp, st); }));
        out = ftn;
    }
    if (out_mode == SO_STEP) {
        ST_TRY(from_internal(f, d_f, B, d, st));
        ST_TRY(from_internal(ftn, d_ft_next, B, d, st));
    } else {
        ST_TRY(from_internal(out, d_out, B, d, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    return APPGA_OK;
}

}  // namespace

extern "C" appga_status appga_op_forward(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                         const float *d_x, const float *d_gamma, float *d_y,
                                         void *hip_stream) {
    clear_error();
    return op_forward_impl(ctx, mat, B, d_x, nullptr, d_gamma, d_y, FM_PROJ, hip_stream);
}

extern "C" appga_status appga_op_ratio(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                       const float *d_x, const float *d_g, const float *d_gamma,
                                       float *d_e, void *hip_stream) {
    clear_error();
    return op_forward_impl(ctx, mat, B, d_x, d_g, d_gamma, d_e, FM_RATIO, hip_stream);
}

extern "C" appga_status appga_op_back(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                      const float *d_r, float *d_out, void *hip_stream) {
    clear_error();
    if (!ctx || !mat || !d_r || !d_out) return fail(APPGA_E_INVALID_ARG, "NULL argument");
    if (B <= 0) return fail(APPGA_E_INVALID_ARG, "B must be >= 1");
    std::vector<double> z(B, 0.0), one(B, 1.0);
    return op_step_impl(ctx, mat, mat->geom.n, B, d_r, z.data(), z.data(), one.data(), nullptr,
                        nullptr, nullptr, nullptr, nullptr, d_out, SO_BACK, hip_stream, 1);
}

extern "C" appga_status appga_op_grad_reg(appga_ctx *ctx, int32_t n, int32_t B,
                                          const double *lambda1, const double *lambda2,
                                          const double *eps, const float *d_x, float *d_out,
                                          void *hip_stream) {
    clear_error();
    if (!ctx || !lambda1 || !lambda2 || !eps || !d_x || !d_out)
        return fail(APPGA_E_INVALID_ARG, "NULL argument");
    if (n <= 0 || B <= 0) return fail(APPGA_E_INVALID_ARG, "n and B must be >= 1");
    for (int b = 0; b < B; ++b)
        if (!(eps[b] > 0) || lambda1[b] < 0 || lambda2[b] < 0)
            return fail(APPGA_E_DOMAIN, "need eps > 0 and lambda >= 0");
    return op_step_impl(ctx, nullptr, n, B, nullptr, lambda1, lambda2, eps, nullptr, nullptr,
                        nullptr, d_x, nullptr, d_out, SO_REG, hip_stream);
}

extern "C" appga_status appga_op_step(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                      const float *d_g, const float *d_gamma,
                                      const double *lambda1, const double *lambda2,
                                      const double *eps, const double *beta,
                                      const double *theta_next, float *d_f, const float *d_ft,
                                      float *d_ft_next, void *hip_stream) {
    clear_error();
    if (!ctx || !mat || !d_g || !lambda1 || !lambda2 || !eps || !beta || !theta_next || !d_f ||
        !d_ft || !d_ft_next)
        return fail(APPGA_E_INVALID_ARG, "NULL argument");
    if (B <= 0) return fail(APPGA_E_INVALID_ARG, "B must be >= 1");
    // e = 1 - g / max(A ft + gamma, tau) first, then the fused step
    const int64_t m = mat->A.n_rows;
    float *e = nullptr;
    HIP_TRY(hipMalloc(&e, sizeof(float) * m * B));
    appga_status rs = op_forward_impl(ctx, mat, B, d_ft, d_g, d_gamma, e, FM_RATIO, hip_stream, 1);
    if (rs == APPGA_OK)
        rs = op_step_impl(ctx, mat, mat->geom.n, B, e, lambda1, lambda2, eps, beta, theta_next, d_f,
                          d_ft, d_ft_next, nullptr, SO_STEP, hip_stream);
    hipFree(e);
    return rs;
}

// --------------------------------------------------------------- serving ---
// (server.cpp)
