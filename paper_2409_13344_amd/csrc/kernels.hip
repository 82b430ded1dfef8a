// HIP kernels of the APPGA iteration for CDNA4 (gfx950).
//
// One APPGA iteration (Section 2.2, eq. APPGAiter with the closed-form prox
// max(., 0) and the gradients of Section 2.2) runs as two kernels:
//
//  forward  : y = A f~ + gamma and e = 1 - g / max(y, tau)      (grad F, first half)
//  step     : grad F = A^T e over the stored transpose, the SHOITV gradient
//             B1^T w1 B1 f~ + B2^T w2 B2 f~ from LDS tiles, the EM
//             preconditioner P = beta f^k / Lambda, f^{k+1} = max(f~ - P (grad F +
//             grad R), 0) and the next extrapolation f~^{k+1} = f^{k+1} +
//             theta_{k+1} (f^{k+1} - f^k) (eq. GNtheta)
//
// Layouts of per-solve vectors:
//  - B = 1: plain vectors.  The "single" kernels give each matrix row a group
//    of G lanes; each lane reads whole 8-entry chunks (16-byte index and value
//    loads) and the group reduces with cross-lane shuffles.
//  - B > 1: the lane layout.  Solves are grouped in chunks of 64 (one
//    wavefront); element i of solve b lives at ((b / 64) n + i) 64 + b % 64.
//    The "batch" kernels give each row one wave whose lanes are the 64 solves
//    of a chunk (blockIdx.y): a matrix entry is wave-uniform (scalar loads of a
//    precomputed byte offset col * 256 and of the value), and the gather of
//    x[col][0:64] is one buffer load with that offset in an SGPR, so a nonzero
//    costs one gather and one FMA.
// Matrix rows are padded with zero entries to multiples of 16 (kRowPad), so no
// kernel handles a ragged tail inside a row.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "appga_internal.h"

namespace appga {

// ------------------------------------------------------------------------
// Value decoding
// ------------------------------------------------------------------------

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ float f16_to_f32(uint32_t h) {
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(h)));
}

// OCP FP8 E4M3 (bias 7, no infinities): normal (1 + m/8) 2^(e-7), subnormal m 2^-9.
__device__ __forceinline__ float fp8_to_f32(uint32_t q) {
    const uint32_t s = (q & 0x80u) << 24;
    const uint32_t e = (q >> 3) & 0xFu;
    const uint32_t mm = q & 7u;
    if (e != 0) return __uint_as_float(s | ((e + 120u) << 23) | (mm << 20));
    const float v = static_cast<float>(mm) * 0.001953125f;
    return s ? -v : v;
}

template <typename IT>
__device__ __forceinline__ void load_cols8(const IT *__restrict__ col, int64_t k, uint32_t c[8]);

template <>
__device__ __forceinline__ void load_cols8<uint16_t>(const uint16_t *__restrict__ col, int64_t k,
                                                     uint32_t c[8]) {
    const uint4 w = *reinterpret_cast<const uint4 *>(col + k);
    c[0] = w.x & 0xFFFFu; c[1] = w.x >> 16;
    c[2] = w.y & 0xFFFFu; c[3] = w.y >> 16;
    c[4] = w.z & 0xFFFFu; c[5] = w.z >> 16;
    c[6] = w.w & 0xFFFFu; c[7] = w.w >> 16;
}

template <>
__device__ __forceinline__ void load_cols8<uint32_t>(const uint32_t *__restrict__ col, int64_t k,
                                                     uint32_t c[8]) {
    const uint4 a = *reinterpret_cast<const uint4 *>(col + k);
    const uint4 b = *reinterpret_cast<const uint4 *>(col + k + 4);
    c[0] = a.x; c[1] = a.y; c[2] = a.z; c[3] = a.w;
    c[4] = b.x; c[5] = b.y; c[6] = b.z; c[7] = b.w;
}

template <int VT>
__device__ __forceinline__ void load_vals8(const void *__restrict__ val, int64_t k, float v[8]) {
    if constexpr (VT == VT_F32) {
        const float4 a = *reinterpret_cast<const float4 *>(static_cast<const float *>(val) + k);
        const float4 b = *reinterpret_cast<const float4 *>(static_cast<const float *>(val) + k + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else if constexpr (VT == VT_BF16 || VT == VT_F16) {
        const uint4 w = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(val) + k);
        const uint32_t h[8] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu, w.y >> 16,
                               w.z & 0xFFFFu, w.z >> 16, w.w & 0xFFFFu, w.w >> 16};
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = (VT == VT_BF16) ? bf16_to_f32(h[t]) : f16_to_f32(h[t]);
    } else {
        const uint2 w = *reinterpret_cast<const uint2 *>(static_cast<const uint8_t *>(val) + k);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            v[t] = fp8_to_f32((w.x >> (8 * t)) & 0xFFu);
            v[t + 4] = fp8_to_f32((w.y >> (8 * t)) & 0xFFu);
        }
    }
}

// Floor of y = A x + gamma before the ratio: tau = 1e-6 gamma, or 1e-30 when gamma = 0.
__device__ __forceinline__ float y_floor(float gam) { return gam > 0.0f ? 1e-6f * gam : 1e-30f; }

// Buffer resource over `bytes` bytes at p (gfx9-family descriptor word 3).
// Loads through it are range-checked by the hardware (out of range reads 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), static_cast<short>(0),
                                             static_cast<int>(bytes), 0x00020000);
}

template <int VT>
__host__ __device__ constexpr uint32_t vbytes() {
    return VT == VT_F32 ? 4u : (VT == VT_FP8 ? 1u : 2u);
}

// 4-byte load at byte offset voff (per lane) + soff (wave-uniform, in an SGPR).
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// Index of element i of solve b in the lane layout of vectors of length n.
__device__ __forceinline__ size_t lidx(int i, int b, int n) {
    return (static_cast<size_t>(b >> 6) * n + i) * 64 + (b & 63);
}

// ------------------------------------------------------------------------
// Row dot products
// ------------------------------------------------------------------------

// Raw value bits of stored entry k + lane (one coalesced vector load per 64 entries).
template <int VT>
__device__ __forceinline__ uint32_t load_val_lane(__amdgpu_buffer_rsrc_t vr, int k) {
    const uint32_t lane = __lane_id();
    if constexpr (VT == VT_F32)
        return __builtin_amdgcn_raw_buffer_load_b32(vr, 4u * (static_cast<uint32_t>(k) + lane), 0, 0);
    else if constexpr (VT == VT_FP8)
        return __builtin_amdgcn_raw_buffer_load_b8(vr, static_cast<uint32_t>(k) + lane, 0, 0);
    else
        return __builtin_amdgcn_raw_buffer_load_b16(vr, 2u * (static_cast<uint32_t>(k) + lane), 0, 0);
}

template <int VT>
__device__ __forceinline__ float decode_val(uint32_t raw) {
    if constexpr (VT == VT_F32) return __uint_as_float(raw);
    else if constexpr (VT == VT_BF16) return bf16_to_f32(raw & 0xFFFFu);
    else if constexpr (VT == VT_F16) return f16_to_f32(raw & 0xFFFFu);
    else return fp8_to_f32(raw & 0xFFu);
}

// Lane-layout gather: sum_k val[k] * x[col[k]][lane] over the stored entries
// [k0, k1) of one wave-uniform row, entries in order.  The matrix holds the
// byte offset col * 256 of each entry's 64-lane record of x.  Each group of 64
// entries is read with one coalesced vector load per array (lane l holds entry
// k + l); v_readlane moves entry t into scalar registers, so a gather is one
// buffer load with a scalar offset and the product one FMA with a scalar
// operand.  The next group's loads are issued before the current gathers.
// Rows are padded to multiples of 16 entries; loads past the array end read 0.
template <int VT>
__device__ __forceinline__ float gather_dot_lanes64(__amdgpu_buffer_rsrc_t cr,
                                                    __amdgpu_buffer_rsrc_t vr,
                                                    __amdgpu_buffer_rsrc_t xr, int k0, int k1,
                                                    uint32_t voff) {
    float acc = 0.0f;
    const uint32_t lane = __lane_id();
    int k = k0;
    uint32_t vc = 0, vv = 0;
    if (k < k1) {
        vc = __builtin_amdgcn_raw_buffer_load_b32(cr, 4u * (static_cast<uint32_t>(k) + lane), 0, 0);
        vv = load_val_lane<VT>(vr, k);
    }
    while (k < k1) {
        const int n = k1 - k;   // multiple of 16
        const int kn = k + 64;
        uint32_t vc2 = 0, vv2 = 0;
        if (kn < k1) {
            vc2 = __builtin_amdgcn_raw_buffer_load_b32(cr, 4u * (static_cast<uint32_t>(kn) + lane), 0, 0);
            vv2 = load_val_lane<VT>(vr, kn);
        }
#pragma unroll
        for (int t0 = 0; t0 < 64; t0 += 16) {
            if (t0 < n) {
                float x[16];
                uint32_t sv[16];
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const uint32_t sc = __builtin_amdgcn_readlane(vc, t0 + t);
                    sv[t] = __builtin_amdgcn_readlane(vv, t0 + t);
                    x[t] = buf_load(xr, voff, sc);
                }
#pragma unroll
                for (int t = 0; t < 16; ++t) acc = fmaf(decode_val<VT>(sv[t]), x[t], acc);
            }
        }
        vc = vc2;
        vv = vv2;
        k = kn;
    }
    return acc;
}

// B = 1: partial dot product of lane gl of a G-lane group over the stored
// entries [k0, k1): lane gl takes chunks gl, gl + G, ...; the gather offset is
// per lane.
// Two chunks per round trip (their index and value loads issued together, then
// their 16 gathers), so that each lane has twice the loads in flight; the
// products are added in chunk order.
template <typename IT, int VT, int G>
__device__ __forceinline__ float gather_dot_group(const IT *__restrict__ col,
                                                  const void *__restrict__ val,
                                                  __amdgpu_buffer_rsrc_t xr, int k0, int k1,
                                                  int gl, int rot_n = 0) {
    // rot_n > 0: gather x at rho(col), rho(r, c) = (c, N - 1 - r) for N = rot_n.
    // r = floor((col + 1/2) / N) in FP32 is exact: the quotient sits at least 1/(2N)
    // from an integer and col < 2^16.  Padding entries (col 0, value 0) stay in range.
    const float inv_n = rot_n > 0 ? 1.0f / static_cast<float>(rot_n) : 0.0f;
    auto rot = [&](uint32_t c) -> uint32_t {
        if (rot_n <= 0) return c;
        const uint32_t r = static_cast<uint32_t>((static_cast<float>(c) + 0.5f) * inv_n);
        const uint32_t cc = c - r * static_cast<uint32_t>(rot_n);
        return cc * static_cast<uint32_t>(rot_n) + (static_cast<uint32_t>(rot_n) - 1u - r);
    };
    float acc = 0.0f;
    int k = k0 + gl * kChunk;
    for (; k + G * kChunk < k1; k += 2 * G * kChunk) {
        uint32_t c[16];
        float v[16], xv[16];
        load_cols8<IT>(col, k, c);
        load_cols8<IT>(col, k + G * kChunk, c + 8);
        load_vals8<VT>(val, k, v);
        load_vals8<VT>(val, k + G * kChunk, v + 8);
#pragma unroll
        for (int t = 0; t < 16; ++t) xv[t] = buf_load(xr, 4u * rot(c[t]), 0u);
#pragma unroll
        for (int t = 0; t < 16; ++t) acc = fmaf(v[t], xv[t], acc);
    }
    if (k < k1) {
        uint32_t c[8];
        float v[8], xv[8];
        load_cols8<IT>(col, k, c);
        load_vals8<VT>(val, k, v);
#pragma unroll
        for (int t = 0; t < 8; ++t) xv[t] = buf_load(xr, 4u * rot(c[t]), 0u);
#pragma unroll
        for (int t = 0; t < 8; ++t) acc = fmaf(v[t], xv[t], acc);
    }
    return acc;
}

// ------------------------------------------------------------------------
// Forward projection + Poisson ratio
// ------------------------------------------------------------------------

// Epilogue for row `row`, solve b, at vector index o; y = acc + gamma.
template <int VT>
__device__ __forceinline__ void fwd_epilogue(const FwdArgs &a, int row, int b, size_t o, float acc,
                                             float gam, bool count) {
    if constexpr (VT == VT_FP8) acc *= a.row_scale[row];
    float y = acc + gam;
    if (a.mode == FM_PROJ) {
        a.out[o] = y;
        return;
    }
    const float tau = y_floor(gam);
    if (y < tau) {
        y = tau;
        if (count && a.clamps) atomicAdd(a.clamps + b, 1ull);
    }
    float ev = 1.0f - a.g[o] / y;
    if constexpr (VT == VT_FP8) {
        if (a.scale_out) ev *= a.row_scale[row];
    }
    a.out[o] = ev;
}

// B = 1: G lanes per row, 256 / G rows per workgroup.
template <typename IT, int VT, int G>
__global__ __launch_bounds__(256) void k_fwd_single(FwdArgs a) {
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int row = blockIdx.x * (256 / G) + threadIdx.x / G;
    const IT *__restrict__ col = static_cast<const IT *>(a.col);
    const auto xr = make_rsrc(a.x, 4u * static_cast<uint32_t>(a.n_x));
    float acc = 0.0f;
    if (row < a.m) {
        // half-stored matrix: the second half of the rows are the first half turned by 90 degrees
        const bool turned = a.sym_half > 0 && row >= a.sym_half;
        const int srow = turned ? row - a.sym_half : row;
        acc = gather_dot_group<IT, VT, G>(col, a.val, xr, a.row_ptr[srow], a.row_ptr[srow + 1], gl,
                                          turned ? a.img_n : 0);
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (row < a.m && gl == 0) {
        const float gam = a.gamma ? a.gamma[row] : (a.gamma_lane ? a.gamma_lane[0] : 0.0f);
        fwd_epilogue<VT>(a, row, 0, row, acc, gam, true);
    }
}

// B > 1: one wave per row at a time, lanes = the 64 solves of chunk
// blockIdx.y; waves stride over the rows (the grid holds about one wave per
// wave slot of the device, so per-wave set-up is paid once, not per row).
template <int VT>
__global__ __launch_bounds__(256) void k_fwd_batch(FwdArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int nwaves = gridDim.x * 4;
    const int chunk = blockIdx.y;
    const int b = chunk * 64 + lane;
    const auto xr = make_rsrc(reinterpret_cast<const char *>(a.x) + static_cast<size_t>(chunk) * a.n_x * 256,
                              256u * static_cast<uint32_t>(a.n_x));
    const float gl = a.gamma_lane ? a.gamma_lane[b] : 0.0f;
    const auto cr = make_rsrc(a.col32, 4u * static_cast<uint32_t>(a.nnz_padded));
    const auto vr = make_rsrc(a.val, static_cast<uint32_t>(a.nnz_padded) * vbytes<VT>());
    for (int row = wave; row < a.m; row += nwaves) {
        const int k0 = a.row_ptr[row], k1 = a.row_ptr[row + 1];
        const float acc = gather_dot_lanes64<VT>(cr, vr, xr, k0, k1, 4u * lane);
        const size_t o = (static_cast<size_t>(chunk) * a.m + row) * 64 + lane;
        const float gam = a.gamma ? a.gamma[o] : gl;
        fwd_epilogue<VT>(a, row, b, o, acc, gam, b < a.B);
    }
}

// ------------------------------------------------------------------------
// SHOITV gradient (Section 2.1 operators, Section 2.2 gradient).
//
// With image index j = r*N + c, X (x) Y acts as X along r and Y along c, and
// (Dx)_c = [c>=1](x_c - x_{c-1}), (D^T y)_c = [c>=1] y_c - [c<=N-2] y_{c+1},
// L = -D^T D: (Lx)_c = [c<=N-2](x_{c+1} - x_c) + [c>=1](x_{c-1} - x_c).
//   u1 = (I(x)D)f, u2 = (D(x)I)f, v1 = (I(x)L)f, v2 = (-D^T(x)D)f,
//   v3 = (L(x)I)f, v4 = (D(x)-D^T)f,
// weights w1 = lambda1 / max(|u|, eps), w2 = lambda2 / max(|v|, eps), and
//   grad R = (I(x)D^T)(w1 u1) + (D^T(x)I)(w1 u2) + (I(x)L)(w2 v1)
//          + (-D(x)D^T)(w2 v2) + (L(x)I)(w2 v3) + (D^T(x)-D)(w2 v4).
// grad R at (r, c) needs the weighted vectors at (r, c) and six neighbours
// within one pixel, which need f within a radius of 2.  A 4 x 4 tile needs
// the weighted vectors on the 6 x 6 block around it (computed once each, kept
// in LDS) and f on the 8 x 8 block around it.
// ------------------------------------------------------------------------

// The six components at (r, c) (0 <= r, c < N); F(r, c) reads the image.  IN
// asserts that (r, c) is at least one pixel away from every edge, which makes
// every boundary condition true at compile time.
template <bool IN = false, typename Fn>
__device__ __forceinline__ void uv6(const Fn &F, int r, int c, int N, float o[6]) {
    const float f00 = F(r, c);
    const bool cl = IN || c >= 1, cr = IN || c <= N - 2, ru = IN || r >= 1, rd = IN || r <= N - 2;
    const float fl = cl ? F(r, c - 1) : 0.0f;
    const float fr = cr ? F(r, c + 1) : 0.0f;
    const float fu = ru ? F(r - 1, c) : 0.0f;
    const float fd = rd ? F(r + 1, c) : 0.0f;
    const float u1 = cl ? f00 - fl : 0.0f;
    const float u2 = ru ? f00 - fu : 0.0f;
    const float v1 = (cr ? fr - f00 : 0.0f) + (cl ? fl - f00 : 0.0f);
    const float u1d = (rd && cl) ? fd - F(r + 1, c - 1) : 0.0f;   // u1 at (r+1, c)
    const float v2 = (rd ? u1d : 0.0f) - (ru ? u1 : 0.0f);
    const float v3 = (rd ? fd - f00 : 0.0f) + (ru ? fu - f00 : 0.0f);
    float v4 = 0.0f;
    if (ru) {
        const float w0 = (cr ? fr : 0.0f) - (cl ? f00 : 0.0f);
        const float w1 = (cr ? F(r - 1, c + 1) : 0.0f) - (cl ? fu : 0.0f);
        v4 = w0 - w1;
    }
    o[0] = u1; o[1] = u2; o[2] = v1; o[3] = v2; o[4] = v3; o[5] = v4;
}

// Weighted vector (w1 u1, w1 u2, w2 v1..v4) at (r, c).
template <bool IN = false, typename Fn>
__device__ __forceinline__ void pq6(const Fn &F, int r, int c, int N, float l1, float l2, float eps,
                                    float o[6]) {
    uv6<IN>(F, r, c, N, o);
    const float n1 = sqrtf(o[0] * o[0] + o[1] * o[1]);
    const float n2 = sqrtf(o[2] * o[2] + o[3] * o[3] + o[4] * o[4] + o[5] * o[5]);
    const float w1 = l1 / fmaxf(n1, eps);
    const float w2 = l2 / fmaxf(n2, eps);
    o[0] *= w1; o[1] *= w1;
    o[2] *= w2; o[3] *= w2; o[4] *= w2; o[5] *= w2;
}

// grad R at (r, c) from the weighted vectors; Q(dr, dc, k) reads component k
// at (r + dr, c + dc) (only in-image positions are read); IN as for uv6.
template <bool IN = false, typename Qf>
__device__ __forceinline__ float combine_grad(const Qf &Q, int r, int c, int N) {
    const bool cl = IN || c >= 1, cr = IN || c <= N - 2, ru = IN || r >= 1, rd = IN || r <= N - 2;
    // (I (x) D^T) p1 and (D^T (x) I) p2
    float g = (cl ? Q(0, 0, 0) : 0.0f) - (cr ? Q(0, 1, 0) : 0.0f);
    g += (ru ? Q(0, 0, 1) : 0.0f) - (rd ? Q(1, 0, 1) : 0.0f);
    // (I (x) L) q1
    g += (cr ? Q(0, 1, 2) - Q(0, 0, 2) : 0.0f) + (cl ? Q(0, -1, 2) - Q(0, 0, 2) : 0.0f);
    // (-D (x) D^T) q2: t(r') = [c>=1] q2(r', c) - [c<=N-2] q2(r', c+1); -[r>=1](t(r) - t(r-1))
    if (ru) {
        const float t0 = (cl ? Q(0, 0, 3) : 0.0f) - (cr ? Q(0, 1, 3) : 0.0f);
        const float t1 = (cl ? Q(-1, 0, 3) : 0.0f) - (cr ? Q(-1, 1, 3) : 0.0f);
        g -= t0 - t1;
    }
    // (L (x) I) q3
    g += (rd ? Q(1, 0, 4) - Q(0, 0, 4) : 0.0f) + (ru ? Q(-1, 0, 4) - Q(0, 0, 4) : 0.0f);
    // (D^T (x) -D) q4: s(r') = -[c>=1](q4(r', c) - q4(r', c-1)); [r>=1] s(r) - [r<=N-2] s(r+1)
    if (cl) {
        const float s0 = -(Q(0, 0, 5) - Q(0, -1, 5));
        const float s1 = rd ? -(Q(1, 0, 5) - Q(1, -1, 5)) : 0.0f;
        g += (ru ? s0 : 0.0f) - s1;
    }
    return g;
}

// Preconditioner value for one pixel/solve (stores it in frozen-update mode).
__device__ __forceinline__ float precond(int pmode, float fk, float lam, const LaneParams &lp,
                                         float *pbuf, size_t o) {
    float P;
    if (pmode == PM_FIXED) {
        P = lp.fixed_p;
    } else if (pmode == PM_STORED) {
        P = pbuf[o];
    } else {
        P = lp.beta * fk / lam;
        if (pmode == PM_EM_STORE) pbuf[o] = P;
    }
    return P;
}

// Maps a workgroup to a tile.  With xcd_remap, workgroups are assumed to be
// dealt round-robin to the 8 XCDs (workgroup w runs on XCD w % 8), and the
// tiles of each XCD form one compact block of the image (2 x 4 blocks), so the
// rays its back projections gather stay in that XCD's L2.
__device__ __forceinline__ int tile_of(int wg, int tiles_x, int tiles_y, int remap) {
    if (!remap) return wg;
    const int bw = tiles_x / 4, bh = tiles_y / 2;
    const int xcd = wg & 7, slot = wg >> 3;
    const int br = xcd >> 2, bc = xcd & 3;
    const int ty = br * bh + slot / bw, tx = bc * bw + slot % bw;
    return ty * tiles_x + tx;
}

// ------------------------------------------------------------------------
// Step kernel, B = 1.  Tile of 4 x 4 pixels per workgroup of 16 G threads:
// lane group p (G lanes) back-projects pixel p; 36 threads compute the
// weighted vectors on the 6 x 6 block from the 8 x 8 halo of f~ in LDS;
// 16 threads combine them and apply the update.
// ------------------------------------------------------------------------

template <typename IT, int VT, int G>
__global__ __launch_bounds__(16 * G) void k_step_single(StepArgs a) {
    __shared__ float halo[64];
    __shared__ float pqs[6][36];
    __shared__ float gfs[16];
    const int tid = threadIdx.x;
    const int gl = tid & (G - 1);
    const int p = tid / G;
    const int N = a.n;
    const int tiles_x = a.tiles_x, tiles_y = (N + 3) / 4;
    const int tile = tile_of(blockIdx.x, tiles_x, tiles_y, a.xcd_remap);
    const int r0 = (tile / tiles_x) * 4, c0 = (tile % tiles_x) * 4;
    const IT *__restrict__ col = static_cast<const IT *>(a.col);

    if (a.out_mode != SO_REG) {
        const int rp = r0 + (p >> 2), cp = c0 + (p & 3);
        float acc = 0.0f;
        if (rp < N && cp < N) {
            const int j = rp * N + cp;
            if (a.gf_in) {   // A^T e given (one partial sum): the group's first lane carries it
                acc = gl == 0 ? a.gf_in[j] : 0.0f;
            } else {
                const auto er = make_rsrc(a.e, 4u * static_cast<uint32_t>(a.m));
                acc = gather_dot_group<IT, VT, G>(col, a.val, er, a.row_ptr[j], a.row_ptr[j + 1], gl);
                if (a.sym_half > 0) {
                    // the turned rays i + sym_half meet pixel j where ray i meets rho^{-1}(j)
                    const int jr = (N - 1 - cp) * N + rp;
                    const auto er2 = make_rsrc(a.e + a.sym_half, 4u * static_cast<uint32_t>(a.m - a.sym_half));
                    acc += gather_dot_group<IT, VT, G>(col, a.val, er2, a.row_ptr[jr], a.row_ptr[jr + 1], gl);
                }
            }
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (gl == 0) gfs[p] = acc;
    }
    if (tid < 64) {
        const int hr = r0 - 2 + (tid >> 3), hc = c0 - 2 + (tid & 7);
        halo[tid] = (hr >= 0 && hr < N && hc >= 0 && hc < N) ? a.ft[hr * N + hc] : 0.0f;
    }
    __syncthreads();
    const LaneParams lp = a.lp[0];
    auto F = [&](int rr, int cc) { return halo[(rr - r0 + 2) * 8 + (cc - c0 + 2)]; };
    if (tid < 36) {
        const int rr = r0 - 1 + tid / 6, cc = c0 - 1 + tid % 6;
        float o[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (rr >= 0 && rr < N && cc >= 0 && cc < N) pq6(F, rr, cc, N, lp.lambda1, lp.lambda2, lp.eps, o);
#pragma unroll
        for (int k = 0; k < 6; ++k) pqs[k][tid] = o[k];
    }
    __syncthreads();
    if (tid >= 16) return;
    const int r = r0 + (tid >> 2), c = c0 + (tid & 3);
    const bool in = r < N && c < N;
    double dd = 0.0, nn = 0.0;
    if (in) {
        const int j = r * N + c;
        auto Q = [&](int dr, int dc, int k) { return pqs[k][(r - r0 + 1 + dr) * 6 + (c - c0 + 1 + dc)]; };
        if (a.out_mode == SO_BACK) {
            a.out[j] = gfs[tid];
        } else {
            const float gR = combine_grad(Q, r, c, N);
            if (a.out_mode == SO_REG) {
                a.out[j] = gR;
            } else {
                const float ftc = F(r, c);
                const float fk = a.f[j];
                const float P = precond(a.pmode, fk, a.lam[j], lp, a.pbuf, j);
                const float z = ftc - P * (gfs[tid] + gR);
                const float fn = z > 0.0f ? z : 0.0f;
                a.f[j] = fn;
                a.ft_next[j] = fn + a.theta_next[0] * (fn - fk);
                const double df = static_cast<double>(fn) - static_cast<double>(fk);
                dd = df * df;
                nn = static_cast<double>(fn) * static_cast<double>(fn);
            }
        }
    }
    if (a.re_part) {
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            dd += __shfl_xor(dd, off, 64);
            nn += __shfl_xor(nn, off, 64);
        }
        if (tid == 0) {
            a.re_part[2 * blockIdx.x] = dd;
            a.re_part[2 * blockIdx.x + 1] = nn;
        }
    }
}

// ------------------------------------------------------------------------
// Step kernel, B > 1 (lane layout).  Tile of 4 x 4 pixels per workgroup of 16
// waves, lanes = the 64 solves of chunk blockIdx.y: wave w back-projects pixel
// w; the 8 x 8 halo of f~ is staged in LDS; the 36 weighted vectors of the
// 6 x 6 block are computed once (waves 0..15 take positions w, w+16, w+32) and
// kept in LDS; wave w combines them for pixel w and applies the update.  Tiles
// whose halo lies inside the image (all but the outer ring) take a copy of the
// stencil code with the boundary conditions removed at compile time.
// ------------------------------------------------------------------------

template <int VT>
__global__ __launch_bounds__(1024, 8) void k_step_batch(StepArgs a) {
    __shared__ float halo[64][64];      // reused for the RE partial sums at the end
    __shared__ float pqs[6][36][64];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int N = a.n;
    const int d = N * N;
    const int chunk = blockIdx.y;
    const int b = chunk * 64 + lane;
    const bool act = b < a.B;
    const int tiles_x = a.tiles_x, tiles_y = (N + 3) / 4;
    const int tile = tile_of(blockIdx.x, tiles_x, tiles_y, a.xcd_remap);
    const int r0 = (tile / tiles_x) * 4, c0 = (tile % tiles_x) * 4;
    const int r = r0 + (w >> 2), c = c0 + (w & 3);
    const bool in = r < N && c < N;
    const size_t vbase = static_cast<size_t>(chunk) * d * 64 + lane;

    float gF = 0.0f;
    // values of the update, loaded before the halo so their latency overlaps it
    const bool upd = in && a.out_mode == SO_STEP;
    const float fk = upd ? a.f[vbase + static_cast<size_t>(r * N + c) * 64] : 0.0f;
    const float lamj = upd ? a.lam[r * N + c] : 1.0f;
    if (a.gf_in) {
        if (in) {
            const size_t o = vbase + static_cast<size_t>(r * N + c) * 64;
            const size_t stride = static_cast<size_t>(a.Bp) * d;
            for (int q = 0; q < a.gf_split; ++q) gF += a.gf_in[q * stride + o];
        }
    } else if (a.out_mode != SO_REG && in) {
        const int j = r * N + c;
        const auto er = make_rsrc(reinterpret_cast<const char *>(a.e) + static_cast<size_t>(chunk) * a.m * 256,
                                  256u * static_cast<uint32_t>(a.m));
        const auto cr = make_rsrc(a.col32, 4u * static_cast<uint32_t>(a.nnz_padded));
        const auto vr = make_rsrc(a.val, static_cast<uint32_t>(a.nnz_padded) * vbytes<VT>());
        gF = gather_dot_lanes64<VT>(cr, vr, er, a.row_ptr[j], a.row_ptr[j + 1], 4u * lane);
    }
    // the 8 x 8 halo inside the image: every stencil position of the tile is interior
    const bool interior = r0 >= 2 && c0 >= 2 && r0 + 6 <= N && c0 + 6 <= N;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int q = w + 16 * k;
        const int hr = r0 - 2 + (q >> 3), hc = c0 - 2 + (q & 7);
        halo[q][lane] = (interior || (hr >= 0 && hr < N && hc >= 0 && hc < N))
                            ? a.ft[vbase + static_cast<size_t>(hr * N + hc) * 64]
                            : 0.0f;
    }
    __syncthreads();
    const LaneParams lp = a.lp[b];
    auto F = [&](int rr, int cc) { return halo[(rr - r0 + 2) * 8 + (cc - c0 + 2)][lane]; };
    auto weighted = [&](auto in_tag) {
        constexpr bool IN = decltype(in_tag)::value;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int q = w + 16 * k;
            if (q >= 36) break;
            const int rr = r0 - 1 + q / 6, cc = c0 - 1 + q % 6;
            float o[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (IN || (rr >= 0 && rr < N && cc >= 0 && cc < N))
                pq6<IN>(F, rr, cc, N, lp.lambda1, lp.lambda2, lp.eps, o);
#pragma unroll
            for (int t = 0; t < 6; ++t) pqs[t][q][lane] = o[t];
        }
    };
    if (interior) {
        weighted(std::true_type{});
    } else {
        weighted(std::false_type{});
    }
    __syncthreads();
    const float ftc = in ? F(r, c) : 0.0f;
    double dd = 0.0, nn = 0.0;
    if (in) {
        const size_t o = vbase + static_cast<size_t>(r * N + c) * 64;
        auto Q = [&](int dr, int dc, int k) {
            return pqs[k][(r - r0 + 1 + dr) * 6 + (c - c0 + 1 + dc)][lane];
        };
        if (a.out_mode == SO_BACK) {
            a.out[o] = gF;
        } else {
            const float gR = interior ? combine_grad<true>(Q, r, c, N) : combine_grad(Q, r, c, N);
            if (a.out_mode == SO_REG) {
                a.out[o] = gR;
            } else {
                const float th = a.theta_next[b];
                const float P = precond(a.pmode, fk, lamj, lp, a.pbuf, o);
                const float z = ftc - P * (gF + gR);
                const float fn = z > 0.0f ? z : 0.0f;
                a.f[o] = fn;
                a.ft_next[o] = fn + th * (fn - fk);
                const double df = static_cast<double>(fn) - static_cast<double>(fk);
                dd = df * df;
                nn = static_cast<double>(fn) * static_cast<double>(fn);
            }
        }
    }
    if (a.re_part) {
        double *red = reinterpret_cast<double *>(&halo[0][0]);   // [16][64][2]
        __syncthreads();                                          // halo no longer read
        red[(w * 64 + lane) * 2] = dd;
        red[(w * 64 + lane) * 2 + 1] = nn;
        __syncthreads();
        if (w < 2 && act) {   // wave 0 sums |f^{k+1} - f^k|^2, wave 1 |f^{k+1}|^2
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) s += red[(q * 64 + lane) * 2 + w];
            a.re_part[(static_cast<size_t>(blockIdx.x) * a.Bp + b) * 2 + w] = s;
        }
    }
}

// ------------------------------------------------------------------------
// AFPPA on the nonsmooth HOITV model (Section 4.3).  With the gradient of the
// fidelity at f~^k in hand (ratio forward projection, back projection):
//   primal  f^{k+1} = max(f~ - P (grad F(f~) + B1^T b~ + B2^T c~), 0),
//           w = 2 f^{k+1} - f~, f~^{k+1} = f^{k+1} + theta_{k+1} (f^{k+1} - f^k),
//           and the max over pixels of P = beta f^k / Lambda per solve;
//   dual    rho1 = 1 / (2 * 8 * p_max), rho2 = 1 / (2 * 64 * p_max);
//           b^{k+1} = rho1 (I - prox_{(lambda1/rho1)||.||})(b~ / rho1 + B1 w) per pixel
//           group of 2 components, c^{k+1} likewise with rho2, lambda2 and the 4
//           components of B2; b~^{k+1} = b^{k+1} + theta_{k+1} (b^{k+1} - b^k), c~ likewise.
// With z' = b~ / rho + B1 w, (I - prox_{t||.||})(z') = z' min(1, t / ||z'||), so
// b^{k+1} = z' min(rho, lambda / ||z'||): the dual kernel forms z' and this
// scale, which stay finite when p_max is tiny (rho huge; an image driven to 0
// by the EM preconditioner), where b~ + rho B1 w would overflow FP32.  For
// Bp == 1 a thread is a pixel (a wave covers 64); else a wave takes kAfppaPix
// pixels in turn, its lanes the 64 solves of a chunk, and issues the loads of
// all of them before the updates.  The
// stencils are those of the smoothed model's kernels: uv6 gives (B1 w, B2 w)
// at a pixel, combine_grad (here in its select-only form) gives B1^T p + B2^T q
// from the 6 components around it.
// ------------------------------------------------------------------------

// B1^T p + B2^T q at (r, c) as combine_grad computes it, written with selects
// only: Q must read values already in registers (every (dr, dc, k) it names
// is evaluated), so no load is moved into a branch and all of them can be in
// flight together.
template <typename Qf>
__device__ __forceinline__ float combine_grad_sel(const Qf &Q, int r, int c, int N) {
    const bool cl = c >= 1, cr = c <= N - 2, ru = r >= 1, rd = r <= N - 2;
    float g = (cl ? Q(0, 0, 0) : 0.0f) - (cr ? Q(0, 1, 0) : 0.0f);
    g += (ru ? Q(0, 0, 1) : 0.0f) - (rd ? Q(1, 0, 1) : 0.0f);
    g += (cr ? Q(0, 1, 2) - Q(0, 0, 2) : 0.0f) + (cl ? Q(0, -1, 2) - Q(0, 0, 2) : 0.0f);
    const float t0 = (cl ? Q(0, 0, 3) : 0.0f) - (cr ? Q(0, 1, 3) : 0.0f);
    const float t1 = (cl ? Q(-1, 0, 3) : 0.0f) - (cr ? Q(-1, 1, 3) : 0.0f);
    g -= ru ? t0 - t1 : 0.0f;
    g += (rd ? Q(1, 0, 4) - Q(0, 0, 4) : 0.0f) + (ru ? Q(-1, 0, 4) - Q(0, 0, 4) : 0.0f);
    const float s0 = -(Q(0, 0, 5) - Q(0, -1, 5));
    const float s1 = rd ? -(Q(1, 0, 5) - Q(1, -1, 5)) : 0.0f;
    g += cl ? (ru ? s0 : 0.0f) - s1 : 0.0f;
    return g;
}

template <bool LANES>
struct AfppaIdx {
    int d, b;
    __device__ __forceinline__ size_t px(int j) const {        // element j of a d-vector
        return LANES ? lidx(j, b, d) : static_cast<size_t>(j);
    }
    __device__ __forceinline__ size_t dual(int k, int j) const {  // component k at pixel j
        return LANES ? lidx(k * d + j, b, 6 * d) : static_cast<size_t>(k) * d + j;
    }
};

constexpr int kAfppaThreads = 256;
constexpr int kAfppaPix = 4;   // pixels per wave in the lane layout (their loads in flight together)

// SPLIT: the number of partial sums of A^T e (1 or 2, compile-time; 0 = a.gf_split)
template <bool LANES, int SPLIT>
__global__ __launch_bounds__(kAfppaThreads) void k_afppa_primal(AfppaArgs a) {
    constexpr int kWaves = kAfppaThreads / 64;
    constexpr int NP = LANES ? kAfppaPix : 1;
    __shared__ float pmr[kWaves][64];
    __shared__ double rer[kWaves][64][2];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int N = a.n, d = N * N;
    const int j0 = LANES ? (blockIdx.x * kWaves + w) * NP : blockIdx.x * kAfppaThreads + tid;
    const int b = LANES ? blockIdx.y * 64 + lane : 0;
    const AfppaIdx<LANES> ix{d, b};
    const LaneParams lp = a.lp[b];
    const float th = a.theta_next[b];
    const size_t stride = static_cast<size_t>(a.Bp) * d;
    // loads of all NP pixels first, then the updates
    // (pixels past the end of the image load pixel d - 1 and store nothing)
    float fk[NP], ftc[NP], gF[NP], gD[NP], lam[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int j = min(j0 + p, d - 1);
        {
            const int r = j / N, c = j - r * N;
            const size_t o = ix.px(j);
            fk[p] = a.f[o];
            ftc[p] = a.ft[o];
            gF[p] = a.gf[o];
            if (SPLIT == 2) gF[p] += a.gf[stride + o];
            if (SPLIT == 0)
                for (int q = 1; q < a.gf_split; ++q) gF[p] += a.gf[q * stride + o];
            // the 3 x 3 neighbourhood of each component, loaded without branches at
            // indices clamped into the image (combine_grad only uses in-image
            // values; the loads it does not use are dropped by the compiler)
            float v[6][3][3];
            const int rr[3] = {max(r - 1, 0), r, min(r + 1, N - 1)};
            const int cc[3] = {max(c - 1, 0), c, min(c + 1, N - 1)};
#pragma unroll
            for (int k = 0; k < 6; ++k)
#pragma unroll
                for (int u = 0; u < 3; ++u)
#pragma unroll
                    for (int t = 0; t < 3; ++t) v[k][u][t] = a.ybar[ix.dual(k, rr[u] * N + cc[t])];
            auto Q = [&](int dr, int dc, int k) { return v[k][dr + 1][dc + 1]; };
            gD[p] = combine_grad_sel(Q, r, c, N);
            lam[p] = a.lam[j];
        }
    }
    float Pk = 0.0f;
    double dd = 0.0, nn = 0.0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int j = j0 + p;
        if (j >= d) continue;
        const size_t o = ix.px(j);
        const float P = a.pmode == PM_FIXED ? lp.fixed_p : lp.beta * fk[p] / lam[p];
        const float z = ftc[p] - P * (gF[p] + gD[p]);
        const float fn = z > 0.0f ? z : 0.0f;
        a.f[o] = fn;
        a.w[o] = 2.0f * fn - ftc[p];
        a.ft_next[o] = fn + th * (fn - fk[p]);
        Pk = fmaxf(Pk, fmaxf(P, 0.0f));
        const double df = static_cast<double>(fn) - static_cast<double>(fk[p]);
        dd += df * df;
        nn += static_cast<double>(fn) * static_cast<double>(fn);
    }
    if (!LANES) {   // one solve: reduce over the 64 pixels of the wave first
        for (int sh = 32; sh >= 1; sh >>= 1) {
            Pk = fmaxf(Pk, __shfl_xor(Pk, sh));
            dd += __shfl_xor(dd, sh);
            nn += __shfl_xor(nn, sh);
        }
    }
    pmr[w][lane] = Pk;
    rer[w][lane][0] = dd;
    rer[w][lane][1] = nn;
    __syncthreads();
    if (w == 0 && (LANES || lane == 0)) {
        float m = 0.0f;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            m = fmaxf(m, pmr[q][lane]);
            s0 += rer[q][lane][0];
            s1 += rer[q][lane][1];
        }
        // one of kAfppaPmSlots accumulators per solve (by workgroup), so that the
        // atomics of all workgroups do not queue on one cache line
        if (a.pmode != PM_FIXED)
            atomicMax(&a.pmax_acc[static_cast<size_t>(blockIdx.x % kAfppaPmSlots) * a.Bp + b], __float_as_uint(m));
        if (a.re_part) {
            const size_t po = (static_cast<size_t>(blockIdx.x) * a.Bp + b) * 2;
            a.re_part[po] = s0;
            a.re_part[po + 1] = s1;
        }
    }
}

template <bool LANES>
__global__ __launch_bounds__(kAfppaThreads) void k_afppa_dual(AfppaArgs a) {
    constexpr int kWaves = kAfppaThreads / 64;
    constexpr int NP = LANES ? kAfppaPix : 1;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int N = a.n, d = N * N;
    const int j0 = LANES ? (blockIdx.x * kWaves + w) * NP : blockIdx.x * kAfppaThreads + tid;
    const int b = LANES ? blockIdx.y * 64 + lane : 0;
    // the next iteration's max accumulators start from 0 (their last reader, the
    // dual kernel two iterations back, has finished)
    if (blockIdx.x == 0 && (LANES ? w == 0 : tid == 0) && a.pmax_clear)
        for (int q = 0; q < kAfppaPmSlots; ++q) a.pmax_clear[static_cast<size_t>(q) * a.Bp + b] = 0u;
    const AfppaIdx<LANES> ix{d, b};
    const LaneParams lp = a.lp[b];
    const float th = a.theta_next[b];
    // p_max of each solve: the first wave reduces the slots, the others read it from LDS
    __shared__ float pm_lds[64];
    if (w == 0) {
        float pmx = 0.0f;
        if (a.pmode != PM_FIXED)
            for (int q = 0; q < kAfppaPmSlots; ++q)
                pmx = fmaxf(pmx, __uint_as_float(a.pmax_in[static_cast<size_t>(q) * a.Bp + b]));
        pm_lds[lane] = pmx;
    }
    __syncthreads();
    const float pm = fmaxf(a.pmode == PM_FIXED ? lp.fixed_p : pm_lds[LANES ? lane : 0], 1e-30f);
    const float irho1 = 16.0f * pm, irho2 = 128.0f * pm;   // 1 / rho1, 1 / rho2
    // loads of all NP pixels first: z' = ybar / rho + (B1 w, B2 w), and the duals y^k
    // (pixels past the end of the image load pixel d - 1 and store nothing)
    float z[NP][6], yo[NP][6];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int j = min(j0 + p, d - 1);
        {
            const int r = j / N, c = j - r * N;
            // the 3 x 3 neighbourhood of w without branches (clamped indices; uv6
            // only uses in-image values)
            float wv[3][3];
            const int rr[3] = {max(r - 1, 0), r, min(r + 1, N - 1)};
            const int cc[3] = {max(c - 1, 0), c, min(c + 1, N - 1)};
#pragma unroll
            for (int u = 0; u < 3; ++u)
#pragma unroll
                for (int t = 0; t < 3; ++t) wv[u][t] = a.w[ix.px(rr[u] * N + cc[t])];
            auto W = [&](int r2, int c2) { return wv[r2 - r + 1][c2 - c + 1]; };
            float u[6];
            uv6(W, r, c, N, u);
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                z[p][k] = a.ybar[ix.dual(k, j)] * (k < 2 ? irho1 : irho2) + u[k];
                yo[p][k] = a.y[ix.dual(k, j)];
            }
        }
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int j = j0 + p;
        if (j >= d) continue;
        const float n1 = sqrtf(z[p][0] * z[p][0] + z[p][1] * z[p][1]);
        const float n2 = sqrtf(z[p][2] * z[p][2] + z[p][3] * z[p][3] + z[p][4] * z[p][4] + z[p][5] * z[p][5]);
        // min(rho, lambda / ||z'||), compared as ||z'|| > lambda / rho
        const float s1 = n1 > lp.lambda1 * irho1 ? lp.lambda1 / n1 : 1.0f / irho1;
        const float s2 = n2 > lp.lambda2 * irho2 ? lp.lambda2 / n2 : 1.0f / irho2;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const size_t o = ix.dual(k, j);
            const float yn = z[p][k] * (k < 2 ? s1 : s2);
            a.y[o] = yn;
            a.ybar[o] = yn + th * (yn - yo[p][k]);
        }
    }
}

// ------------------------------------------------------------------------
// Projections for B > 1 over tiles (Section 2.2: grad F = A^T e needs A x
// and A^T e every iteration).
//
// A row-by-row kernel gathers, for every stored entry, the 256-byte lane
// record of its input from L2, and that gather rate is what bounds it.  Here
// a workgroup owns a tile of 64 outputs and stages in LDS, window after
// window, the input records its entries refer to; each staged record serves
// several entries (about 8 for the back projection, whose windows are the
// rays that cross an 8 x 8 pixel tile at a group of consecutive angles, about
// 6.6 for the forward projection, whose windows are runs of the pixels that
// a block of 8 angles x 8 bins of rays crosses).  LDS serves 16-byte reads
// about 8 times faster than L2 serves such gathers.  Windows are double
// buffered and their loads issued two windows ahead.  Workgroup = 8 waves,
// each owning 8 tile slots as two quads of 4; within a wave, 16-lane row q
// takes slot q of the quad and each of its lanes 4 of the 64 solves of chunk
// blockIdx.y.  An entry is a pair of words (LDS byte offset of its record,
// FP32 value).  Each row reads 16 words (8 entries) of its own slot's list
// with one LDS read per lane, and a DPP row broadcast hands word j to all
// lanes of the row as an operand.  Per 4 entries (one per slot of the quad):
// one OR (record addresses), one 16-byte LDS read per lane (the four
// records), one broadcast of the value and four FMAs.  An output's entries
// are summed window by window in stored order.  The back projection may split
// a tile's windows between `split` workgroups (partial sums, added in order
// by the step kernel) so that two workgroups share a CU.
// ------------------------------------------------------------------------

// Word J of the calling lane's 16-lane row, in every lane of the row.
template <int J>
__device__ __forceinline__ uint32_t row_bcast(uint32_t v) {
    return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x150 + J, 0xF, 0xF, true));
}

constexpr int kBackThreads = 512;
constexpr int kBackPix = 8;         // tile slots per wave

// LDS of the tile kernel: one array at LDS address 0 (the kernel's only LDS
// object, 32 KB aligned) so that the second window starts at 32 KB and a
// record's byte address within a window is (slot * 256) | (lane offset), the
// window's base being the LDS read's immediate offset.  Between and after the
// windows: a ring of four windows' word offsets (absolute, 65 per window),
// two buffers of staged words (16 words of slack after them) and a ring of
// four windows' record ids.
constexpr uint32_t kWinBytes = (kBackSlots + 1) * 256;
constexpr uint32_t kWin1 = 32768;
constexpr uint32_t kOffsOff = kWinBytes;                                 // u32 [4][65]
constexpr uint32_t kWordsOff = kWin1 + kWinBytes;                        // u32 [2][kBackMaxWords] + 16
constexpr uint32_t kIdsOff = kWordsOff + (2 * kBackMaxWords + 16) * 4;   // u32 [4][kBackSlots]
constexpr uint32_t kBackLds = kIdsOff + 4 * kBackSlots * 4;
static_assert(kOffsOff + 4 * 65 * 4 <= kWin1, "tile kernel LDS layout");
static_assert(kBackSlots * 256 + 256 <= kWin1, "a record address is its slot offset OR the lane offset");
static_assert(kBackMaxWords == 4 * kBackThreads, "one 16-byte word quad per thread");
static_assert(kBackSlots <= kBackThreads && 65 <= kBackThreads, "one record id and one offset per thread");

template <int MODE, int VT>
__global__ __launch_bounds__(kBackThreads) void k_gather_tiles(GatherTileArgs a, FwdArgs f) {
    __shared__ __attribute__((aligned(32768))) uint32_t lds[kBackLds / 4];
    char *const lb = reinterpret_cast<char *>(lds);
    uint32_t *const ids = reinterpret_cast<uint32_t *>(lb + kIdsOff);
    uint32_t *const offs = reinterpret_cast<uint32_t *>(lb + kOffsOff);
    uint32_t *const words = reinterpret_cast<uint32_t *>(lb + kWordsOff);
    constexpr int kQ = (kBackSlots * 16 + kBackThreads - 1) / kBackThreads;   // window quads per thread
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int chunk = blockIdx.y;
    // this workgroup's tile and windows [W0, W0 + cnt): a listed part, or part
    // `part` of `split` equal runs of its tile's windows
    int part, tile, W0, cnt;
    uint32_t pslot = kNoSlot;
    if (a.parts) {
        const uint4 pd = a.parts[blockIdx.x];
        part = 0;
        tile = static_cast<int>(pd.x);
        W0 = static_cast<int>(pd.y);
        cnt = static_cast<int>(pd.z - pd.y);
        pslot = pd.w;
    } else {
        part = blockIdx.x / a.n_tiles;
        const int wg = blockIdx.x - part * a.n_tiles;
        tile = a.tiles_x > 0 ? tile_of(wg, a.tiles_x, a.tiles_x, a.xcd_remap) : wg;
        const int wt0 = a.win_off[tile], nwt = a.win_off[tile + 1] - wt0;
        const int i0 = part * nwt / a.split, i1 = (part + 1) * nwt / a.split;
        W0 = wt0 + i0;
        cnt = i1 - i0;
    }
    // Every global load below is unconditional and range-checked by its buffer
    // descriptor (out of range reads 0); loads for windows past the range fetch
    // the last window again and are never stored.  So the wait counts are static.
    const auto er = make_rsrc(reinterpret_cast<const char *>(a.in) + static_cast<size_t>(chunk) * a.n_in * 256,
                              256u * static_cast<uint32_t>(a.n_in));
    const auto rr = make_rsrc(a.records, 4u * a.n_records);
    const auto wr = make_rsrc(a.word, 4u * a.n_words);
    const auto pr = make_rsrc(a.rp + static_cast<size_t>(W0) * 64, 4u * static_cast<uint32_t>(cnt * 64 + 1));
    const int jlast = cnt - 1;

    float4 acc[2] = {make_float4(0.f, 0.f, 0.f, 0.f), make_float4(0.f, 0.f, 0.f, 0.f)};
    const uint32_t k16 = static_cast<uint32_t>(lane & 15) << 4;
    const uint32_t l16 = static_cast<uint32_t>(lane) & 15u;
    const int qrow = lane >> 4;

    if (cnt > 0) {
        if (w == 0) {   // zero records
            lds[(kBackSlots * 256) / 4 + lane] = 0u;
            lds[(kWin1 + kBackSlots * 256) / 4 + lane] = 0u;
        }
        // record ids and word offsets of window j: global -> registers -> LDS
        // ring slot j & 3 (ids: threads < kBackSlots, offsets: threads <= 64)
        auto ids_load = [&](int j) {
            const int jl = min(j, jlast);
            return make_uint2(__builtin_amdgcn_raw_buffer_load_b32(rr, 4u * (a.rec_off[W0 + jl] + tid), 0, 0),
                              __builtin_amdgcn_raw_buffer_load_b32(pr, 4u * (64u * jl + min(tid, 64)), 0, 0));
        };
        auto ids_store = [&](int j, uint2 v) {
            if (tid < kBackSlots) ids[(j & 3) * kBackSlots + tid] = v.x;
            if (tid <= 64) offs[(j & 3) * 65 + tid] = v.y;
        };
        // a window's records (thread tid moves quads tid + kBackThreads i of 16
        // per record) and its words (one quad per thread), in one of two
        // register sets
        struct Stage {
            uint4 q[kQ];
            uint4 wq;
        };
        auto stage_load = [&](int j, Stage &r) {
            const int jl = min(j, jlast);
            const uint32_t *idg = ids + (jl & 3) * kBackSlots;
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const uint32_t q = tid + kBackThreads * i, qp = q & 15u;
                const uint32_t rec = idg[min(q >> 4, static_cast<uint32_t>(kBackSlots - 1))];
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(er, rec * 256u + qp * 16u, 0, 0);
                r.q[i] = make_uint4(v[0], v[1], v[2], v[3]);
            }
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(wr, 4u * (offs[(jl & 3) * 65] + 4u * tid), 0, 0);
            r.wq = make_uint4(v[0], v[1], v[2], v[3]);
        };
        auto stage_store = [&](int j, int buf, const Stage &r) {
            const uint32_t S = a.rec_off[W0 + j + 1] - a.rec_off[W0 + j];
            char *const wb = lb + (buf ? kWin1 : 0u);
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const uint32_t q = tid + kBackThreads * i, rec = q >> 4, qp = q & 15u;
                if (rec < S) *reinterpret_cast<uint4 *>(wb + rec * 256 + qp * 16) = r.q[i];
            }
            const uint32_t *oj = offs + (j & 3) * 65;
            if (4u * tid < oj[64] - oj[0]) *reinterpret_cast<uint4 *>(&words[buf * kBackMaxWords + 4 * tid]) = r.wq;
        };

        // sums of window j from buffer BUF (a compile-time buffer, so that its
        // base is the LDS read's immediate offset).  The four lists of a quad
        // have equal lengths; they are summed in blocks of 8 entries and a tail
        // of 1-7.  Reading 16 words may run past a list's end into the next
        // list or the slack after the buffers; such words are never used.
        auto compute = [&](int j, auto bufc) {
            constexpr int BUF = decltype(bufc)::value;
            const char *const wbase_lds = lb + (BUF ? kWin1 : 0u);
            const uint32_t *wl = words + BUF * kBackMaxWords;
            const uint32_t *oj = offs + (j & 3) * 65;
            const uint32_t ob = oj[0];
            const uint32_t *rg = oj + w * kBackPix;
            // R entries of each list from the row's words q: the record reads
            // are all issued before the FMAs (a scheduling barrier keeps the
            // compiler from sinking each read to its FMA)
            auto block = [&](auto rc, uint32_t q, float4 &u) {
                constexpr int R = decltype(rc)::value;
                float4 x[R];
                [&]<int... J>(std::integer_sequence<int, J...>) {
                    ((x[J] = *reinterpret_cast<const float4 *>(wbase_lds + (row_bcast<2 * J>(q) | k16))), ...);
                    __builtin_amdgcn_sched_barrier(0);
                    auto fma4 = [&](float v, const float4 &xj) {
                        u.x = fmaf(v, xj.x, u.x);
                        u.y = fmaf(v, xj.y, u.y);
                        u.z = fmaf(v, xj.z, u.z);
                        u.w = fmaf(v, xj.w, u.w);
                    };
                    (fma4(__uint_as_float(row_bcast<2 * J + 1>(q)), x[J]), ...);
                }(std::make_integer_sequence<int, R>{});
            };
#pragma unroll
            for (int qd = 0; qd < 2; ++qd) {
                const int s0 = __builtin_amdgcn_readfirstlane(rg[4 * qd]);
                const int s1 = __builtin_amdgcn_readfirstlane(rg[4 * qd + 1]);
                const int n = (s1 - s0) >> 1;                              // entries of each list
                const uint32_t *wq = wl + (rg[4 * qd + qrow] - ob) + l16;   // this row's list
                float4 u = acc[qd];
                int t = 0;
                for (; t + 8 <= n; t += 8) block(std::integral_constant<int, 8>{}, wq[2 * t], u);
                if (t < n) {
                    const uint32_t q = wq[2 * t];
                    switch (n - t) {
                        case 1: block(std::integral_constant<int, 1>{}, q, u); break;
                        case 2: block(std::integral_constant<int, 2>{}, q, u); break;
                        case 3: block(std::integral_constant<int, 3>{}, q, u); break;
                        case 4: block(std::integral_constant<int, 4>{}, q, u); break;
                        case 5: block(std::integral_constant<int, 5>{}, q, u); break;
                        case 6: block(std::integral_constant<int, 6>{}, q, u); break;
                        default: block(std::integral_constant<int, 7>{}, q, u); break;
                    }
                }
                acc[qd] = u;
            }
        };

        // Software pipeline over the windows j: window j uses buffer j & 1 and
        // register set j & 1.  At the start of step j (after a barrier) buffer
        // j & 1 holds window j, register set (j + 1) & 1 holds window j + 1's
        // loads (issued one step earlier) and the rings hold windows j .. j + 2.
        // Step j issues window j + 3's ids and offsets and window j + 2's loads,
        // sums window j, stores window j + 1 into the other buffer and window
        // j + 3's ids and offsets into the rings (the slot of window j - 1, last
        // read in step j - 1), then waits at the barrier: a load has two steps'
        // sums to land in.
        Stage rs0, rs1;
        auto step = [&](int j, auto pc) {
            constexpr int P = decltype(pc)::value;
            Stage &mine = P ? rs1 : rs0;
            Stage &next = P ? rs0 : rs1;
            const uint2 rid = ids_load(j + 3);
            stage_load(j + 2, mine);
            compute(j, std::integral_constant<int, P>{});
            if (j + 1 < cnt) stage_store(j + 1, P ^ 1, next);
            if (j + 3 < cnt) ids_store(j + 3, rid);
            __syncthreads();
        };
        {
            const uint2 r0 = ids_load(0), r1 = ids_load(1), r2 = ids_load(2);
            ids_store(0, r0);
            ids_store(1, r1);
            if (2 < cnt) ids_store(2, r2);
            __syncthreads();
            stage_load(0, rs0);
            stage_load(1, rs1);
            stage_store(0, 0, rs0);
            __syncthreads();
        }
        for (int j = 0; j < cnt; j += 2) {
            step(j, std::integral_constant<int, 0>{});
            if (j + 1 < cnt) step(j + 1, std::integral_constant<int, 1>{});
        }
    }

#pragma unroll
    for (int qd = 0; qd < 2; ++qd) {
        const int idx = a.outs[tile * 64 + w * kBackPix + 4 * qd + qrow];
        if (idx < 0) continue;
        const int bl = 4 * (lane & 15);
        if constexpr (MODE == GM_BACK) {
            float *out = a.out + (static_cast<size_t>(part) * gridDim.y + chunk) * a.n_out * 64;
            *reinterpret_cast<float4 *>(out + static_cast<size_t>(idx) * 64 + bl) = acc[qd];
        } else if (pslot != kNoSlot) {   // a part of a split tile: partial sums
            const int o = w * kBackPix + 4 * qd + qrow;
            float *pp = f.tile_part + ((static_cast<size_t>(chunk) * a.n_pslots + pslot) * 64 + o) * 64;
            *reinterpret_cast<float4 *>(pp + bl) = acc[qd];
        } else {
            const float v[4] = {acc[qd].x, acc[qd].y, acc[qd].z, acc[qd].w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int b = chunk * 64 + bl + c;
                const size_t o = (static_cast<size_t>(chunk) * f.m + idx) * 64 + bl + c;
                const float gl = f.gamma_lane ? f.gamma_lane[b] : 0.0f;
                const float gam = f.gamma ? f.gamma[o] : gl;
                fwd_epilogue<VT>(f, idx, b, o, v[c], gam, b < f.B);
            }
        }
    }
}

// Forward projection, tiles split between parts: the sum of the parts'
// partial sums in part order, then the epilogue.  Workgroup = one tile of
// chunk blockIdx.y; thread t takes tile slot t / 16 and solves 4 (t % 16) .. +3
// (4 passes of 256 threads cover the 64 slots).
template <int VT>
__global__ __launch_bounds__(256) void k_fwd_reduce(GatherTileArgs a, FwdArgs f) {
    const uint4 rd = a.reds[blockIdx.x];
    const int chunk = blockIdx.y;
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        const int t = pass * 256 + threadIdx.x;
        const int o = t >> 4, bl = 4 * (t & 15);
        const int idx = a.outs[rd.x * 64 + o];
        if (idx < 0) continue;
        float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
        for (uint32_t p = 0; p < rd.z; ++p) {
            const float4 v = *reinterpret_cast<const float4 *>(
                f.tile_part + ((static_cast<size_t>(chunk) * a.n_pslots + rd.y + p) * 64 + o) * 64 + bl);
            if (p == 0) {
                s = v;
            } else {
                s.x += v.x;
                s.y += v.y;
                s.z += v.z;
                s.w += v.w;
            }
        }
        const float v[4] = {s.x, s.y, s.z, s.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int b = chunk * 64 + bl + c;
            const size_t oi = (static_cast<size_t>(chunk) * f.m + idx) * 64 + bl + c;
            const float gl = f.gamma_lane ? f.gamma_lane[b] : 0.0f;
            const float gam = f.gamma ? f.gamma[oi] : gl;
            fwd_epilogue<VT>(f, idx, b, oi, v[c], gam, b < f.B);
        }
    }
}

// ------------------------------------------------------------------------
// FP64 monitoring reductions (deterministic: fixed per-block order, then a
// fixed-order sum over blocks).  Vectors in the layout of B (plain for B = 1,
// lane layout otherwise); partials part[blk][Bp].
// ------------------------------------------------------------------------

__device__ __forceinline__ size_t vidx(int i, int b, int n, int B) {
    return B == 1 ? static_cast<size_t>(i) : lidx(i, b, n);
}

// part[blk][b] = sum over rows of the block of (y - gamma) - g ln y  (y = A x + gamma).
__global__ __launch_bounds__(256) void k_fidelity_terms(int m, int B, int Bp, const float *y,
                                                        const float *g, const float *gamma,
                                                        const float *gamma_lane, double *part) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    double s = 0.0;
    if (b < B) {
        for (int i = blockIdx.x * 4 + w; i < m; i += gridDim.x * 4) {
            const size_t o = vidx(i, b, m, B);
            const double gam = gamma ? gamma[o] : (gamma_lane ? gamma_lane[b] : 0.0f);
            const double yy = y[o];
            s += yy - gam;
            if (g[o] != 0.0f) s -= static_cast<double>(g[o]) * log(yy);
        }
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && b < B)
        part[static_cast<size_t>(blockIdx.x) * Bp + b] =
            red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

// part[blk][b] = lambda1 sum s_eps(u) + lambda2 sum s_eps(v) over the block's pixels (FP64).
__global__ __launch_bounds__(256) void k_reg_value(int n, int B, int Bp, const float *x,
                                                   const LaneParams *lp, double *part) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    const int d = n * n;
    double s = 0.0;
    if (b < B) {
        const LaneParams p = lp[b];
        const double eps = p.eps;
        auto F = [&](int rr, int cc) { return x[vidx(rr * n + cc, b, d, B)]; };
        for (int j = blockIdx.x * 4 + w; j < d; j += gridDim.x * 4) {
            float o[6];
            uv6(F, j / n, j % n, n, o);
            const double q1 = static_cast<double>(o[0]) * o[0] + static_cast<double>(o[1]) * o[1];
            const double q2 = static_cast<double>(o[2]) * o[2] + static_cast<double>(o[3]) * o[3] +
                              static_cast<double>(o[4]) * o[4] + static_cast<double>(o[5]) * o[5];
            const double n1 = sqrt(q1), n2 = sqrt(q2);
            // eps = 0 (the nonsmooth model) takes the first branch: the plain norm
            const double s1 = n1 >= eps ? n1 - eps / 2 : q1 / (2 * eps);
            const double s2 = n2 >= eps ? n2 - eps / 2 : q2 / (2 * eps);
            s += static_cast<double>(p.lambda1) * s1 + static_cast<double>(p.lambda2) * s2;
        }
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && b < B)
        part[static_cast<size_t>(blockIdx.x) * Bp + b] =
            red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

// part[blk][b] = sum over the block's rows of g - gamma (for ACTc of the initial image).
__global__ __launch_bounds__(256) void k_sum_g_minus_gamma(int m, int B, int Bp, const float *g,
                                                           const float *gamma,
                                                           const float *gamma_lane, double *part) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    double s = 0.0;
    if (b < B) {
        for (int i = blockIdx.x * 4 + w; i < m; i += gridDim.x * 4) {
            const size_t o = vidx(i, b, m, B);
            const double gam = gamma ? gamma[o] : (gamma_lane ? gamma_lane[b] : 0.0f);
            s += static_cast<double>(g[o]) - gam;
        }
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && b < B)
        part[static_cast<size_t>(blockIdx.x) * Bp + b] =
            red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

// out[b*ncomp + c] = sum_blk part[(blk*Bp + b)*ncomp + c] for b < B: one wave
// per output, lane l sums blocks l, l+64, ... in order, then a fixed xor tree.
__global__ __launch_bounds__(64) void k_reduce_partials(const double *part, int nblocks, int B,
                                                        int Bp, int ncomp, double *out) {
    const int t = blockIdx.x;
    const int b = t / ncomp, c = t % ncomp;
    if (b >= B) return;
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int k = lane; k < nblocks; k += 64) s += part[(static_cast<size_t>(k) * Bp + b) * ncomp + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) out[t] = s;
}

// ------------------------------------------------------------------------
// Layout conversion and initialisation helpers.
// ------------------------------------------------------------------------

// Solve-major in[b][i] (B rows of n) -> lane layout; padding lanes get 0.
// Grid: (ceil(n/32), 2, chunks); 32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void k_to_lanes(const float *in, float *out, int n, int B) {
    __shared__ float t[32][33];
    const int i0 = blockIdx.x * 32, l0 = blockIdx.y * 32, chunk = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int b = chunk * 64 + l0 + k, i = i0 + tx;
        t[k][tx] = (b < B && i < n) ? in[static_cast<size_t>(b) * n + i] : 0.0f;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int i = i0 + k, l = l0 + tx;
        if (i < n) out[(static_cast<size_t>(chunk) * n + i) * 64 + l] = t[tx][k];
    }
}

// Lane layout -> solve-major out[b][i] for b < B.
__global__ __launch_bounds__(256) void k_from_lanes(const float *in, float *out, int n, int B) {
    __shared__ float t[32][33];
    const int i0 = blockIdx.x * 32, l0 = blockIdx.y * 32, chunk = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int i = i0 + k;
        t[k][tx] = i < n ? in[(static_cast<size_t>(chunk) * n + i) * 64 + l0 + tx] : 0.0f;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int b = chunk * 64 + l0 + k, i = i0 + tx;
        if (b < B && i < n) out[static_cast<size_t>(b) * n + i] = t[tx][k];
    }
}

// Initial image of Section 4.1: TMC * 1_disk (disk of radius N/2 about the
// centre) in the layout of B; padding lanes 0.
__global__ void k_disk_init(int n, int B, int Bp, const double *tmc, float *f, float *ft) {
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t d = static_cast<size_t>(n) * n;
    if (t >= d * Bp) return;
    int j, b;
    if (B == 1) {
        j = static_cast<int>(t);
        b = 0;
    } else {
        const size_t chunk = t / (d * 64), rem = t % (d * 64);
        j = static_cast<int>(rem / 64);
        b = static_cast<int>(chunk * 64 + rem % 64);
    }
    const int r = j / n, c = j % n;
    const double ctr = (n - 1) / 2.0, rad = n / 2.0;
    const bool in = (c - ctr) * (c - ctr) + (r - ctr) * (r - ctr) <= rad * rad;
    const float v = (in && b < B) ? static_cast<float>(tmc[b]) : 0.0f;
    f[t] = v;
    ft[t] = v;
}

__global__ void k_fill(float *p, size_t n, float v) {
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// e[i][b] *= scale[i] (a residual handed to the FP8 transpose, which has no row scales).
__global__ void k_scale_rows(float *e, const float *scale, int m, int B, int Bp) {
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<size_t>(m) * Bp) return;
    const int i = B == 1 ? static_cast<int>(t) : static_cast<int>((t / 64) % m);
    e[t] *= scale[i];
}

__global__ void k_copy(float *dst, const float *src, size_t n) {
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) dst[t] = src[t];
}

// ------------------------------------------------------------------------
// Serving: single-lane transfers in a one-chunk lane layout.
// ------------------------------------------------------------------------

// theta_{k+1} = (t_k - 1) / t_{k+1}, t_k = a k^omega + b (eq. GNtheta), FP64,
// after advancing k; one thread per lane.
__global__ void k_lane_theta(int *lane_k, const double *mom, float *theta) {
    const int b = threadIdx.x;
    const int k = lane_k[b] + 1;
    lane_k[b] = k;
    const double *mm = mom + 4 * b;
    const double tk = mm[0] * pow(static_cast<double>(k), mm[2]) + mm[1];
    const double tk1 = mm[0] * pow(static_cast<double>(k) + 1.0, mm[2]) + mm[1];
    theta[b] = mm[3] != 0.0 ? 0.0f : static_cast<float>((tk - 1.0) / tk1);
}

__global__ void k_lane_scatter(const float *src, float *dst, int n, int lane) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[static_cast<size_t>(i) * 64 + lane] = src[i];
}

__global__ void k_lane_fill(float *dst, int n, int lane, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[static_cast<size_t>(i) * 64 + lane] = v;
}

__global__ void k_lane_gather(const float *src, float *dst, int n, int lane) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[static_cast<size_t>(i) * 64 + lane];
}

// Initial image of Section 4.1 for one lane: TMC * 1_disk.
__global__ void k_lane_disk_init(int n, int lane, double tmc, float *f, float *ft) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n * n) return;
    const int r = j / n, c = j % n;
    const double ctr = (n - 1) / 2.0, rad = n / 2.0;
    const bool in = (c - ctr) * (c - ctr) + (r - ctr) * (r - ctr) <= rad * rad;
    const float v = in ? static_cast<float>(tmc) : 0.0f;
    f[static_cast<size_t>(j) * 64 + lane] = v;
    ft[static_cast<size_t>(j) * 64 + lane] = v;
}

// ------------------------------------------------------------------------
// Launch helpers
// ------------------------------------------------------------------------

namespace {

template <typename IT, int VT>
hipError_t fwd_dispatch(const FwdArgs &a, int group, hipStream_t st) {
    if (a.B == 1) {
        switch (group) {
#define APPGA_FWD_CASE(GG)                                                                       \
    case GG: {                                                                                   \
        const int rows = 256 / GG;                                                               \
        hipLaunchKernelGGL((k_fwd_single<IT, VT, GG>), dim3((a.m + rows - 1) / rows), dim3(256), \
                           0, st, a);                                                            \
        break;                                                                                   \
    }
            APPGA_FWD_CASE(4)
            APPGA_FWD_CASE(8)
            APPGA_FWD_CASE(16)
            APPGA_FWD_CASE(32)
            APPGA_FWD_CASE(64)
#undef APPGA_FWD_CASE
            default:
                return hipErrorInvalidValue;
        }
    } else {
        const int wgs = std::min((a.m + 3) / 4, a.fwd_wgs > 0 ? a.fwd_wgs : 2048);
        hipLaunchKernelGGL((k_fwd_batch<VT>), dim3(wgs, a.Bp / 64), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

template <typename IT, int VT>
hipError_t step_dispatch(const StepArgs &a, int group, hipStream_t st) {
    const int tiles = ((a.n + 3) / 4) * ((a.n + 3) / 4);
    if (a.B == 1) {
        switch (group) {
#define APPGA_STEP_CASE(GG)                                                                    \
    case GG:                                                                                   \
        hipLaunchKernelGGL((k_step_single<IT, VT, GG>), dim3(tiles), dim3(16 * GG), 0, st, a); \
        break;
            APPGA_STEP_CASE(4)
            APPGA_STEP_CASE(8)
            APPGA_STEP_CASE(16)
            APPGA_STEP_CASE(32)
            APPGA_STEP_CASE(64)
#undef APPGA_STEP_CASE
            default:
                return hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL((k_step_batch<VT>), dim3(tiles, a.Bp / 64), dim3(1024), 0, st, a);
    }
    return hipGetLastError();
}

template <typename F>
hipError_t by_type(int idx16, int vtype, F &&f) {
    if (idx16) {
        switch (vtype) {
            case VT_F32: return f(uint16_t{}, std::integral_constant<int, VT_F32>{});
            case VT_BF16: return f(uint16_t{}, std::integral_constant<int, VT_BF16>{});
            case VT_F16: return f(uint16_t{}, std::integral_constant<int, VT_F16>{});
            case VT_FP8: return f(uint16_t{}, std::integral_constant<int, VT_FP8>{});
        }
    } else {
        switch (vtype) {
            case VT_F32: return f(uint32_t{}, std::integral_constant<int, VT_F32>{});
            case VT_BF16: return f(uint32_t{}, std::integral_constant<int, VT_BF16>{});
            case VT_F16: return f(uint32_t{}, std::integral_constant<int, VT_F16>{});
            case VT_FP8: return f(uint32_t{}, std::integral_constant<int, VT_FP8>{});
        }
    }
    return hipErrorInvalidValue;
}

unsigned blocks_for(size_t n) { return static_cast<unsigned>((n + 255) / 256); }

}  // namespace

hipError_t launch_forward(const DevCsr &A, const FwdArgs &args, int group, hipStream_t st) {
    return by_type(A.idx16, A.vtype, [&](auto it, auto vt) {
        return fwd_dispatch<decltype(it), decltype(vt)::value>(args, group, st);
    });
}

hipError_t launch_step(const DevCsr &AT, const StepArgs &args, int group, hipStream_t st) {
    return by_type(AT.idx16, AT.vtype, [&](auto it, auto vt) {
        return step_dispatch<decltype(it), decltype(vt)::value>(args, group, st);
    });
}

// One pass of the separable PSF blur.  Grid: blockIdx.y = chunk of 64 solves
// (Bp == 1: one chunk of one solve); within a chunk, thread u is pixel u / 64,
// lane u % 64 (Bp == 1: pixel u).  The 2R + 1 inputs along the pass's axis are
// read at indices clamped into the image and weighted 0 outside it, so the
// loads carry no branches.  SPLIT: partial sums of the input added first
// (1 or 2; 0 = n_parts at run time).
template <bool LANES, int SPLIT>
__global__ __launch_bounds__(256) void k_psf_pass(const float *in, int n_parts, float *out, int n, int Bp,
                                                  int axis, const float *taps, int R) {
    const int d = n * n;
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= (LANES ? d * 64 : d)) return;
    const int j = LANES ? (u >> 6) : u;
    const size_t base = LANES ? static_cast<size_t>(blockIdx.y) * d * 64 + (u & 63) : 0;
    const int r = j / n, c = j - r * n;
    const int pos = axis == 0 ? c : r;
    const size_t stride = static_cast<size_t>(d) * Bp;
    float acc = 0.0f;
#pragma unroll 9
    for (int k = 0; k <= 2 * R; ++k) {
        const int q = pos + k - R;
        const int qc = min(max(q, 0), n - 1);
        const int jj = axis == 0 ? r * n + qc : qc * n + c;
        const size_t o = LANES ? base + static_cast<size_t>(jj) * 64 : static_cast<size_t>(jj);
        float v = in[o];
        if (SPLIT == 2) v += in[stride + o];
        if (SPLIT == 0)
            for (int p = 1; p < n_parts; ++p) v += in[p * stride + o];
        acc += (q == qc ? taps[k] : 0.0f) * v;
    }
    out[base + (LANES ? static_cast<size_t>(j) * 64 : static_cast<size_t>(j))] = acc;
}

// The same pass for the lane layout with a radius R known at compile time: a
// thread takes a run of P consecutive pixels along the pass's axis for one
// solve, holds the P + 2R inputs they need in registers (indices clamped into
// the image, as above) and forms each output from them with the same weights
// in the same order, so the results equal k_psf_pass's.  Each input is loaded
// once per run instead of once per output, and a wave keeps P + 2R loads in
// flight.
template <int SPLIT, int R, int P>
__global__ __launch_bounds__(256) void k_psf_run(const float *in, float *out, int n, int Bp, int axis,
                                                 const float *taps) {
    const int d = n * n;
    const int runs = (n + P - 1) / P;
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= n * runs * 64) return;
    const int s = u >> 6;
    const int line = s / runs, p0 = (s - line * runs) * P;
    const size_t base = static_cast<size_t>(blockIdx.y) * d * 64 + (u & 63);
    const size_t stride = static_cast<size_t>(d) * Bp;
    auto at = [&](int q) {   // vector index of position q of this line
        const int jj = axis == 0 ? line * n + q : q * n + line;
        return base + static_cast<size_t>(jj) * 64;
    };
    float w[2 * R + 1];
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) w[k] = taps[k];
    float v[P + 2 * R];
#pragma unroll
    for (int t = 0; t < P + 2 * R; ++t) {
        const int qc = min(max(p0 + t - R, 0), n - 1);
        const size_t o = at(qc);
        float x = in[o];
        if (SPLIT == 2) x += in[stride + o];
        v[t] = x;
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
        if (p0 + i >= n) break;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k <= 2 * R; ++k) {
            const int q = p0 + i + k - R;
            acc = fmaf((q >= 0 && q < n) ? w[k] : 0.0f, v[i + k], acc);
        }
        out[at(p0 + i)] = acc;
    }
}

// Run length of k_psf_run (8 measured a little faster than 4 at 128^2 x 64).
constexpr int kPsfRun = 8;

template <int SPLIT>
static hipError_t launch_psf_run(const float *in, float *out, int n, int Bp, int axis, const float *taps, int R,
                                 hipStream_t st) {
    constexpr int P = kPsfRun;
    const int runs = (n + P - 1) / P;
    const dim3 grid((n * runs * 64 + 255) / 256, Bp / 64), block(256);
    switch (R) {
#define APPGA_PSF_RUN_CASE(RR)                                                                               \
    case RR:                                                                                                  \
        hipLaunchKernelGGL((k_psf_run<SPLIT, RR, P>), grid, block, 0, st, in, out, n, Bp, axis, taps);        \
        break;
        APPGA_PSF_RUN_CASE(1)
        APPGA_PSF_RUN_CASE(2)
        APPGA_PSF_RUN_CASE(3)
        APPGA_PSF_RUN_CASE(4)
        APPGA_PSF_RUN_CASE(5)
        APPGA_PSF_RUN_CASE(6)
        APPGA_PSF_RUN_CASE(7)
        APPGA_PSF_RUN_CASE(8)
#undef APPGA_PSF_RUN_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Both passes of the blur in one launch, for the lane layout with R <= 4 known
// at compile time (wider PSFs take k_psf_run twice: their register windows
// would not fit a 1024-thread workgroup).  A workgroup takes an 8 x 8 tile of
// pixels for the 64 solves of chunk blockIdx.y.  Pass 1 (along c): wave w
// takes row w of the tile's 8 + 2R rows (image rows clamped as in
// k_psf_pass), loads its 8 + 2R inputs once and writes its 8 partial outputs
// to LDS.  Pass 2
// (along r): wave w < 8 takes column w of the tile and forms its outputs from
// the 8 + 2R LDS rows they need.  Each LDS row t holds pass 1's result for
// image row clamp(r0 - R + t), the value the second launch of the two-pass
// form reads, and weights and order are those of the two launches, so the
// results are equal; the intermediate image never leaves the CU.
template <int SPLIT, int R>
__global__ __launch_bounds__(1024) void k_psf_2d(const float *in, float *out, int n, int Bp, const float *taps) {
    constexpr int T = 8, ROWS = T + 2 * R;
    static_assert(ROWS <= 16, "one row of the tile per wave");
    __shared__ float mid[ROWS][T][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int d = n * n;
    const int tiles_x = (n + T - 1) / T;
    const int r0 = (blockIdx.x / tiles_x) * T, c0 = (blockIdx.x % tiles_x) * T;
    const size_t base = static_cast<size_t>(blockIdx.y) * d * 64 + lane;
    const size_t stride = static_cast<size_t>(d) * Bp;
    float wt[2 * R + 1];
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) wt[k] = taps[k];
    if (w < ROWS) {
        const int t = w;
        const int rr = min(max(r0 - R + t, 0), n - 1);
        float v[T + 2 * R];
#pragma unroll
        for (int i = 0; i < T + 2 * R; ++i) {
            const int qc = min(max(c0 - R + i, 0), n - 1);
            const size_t o = base + static_cast<size_t>(rr * n + qc) * 64;
            float x = in[o];
            if (SPLIT == 2) x += in[stride + o];
            v[i] = x;
        }
#pragma unroll
        for (int j = 0; j < T; ++j) {
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k <= 2 * R; ++k) {
                const int q = c0 + j + k - R;
                acc = fmaf((q >= 0 && q < n) ? wt[k] : 0.0f, v[j + k], acc);
            }
            mid[t][j][lane] = acc;
        }
    }
    __syncthreads();
    const int c = c0 + w;
    if (w >= T || c >= n) return;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        const int r = r0 + i;
        if (r >= n) break;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k <= 2 * R; ++k) {
            const int q = r + k - R;
            acc = fmaf((q >= 0 && q < n) ? wt[k] : 0.0f, mid[i + k][w][lane], acc);
        }
        out[base + static_cast<size_t>(r * n + c) * 64] = acc;
    }
}

hipError_t launch_psf_blur(const float *in, int n_parts, float *tmp, float *out, int n, int B, int Bp,
                           const float *taps, int R, hipStream_t st) {
    if (Bp != 1 && Bp % 64 == 0 && R >= 1 && R <= 4 && (n_parts == 1 || n_parts == 2)) {
        const int tiles_x = (n + 7) / 8;
        const dim3 grid(tiles_x * tiles_x, Bp / 64), block(1024);
        switch (R * 4 + n_parts) {
#define APPGA_PSF_2D_CASE(RR)                                                                         \
    case RR * 4 + 1:                                                                                   \
        hipLaunchKernelGGL((k_psf_2d<1, RR>), grid, block, 0, st, in, out, n, Bp, taps);               \
        break;                                                                                         \
    case RR * 4 + 2:                                                                                   \
        hipLaunchKernelGGL((k_psf_2d<2, RR>), grid, block, 0, st, in, out, n, Bp, taps);               \
        break;
            APPGA_PSF_2D_CASE(1)
            APPGA_PSF_2D_CASE(2)
            APPGA_PSF_2D_CASE(3)
            APPGA_PSF_2D_CASE(4)
#undef APPGA_PSF_2D_CASE
            default:
                return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    hipError_t he = launch_psf_pass(in, n_parts, tmp, n, B, Bp, 0, taps, R, st);
    if (he == hipSuccess) he = launch_psf_pass(tmp, 1, out, n, B, Bp, 1, taps, R, st);
    return he;
}

hipError_t launch_psf_pass(const float *in, int n_parts, float *out, int n, int B, int Bp, int axis,
                           const float *taps, int R, hipStream_t st) {
    (void)B;
    if (R < 0 || 2 * R + 1 > kPsfMaxTaps || n_parts < 1 || (Bp != 1 && Bp % 64 != 0)) return hipErrorInvalidValue;
    const int d = n * n;
    const dim3 block(256);
    if (Bp != 1 && R >= 1 && R <= 8 && n_parts <= 2)
        return n_parts == 1 ? launch_psf_run<1>(in, out, n, Bp, axis, taps, R, st)
                            : launch_psf_run<2>(in, out, n, Bp, axis, taps, R, st);
    if (Bp == 1) {
        const dim3 grid((d + 255) / 256, 1);
        if (n_parts == 1)
            hipLaunchKernelGGL((k_psf_pass<false, 1>), grid, block, 0, st, in, n_parts, out, n, Bp, axis, taps, R);
        else
            hipLaunchKernelGGL((k_psf_pass<false, 0>), grid, block, 0, st, in, n_parts, out, n, Bp, axis, taps, R);
    } else {
        const dim3 grid((d * 64 + 255) / 256, Bp / 64);
        if (n_parts == 1)
            hipLaunchKernelGGL((k_psf_pass<true, 1>), grid, block, 0, st, in, n_parts, out, n, Bp, axis, taps, R);
        else if (n_parts == 2)
            hipLaunchKernelGGL((k_psf_pass<true, 2>), grid, block, 0, st, in, n_parts, out, n, Bp, axis, taps, R);
        else
            hipLaunchKernelGGL((k_psf_pass<true, 0>), grid, block, 0, st, in, n_parts, out, n, Bp, axis, taps, R);
    }
    return hipGetLastError();
}

int afppa_blocks(int n, int Bp) {
    const int d = n * n;
    const int per_block = Bp == 1 ? kAfppaThreads : (kAfppaThreads / 64) * kAfppaPix;
    return (d + per_block - 1) / per_block;
}

hipError_t launch_afppa_primal(const AfppaArgs &a, hipStream_t st) {
    const dim3 grid(afppa_blocks(a.n, a.Bp), a.Bp == 1 ? 1 : a.Bp / 64);
    const dim3 block(kAfppaThreads);
    if (a.gf_split < 1) return hipErrorInvalidValue;
    if (a.Bp == 1) {
        if (a.gf_split == 1)
            hipLaunchKernelGGL((k_afppa_primal<false, 1>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_afppa_primal<false, 0>), grid, block, 0, st, a);
    } else if (a.gf_split == 1) {
        hipLaunchKernelGGL((k_afppa_primal<true, 1>), grid, block, 0, st, a);
    } else if (a.gf_split == 2) {
        hipLaunchKernelGGL((k_afppa_primal<true, 2>), grid, block, 0, st, a);
    } else {
        hipLaunchKernelGGL((k_afppa_primal<true, 0>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_afppa_dual(const AfppaArgs &a, hipStream_t st) {
    const dim3 grid(afppa_blocks(a.n, a.Bp), a.Bp == 1 ? 1 : a.Bp / 64);
    if (a.Bp == 1)
        hipLaunchKernelGGL(k_afppa_dual<false>, grid, dim3(kAfppaThreads), 0, st, a);
    else
        hipLaunchKernelGGL(k_afppa_dual<true>, grid, dim3(kAfppaThreads), 0, st, a);
    return hipGetLastError();
}

int pad_lanes(int B) { return B == 1 ? 1 : (B + 63) / 64 * 64; }

int step_blocks(int n, int B) {
    (void)B;
    return ((n + 3) / 4) * ((n + 3) / 4);
}

int fidelity_blocks(int m) { return std::min(1024, std::max(1, (m + 63) / 64)); }
int reg_value_blocks(int n) { return std::min(1024, std::max(1, (n * n + 63) / 64)); }
int sum_blocks(int m) { return fidelity_blocks(m); }

hipError_t launch_fidelity_terms(int m, int B, const float *y, const float *g, const float *gamma,
                                 const float *gamma_lane, double *part, hipStream_t st) {
    hipLaunchKernelGGL(k_fidelity_terms, dim3(fidelity_blocks(m), (B + 63) / 64), dim3(256), 0, st,
                       m, B, pad_lanes(B), y, g, gamma, gamma_lane, part);
    return hipGetLastError();
}

hipError_t launch_reg_value(int n, int B, const float *x, const LaneParams *lp, double *part,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_reg_value, dim3(reg_value_blocks(n), (B + 63) / 64), dim3(256), 0, st, n,
                       B, pad_lanes(B), x, lp, part);
    return hipGetLastError();
}

hipError_t launch_sum_g_minus_gamma(int m, int B, const float *g, const float *gamma,
                                    const float *gamma_lane, double *part, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_g_minus_gamma, dim3(sum_blocks(m), (B + 63) / 64), dim3(256), 0, st,
                       m, B, pad_lanes(B), g, gamma, gamma_lane, part);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const double *part, int nblocks, int B, int ncomp, double *out,
                                  hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(B * ncomp), dim3(64), 0, st, part, nblocks, B,
                       pad_lanes(B), ncomp, out);
    return hipGetLastError();
}

hipError_t launch_to_lanes(const float *in, float *out, int n, int B, hipStream_t st) {
    hipLaunchKernelGGL(k_to_lanes, dim3((n + 31) / 32, 2, (B + 63) / 64), dim3(256), 0, st, in, out,
                       n, B);
    return hipGetLastError();
}

hipError_t launch_from_lanes(const float *in, float *out, int n, int B, hipStream_t st) {
    hipLaunchKernelGGL(k_from_lanes, dim3((n + 31) / 32, 2, (B + 63) / 64), dim3(256), 0, st, in,
                       out, n, B);
    return hipGetLastError();
}

hipError_t launch_disk_init(int n, int B, const double *tmc, float *f, float *ft, hipStream_t st) {
    const size_t total = static_cast<size_t>(n) * n * pad_lanes(B);
    hipLaunchKernelGGL(k_disk_init, dim3(blocks_for(total)), dim3(256), 0, st, n, B, pad_lanes(B),
                       tmc, f, ft);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, size_t n, float v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_scale_rows(float *e, const float *scale, int m, int B, hipStream_t st) {
    const size_t n = static_cast<size_t>(m) * pad_lanes(B);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_rows, dim3(blocks_for(n)), dim3(256), 0, st, e, scale, m, B,
                       pad_lanes(B));
    return hipGetLastError();
}

int back_tiles_split(const DevGatherTiles &bt) {
    return (bt.n_tiles < 512 && bt.n_groups >= 2) ? 2 : 1;
}

static GatherTileArgs gather_args(const DevGatherTiles &t) {
    GatherTileArgs a{};
    a.parts = nullptr;
    a.reds = nullptr;
    a.n_pslots = 0;
    a.win_off = t.win_off;
    a.rec_off = t.rec_off;
    a.records = t.records;
    a.rp = t.rp;
    a.word = t.word;
    a.outs = t.outs;
    a.n_records = static_cast<uint32_t>(t.n_records);
    a.n_words = static_cast<uint32_t>(t.n_words);
    a.n_tiles = t.n_tiles;
    a.tiles_x = t.tiles_x;
    return a;
}

hipError_t launch_back_tiles(const DevGatherTiles &bt, int vtype, int n, int m, int Bp, int xcd_remap,
                             int split, const float *e, float *out, hipStream_t st) {
    (void)vtype;
    if (!bt.valid || Bp < 64 || Bp % 64 != 0 || split < 1 || split > std::max(1, bt.n_groups))
        return hipErrorInvalidValue;
    GatherTileArgs a = gather_args(bt);
    a.xcd_remap = xcd_remap;
    a.split = split;
    a.n_in = m;
    a.n_out = n * n;
    a.in = e;
    a.out = out;
    const FwdArgs f{};
    const dim3 grid(static_cast<unsigned>(bt.n_tiles * split), static_cast<unsigned>(Bp / 64));
    hipLaunchKernelGGL((k_gather_tiles<GM_BACK, VT_F32>), grid, dim3(kBackThreads), 0, st, a, f);
    return hipGetLastError();
}

hipError_t launch_fwd_tiles(const DevGatherTiles &ft, int vtype, const FwdArgs &fa, hipStream_t st) {
    if (!ft.valid || fa.Bp < 64 || fa.Bp % 64 != 0 || !ft.parts || (ft.n_reds > 0 && !fa.tile_part))
        return hipErrorInvalidValue;
    GatherTileArgs a = gather_args(ft);
    a.xcd_remap = 0;
    a.split = 1;
    a.n_in = fa.n_x;
    a.n_out = fa.m;
    a.in = fa.x;
    a.out = nullptr;
    a.parts = ft.parts;
    a.reds = ft.reds;
    a.n_pslots = ft.n_pslots;
    const dim3 grid(static_cast<unsigned>(ft.n_parts), static_cast<unsigned>(fa.Bp / 64));
    if (vtype == VT_FP8)
        hipLaunchKernelGGL((k_gather_tiles<GM_FWD, VT_FP8>), grid, dim3(kBackThreads), 0, st, a, fa);
    else
        hipLaunchKernelGGL((k_gather_tiles<GM_FWD, VT_F32>), grid, dim3(kBackThreads), 0, st, a, fa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ft.n_reds == 0) return e;
    const dim3 rgrid(static_cast<unsigned>(ft.n_reds), static_cast<unsigned>(fa.Bp / 64));
    if (vtype == VT_FP8)
        hipLaunchKernelGGL(k_fwd_reduce<VT_FP8>, rgrid, dim3(256), 0, st, a, fa);
    else
        hipLaunchKernelGGL(k_fwd_reduce<VT_F32>, rgrid, dim3(256), 0, st, a, fa);
    return hipGetLastError();
}

hipError_t launch_lane_theta(int *lane_k, const double *mom, float *theta, hipStream_t st) {
    hipLaunchKernelGGL(k_lane_theta, dim3(1), dim3(64), 0, st, lane_k, mom, theta);
    return hipGetLastError();
}

hipError_t launch_lane_scatter(const float *src, float *dst, int n, int lane, hipStream_t st) {
    hipLaunchKernelGGL(k_lane_scatter, dim3(blocks_for(n)), dim3(256), 0, st, src, dst, n, lane);
    return hipGetLastError();
}

hipError_t launch_lane_fill(float *dst, int n, int lane, float v, hipStream_t st) {
    hipLaunchKernelGGL(k_lane_fill, dim3(blocks_for(n)), dim3(256), 0, st, dst, n, lane, v);
    return hipGetLastError();
}

hipError_t launch_lane_gather(const float *src, float *dst, int n, int lane, hipStream_t st) {
    hipLaunchKernelGGL(k_lane_gather, dim3(blocks_for(n)), dim3(256), 0, st, src, dst, n, lane);
    return hipGetLastError();
}

hipError_t launch_lane_disk_init(int n, int lane, double tmc, float *f, float *ft, hipStream_t st) {
    hipLaunchKernelGGL(k_lane_disk_init, dim3(blocks_for(static_cast<size_t>(n) * n)), dim3(256), 0,
                       st, n, lane, tmc, f, ft);
    return hipGetLastError();
}

hipError_t launch_copy(float *dst, const float *src, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(blocks_for(n)), dim3(256), 0, st, dst, src, n);
    return hipGetLastError();
}

}  // namespace appga
