// HIP kernels of the APPGA iteration for CDNA4 (gfx950).
//
// One APPGA iteration (Section 2.2, eq. APPGAiter with the closed-form prox
// max(., 0) and the gradients of Section 2.2) runs as two kernels:
//
//  forward  : y = A f~ + gamma and e = 1 - g / max(y, tau)      (grad F, first half)
//  step     : grad F = A^T e over the stored transpose, the SHOITV gradient
//             B1^T w1 B1 f~ + B2^T w2 B2 f~ from an LDS halo tile, the EM
//             preconditioner P = beta f^k / Lambda, f^{k+1} = max(f~ - P (grad F +
//             grad R), 0) and the next extrapolation f~^{k+1} = f^{k+1} +
//             theta_{k+1} (f^{k+1} - f^k) (eq. GNtheta)
//
// Layouts: every per-solve vector is stored [index][B] (solves innermost).
//  - B = 1 ("single") kernels give each matrix row a group of G lanes; each
//    lane reads whole 8-entry chunks (16-byte index and value loads) and the
//    group reduces with cross-lane shuffles.
//  - B > 1 ("batch") kernels give each row one wave whose 64 lanes are 64
//    solves: the matrix entry is wave-uniform (scalar loads) and the gather of
//    x[col][0:B] is one coalesced B*4-byte access per nonzero.
// Matrix rows are padded with zero entries to multiples of 8 (kChunk), so no
// kernel handles a ragged tail inside a row.

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

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

// ------------------------------------------------------------------------
// Forward projection, B = 1: G lanes per row.
// ------------------------------------------------------------------------

template <typename IT, int VT, int G>
__global__ __launch_bounds__(256) void k_fwd_single(FwdArgs a) {
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int row = blockIdx.x * (256 / G) + threadIdx.x / G;
    const IT *__restrict__ col = static_cast<const IT *>(a.col);
    const float *__restrict__ x = a.x;
    float acc = 0.0f;
    if (row < a.m) {
        const int k0 = a.row_ptr[row], k1 = a.row_ptr[row + 1];
        for (int k = k0 + gl * kChunk; k < k1; k += G * kChunk) {
            uint32_t c[8];
            float v[8], xv[8];
            load_cols8<IT>(col, k, c);
            load_vals8<VT>(a.val, k, v);
#pragma unroll
            for (int t = 0; t < 8; ++t) xv[t] = x[c[t]];
#pragma unroll
            for (int t = 0; t < 8; ++t) acc = fmaf(v[t], xv[t], acc);
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (row < a.m && gl == 0) {
        if constexpr (VT == VT_FP8) acc *= a.row_scale[row];
        const float gam = a.gamma ? a.gamma[row] : (a.gamma_lane ? a.gamma_lane[0] : 0.0f);
        float y = acc + gam;
        if (a.mode == FM_PROJ) {
            a.out[row] = y;
        } else {
            const float tau = y_floor(gam);
            if (y < tau) {
                y = tau;
                if (a.clamps) atomicAdd(a.clamps, 1ull);
            }
            float ev = 1.0f - a.g[row] / y;
            if constexpr (VT == VT_FP8) if (a.scale_out) ev *= a.row_scale[row];
            a.out[row] = ev;
        }
    }
}

// ------------------------------------------------------------------------
// Forward projection, B > 1: one wave per row, lanes = solves (64 per
// blockIdx.y chunk).
// ------------------------------------------------------------------------

template <typename IT, int VT>
__global__ __launch_bounds__(256) void k_fwd_batch(FwdArgs a) {
    const int lane = threadIdx.x & 63;
    const int row = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (row >= a.m) return;
    const int B = a.B;
    const int b = blockIdx.y * 64 + lane;
    const bool act = b < B;
    const int bl = act ? b : B - 1;  // idle lanes re-read a valid element (same cache line)
    const IT *__restrict__ col = static_cast<const IT *>(a.col);
    const float *__restrict__ x = a.x;
    const int k0 = a.row_ptr[row], k1 = a.row_ptr[row + 1];
    float acc = 0.0f;
    for (int k = k0; k < k1; k += kChunk) {
        uint32_t c[8];
        float v[8], xv[8];
        load_cols8<IT>(col, k, c);
        load_vals8<VT>(a.val, k, v);
#pragma unroll
        for (int t = 0; t < 8; ++t) xv[t] = x[static_cast<size_t>(c[t]) * B + bl];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc = fmaf(v[t], xv[t], acc);
    }
    if (!act) return;
    if constexpr (VT == VT_FP8) acc *= a.row_scale[row];
    const size_t o = static_cast<size_t>(row) * B + b;
    const float gam = a.gamma ? a.gamma[o] : (a.gamma_lane ? a.gamma_lane[b] : 0.0f);
    float y = acc + gam;
    if (a.mode == FM_PROJ) {
        a.out[o] = y;
    } else {
        const float tau = y_floor(gam);
        if (y < tau) {
            y = tau;
            if (a.clamps) atomicAdd(a.clamps + b, 1ull);
        }
        float ev = 1.0f - a.g[o] / y;
        if constexpr (VT == VT_FP8) if (a.scale_out) ev *= a.row_scale[row];
        a.out[o] = ev;
    }
}

// ------------------------------------------------------------------------
// SHOITV gradient on a tile (Section 2.1 operators, Section 2.2 gradient).
//
// With image index j = r*N + c, X (x) Y acts as X along r and Y along c, and
// (Dx)_c = [c>=1](x_c - x_{c-1}), (D^T y)_c = [c>=1] y_c - [c<=N-2] y_{c+1},
// L = -D^T D: (Lx)_c = [c<=N-2](x_{c+1} - x_c) + [c>=1](x_{c-1} - x_c).
//   u1 = (I(x)D)f, u2 = (D(x)I)f, v1 = (I(x)L)f, v2 = (-D^T(x)D)f,
//   v3 = (L(x)I)f, v4 = (D(x)-D^T)f,
// weights w1 = lambda1 / max(|u|, eps), w2 = lambda2 / max(|v|, eps), and
//   grad R = (I(x)D^T)(w1 u1) + (D^T(x)I)(w1 u2) + (I(x)L)(w2 v1)
//          + (-D(x)D^T)(w2 v2) + (L(x)I)(w2 v3) + (D^T(x)-D)(w2 v4).
// The value at (r, c) needs the weighted vectors at (r, c) and six
// neighbours, which need f within a radius of 2.
// ------------------------------------------------------------------------

// The six components at (r, c) (0 <= r, c < N); F(r, c) reads the image.
template <typename Fn>
__device__ __forceinline__ void uv6(const Fn &F, int r, int c, int N, float o[6]) {
    const float f00 = F(r, c);
    const bool cl = c >= 1, cr = c <= N - 2, ru = r >= 1, rd = r <= N - 2;
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
template <typename Fn>
__device__ __forceinline__ void pq6(const Fn &F, int r, int c, int N, float l1, float l2, float eps,
                                    float o[6]) {
    uv6(F, r, c, N, o);
    const float n1 = sqrtf(o[0] * o[0] + o[1] * o[1]);
    const float n2 = sqrtf(o[2] * o[2] + o[3] * o[3] + o[4] * o[4] + o[5] * o[5]);
    const float w1 = l1 / fmaxf(n1, eps);
    const float w2 = l2 / fmaxf(n2, eps);
    o[0] *= w1; o[1] *= w1;
    o[2] *= w2; o[3] *= w2; o[4] *= w2; o[5] *= w2;
}

template <typename Fn>
__device__ __forceinline__ float grad_reg_at(const Fn &F, int r, int c, int N, float l1, float l2,
                                             float eps) {
    const bool cl = c >= 1, cr = c <= N - 2, ru = r >= 1, rd = r <= N - 2;
    float P0[6], Pr[6] = {0}, Pd[6] = {0}, Pl[6] = {0}, Pu[6] = {0}, Pur[6] = {0}, Pdl[6] = {0};
    pq6(F, r, c, N, l1, l2, eps, P0);
    if (cr) pq6(F, r, c + 1, N, l1, l2, eps, Pr);
    if (rd) pq6(F, r + 1, c, N, l1, l2, eps, Pd);
    if (cl) pq6(F, r, c - 1, N, l1, l2, eps, Pl);
    if (ru) pq6(F, r - 1, c, N, l1, l2, eps, Pu);
    if (ru && cr) pq6(F, r - 1, c + 1, N, l1, l2, eps, Pur);
    if (rd && cl) pq6(F, r + 1, c - 1, N, l1, l2, eps, Pdl);
    // (I (x) D^T) p1 and (D^T (x) I) p2
    float g = (cl ? P0[0] : 0.0f) - (cr ? Pr[0] : 0.0f);
    g += (ru ? P0[1] : 0.0f) - (rd ? Pd[1] : 0.0f);
    // (I (x) L) q1
    g += (cr ? Pr[2] - P0[2] : 0.0f) + (cl ? Pl[2] - P0[2] : 0.0f);
    // (-D (x) D^T) q2: t(r') = [c>=1] q2(r', c) - [c<=N-2] q2(r', c+1); -[r>=1](t(r) - t(r-1))
    if (ru) {
        const float t0 = (cl ? P0[3] : 0.0f) - (cr ? Pr[3] : 0.0f);
        const float t1 = (cl ? Pu[3] : 0.0f) - (cr ? Pur[3] : 0.0f);
        g -= t0 - t1;
    }
    // (L (x) I) q3
    g += (rd ? Pd[4] - P0[4] : 0.0f) + (ru ? Pu[4] - P0[4] : 0.0f);
    // (D^T (x) -D) q4: s(r') = -[c>=1](q4(r', c) - q4(r', c-1)); [r>=1] s(r) - [r<=N-2] s(r+1)
    if (cl) {
        const float s0 = -(P0[5] - Pl[5]);
        const float s1 = -(Pd[5] - Pdl[5]);
        g += (ru ? s0 : 0.0f) - (rd ? s1 : 0.0f);
    }
    return g;
}

// Preconditioned gradient step, prox and extrapolation for one pixel/solve.
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
// Step kernel, B = 1.  Tile of 4 x 4 pixels per workgroup (256 threads);
// groups of G lanes back-project one pixel each, then 16 threads apply the
// stencil and the update from an 8 x 8 halo in LDS.
// ------------------------------------------------------------------------

template <typename IT, int VT, int G>
__global__ __launch_bounds__(256) void k_step_single(StepArgs a) {
    __shared__ float halo[64];
    __shared__ float gfs[16];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int gl = lane & (G - 1);
    const int grp = tid / G;
    constexpr int NG = 256 / G;
    const int N = a.n;
    const int tiles_x = a.tiles_x, tiles_y = (N + 3) / 4;
    const int tile = tile_of(blockIdx.x, tiles_x, tiles_y, a.xcd_remap);
    const int r0 = (tile / tiles_x) * 4, c0 = (tile % tiles_x) * 4;
    const IT *__restrict__ col = static_cast<const IT *>(a.col);
    const float *__restrict__ e = a.e;

    if (a.out_mode != SO_REG) {
        for (int p = grp; p < 16; p += NG) {
            const int r = r0 + (p >> 2), c = c0 + (p & 3);
            float acc = 0.0f;
            if (r < N && c < N) {
                const int j = r * N + c;
                const int k0 = a.row_ptr[j], k1 = a.row_ptr[j + 1];
                for (int k = k0 + gl * kChunk; k < k1; k += G * kChunk) {
                    uint32_t cc[8];
                    float v[8], ev[8];
                    load_cols8<IT>(col, k, cc);
                    load_vals8<VT>(a.val, k, v);
#pragma unroll
                    for (int t = 0; t < 8; ++t) ev[t] = e[cc[t]];
#pragma unroll
                    for (int t = 0; t < 8; ++t) acc = fmaf(v[t], ev[t], acc);
                }
            }
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (gl == 0) gfs[p] = acc;
        }
    }
    if (tid < 64) {
        const int hr = r0 - 2 + (tid >> 3), hc = c0 - 2 + (tid & 7);
        halo[tid] = (hr >= 0 && hr < N && hc >= 0 && hc < N) ? a.ft[hr * N + hc] : 0.0f;
    }
    __syncthreads();
    if (tid >= 16) return;
    const int r = r0 + (tid >> 2), c = c0 + (tid & 3);
    const bool in = r < N && c < N;
    double dd = 0.0, nn = 0.0;
    if (in) {
        const LaneParams lp = a.lp[0];
        auto F = [&](int rr, int cc) { return halo[(rr - r0 + 2) * 8 + (cc - c0 + 2)]; };
        const float gR = grad_reg_at(F, r, c, N, lp.lambda1, lp.lambda2, lp.eps);
        const int j = r * N + c;
        if (a.out_mode == SO_BACK) {
            a.out[j] = gfs[tid];
        } else if (a.out_mode == SO_REG) {
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
// Step kernel, B > 1.  Tile of 4 x 4 pixels, 4 waves; wave w owns tile row w;
// lanes = solves (64 per blockIdx.y chunk).
// ------------------------------------------------------------------------

template <typename IT, int VT>
__global__ __launch_bounds__(256) void k_step_batch(StepArgs a) {
    __shared__ float halo[64][64];
    __shared__ double red[4][64][2];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int N = a.n, B = a.B;
    const int tiles_x = a.tiles_x, tiles_y = (N + 3) / 4;
    const int tile = tile_of(blockIdx.x, tiles_x, tiles_y, a.xcd_remap);
    const int r0 = (tile / tiles_x) * 4, c0 = (tile % tiles_x) * 4;
    const int b = blockIdx.y * 64 + lane;
    const bool act = b < B;
    const int bl = act ? b : B - 1;  // idle lanes re-read a valid element (same cache line)
    const IT *__restrict__ col = static_cast<const IT *>(a.col);
    const float *__restrict__ e = a.e;
    const int r = r0 + w;

    float gF[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (a.out_mode != SO_REG) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int c = c0 + p;
            if (r < N && c < N) {
                const int j = r * N + c;
                const int k0 = a.row_ptr[j], k1 = a.row_ptr[j + 1];
                float acc = 0.0f;
                for (int k = k0; k < k1; k += kChunk) {
                    uint32_t cc[8];
                    float v[8], ev[8];
                    load_cols8<IT>(col, k, cc);
                    load_vals8<VT>(a.val, k, v);
#pragma unroll
                    for (int t = 0; t < 8; ++t) ev[t] = e[static_cast<size_t>(cc[t]) * B + bl];
#pragma unroll
                    for (int t = 0; t < 8; ++t) acc = fmaf(v[t], ev[t], acc);
                }
                gF[p] = acc;
            }
        }
    }
    for (int q = w; q < 64; q += 4) {
        const int hr = r0 - 2 + (q >> 3), hc = c0 - 2 + (q & 7);
        halo[q][lane] = (hr >= 0 && hr < N && hc >= 0 && hc < N)
                            ? a.ft[static_cast<size_t>(hr * N + hc) * B + bl]
                            : 0.0f;
    }
    __syncthreads();
    double dd = 0.0, nn = 0.0;
    if (act && r < N) {
        const LaneParams lp = a.lp[b];
        const float th = a.theta_next ? a.theta_next[b] : 0.0f;
        auto F = [&](int rr, int cc) { return halo[(rr - r0 + 2) * 8 + (cc - c0 + 2)][lane]; };
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int c = c0 + p;
            if (c >= N) continue;
            const size_t o = static_cast<size_t>(r * N + c) * B + b;
            if (a.out_mode == SO_BACK) {
                a.out[o] = gF[p];
                continue;
            }
            const float gR = grad_reg_at(F, r, c, N, lp.lambda1, lp.lambda2, lp.eps);
            if (a.out_mode == SO_REG) {
                a.out[o] = gR;
                continue;
            }
            const float ftc = F(r, c);
            const float fk = a.f[o];
            const float P = precond(a.pmode, fk, a.lam[r * N + c], lp, a.pbuf, o);
            const float z = ftc - P * (gF[p] + gR);
            const float fn = z > 0.0f ? z : 0.0f;
            a.f[o] = fn;
            a.ft_next[o] = fn + th * (fn - fk);
            const double df = static_cast<double>(fn) - static_cast<double>(fk);
            dd += df * df;
            nn += static_cast<double>(fn) * static_cast<double>(fn);
        }
    }
    if (a.re_part) {
        red[w][lane][0] = dd;
        red[w][lane][1] = nn;
        __syncthreads();
        if (w == 0 && act) {
            const double s0 = red[0][lane][0] + red[1][lane][0] + red[2][lane][0] + red[3][lane][0];
            const double s1 = red[0][lane][1] + red[1][lane][1] + red[2][lane][1] + red[3][lane][1];
            const size_t o = (static_cast<size_t>(blockIdx.x) * B + b) * 2;
            a.re_part[o] = s0;
            a.re_part[o + 1] = s1;
        }
    }
}

// ------------------------------------------------------------------------
// FP64 monitoring reductions (deterministic: fixed per-block order, then a
// fixed-order sum over blocks).
// ------------------------------------------------------------------------

// part[blk][b] = sum over rows of the block of (y - gamma) - g ln y  (y = A x + gamma).
__global__ __launch_bounds__(256) void k_fidelity_terms(int m, int B, const float *y, const float *g,
                                                        const float *gamma, const float *gamma_lane,
                                                        double *part) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    double s = 0.0;
    if (b < B) {
        for (int i = blockIdx.x * 4 + w; i < m; i += gridDim.x * 4) {
            const size_t o = static_cast<size_t>(i) * B + b;
            const double gam = gamma ? gamma[o] : (gamma_lane ? gamma_lane[b] : 0.0f);
            const double yy = y[o];
            s += yy - gam;
            if (g[o] != 0.0f) s -= static_cast<double>(g[o]) * log(yy);
        }
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && b < B)
        part[static_cast<size_t>(blockIdx.x) * B + b] =
            red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

// part[blk][b] = lambda1 sum s_eps(u) + lambda2 sum s_eps(v) over the block's pixels (FP64).
__global__ __launch_bounds__(256) void k_reg_value(int n, int B, const float *x,
                                                   const LaneParams *lp, double *part) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    const int d = n * n;
    double s = 0.0;
    if (b < B) {
        const LaneParams p = lp[b];
        const double eps = p.eps;
        auto F = [&](int rr, int cc) { return x[static_cast<size_t>(rr * n + cc) * B + b]; };
        for (int j = blockIdx.x * 4 + w; j < d; j += gridDim.x * 4) {
            float o[6];
            uv6(F, j / n, j % n, n, o);
            const double q1 = static_cast<double>(o[0]) * o[0] + static_cast<double>(o[1]) * o[1];
            const double q2 = static_cast<double>(o[2]) * o[2] + static_cast<double>(o[3]) * o[3] +
                              static_cast<double>(o[4]) * o[4] + static_cast<double>(o[5]) * o[5];
            const double n1 = sqrt(q1), n2 = sqrt(q2);
            const double s1 = n1 > eps ? n1 - eps / 2 : q1 / (2 * eps);
            const double s2 = n2 > eps ? n2 - eps / 2 : q2 / (2 * eps);
            s += static_cast<double>(p.lambda1) * s1 + static_cast<double>(p.lambda2) * s2;
        }
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && b < B)
        part[static_cast<size_t>(blockIdx.x) * B + b] =
            red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

// part[blk][b] = sum over the block's rows of g - gamma (for ACTc of the initial image).
__global__ __launch_bounds__(256) void k_sum_g_minus_gamma(int m, int B, const float *g,
                                                           const float *gamma,
                                                           const float *gamma_lane, double *part) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    double s = 0.0;
    if (b < B) {
        for (int i = blockIdx.x * 4 + w; i < m; i += gridDim.x * 4) {
            const size_t o = static_cast<size_t>(i) * B + b;
            const double gam = gamma ? gamma[o] : (gamma_lane ? gamma_lane[b] : 0.0f);
            s += static_cast<double>(g[o]) - gam;
        }
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && b < B)
        part[static_cast<size_t>(blockIdx.x) * B + b] =
            red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

// out[b*ncomp + c] = sum_blk part[(blk*B + b)*ncomp + c], blocks in order.
__global__ void k_reduce_partials(const double *part, int nblocks, int B, int ncomp, double *out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * ncomp) return;
    const int b = t / ncomp, c = t % ncomp;
    double s = 0.0;
    for (int k = 0; k < nblocks; ++k) s += part[(static_cast<size_t>(k) * B + b) * ncomp + c];
    out[t] = s;
}

// ------------------------------------------------------------------------
// Layout and initialisation helpers.
// ------------------------------------------------------------------------

// out[c][r] = in[r][c] for an rows x cols array (32 x 32 LDS tiles).
__global__ __launch_bounds__(256) void k_transpose(const float *in, float *out, int rows, int cols) {
    __shared__ float t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int r = by + k, c = bx + tx;
        if (r < rows && c < cols) t[k][tx] = in[static_cast<size_t>(r) * cols + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int c = bx + k, r = by + tx;
        if (r < rows && c < cols) out[static_cast<size_t>(c) * rows + r] = t[tx][k];
    }
}

// Initial image of Section 4.1: TMC * 1_disk (disk of radius N/2 about the centre).
__global__ void k_disk_init(int n, int B, const double *tmc, float *f, float *ft) {
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t total = static_cast<size_t>(n) * n * B;
    if (t >= total) return;
    const int b = static_cast<int>(t % B);
    const int j = static_cast<int>(t / B);
    const int r = j / n, c = j % n;
    const double ctr = (n - 1) / 2.0, rad = n / 2.0;
    const bool in = (c - ctr) * (c - ctr) + (r - ctr) * (r - ctr) <= rad * rad;
    const float v = in ? static_cast<float>(tmc[b]) : 0.0f;
    f[t] = v;
    ft[t] = v;
}

__global__ void k_fill(float *p, size_t n, float v) {
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// e[i][b] *= scale[i] (a residual handed to the FP8 transpose, which has no row scales).
__global__ void k_scale_rows(float *e, const float *scale, int m, int B) {
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < static_cast<size_t>(m) * B) e[t] *= scale[t / B];
}

__global__ void k_copy(float *dst, const float *src, size_t n) {
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) dst[t] = src[t];
}

// ------------------------------------------------------------------------
// Launch helpers
// ------------------------------------------------------------------------

namespace {

template <typename IT, int VT>
hipError_t fwd_dispatch_g(const FwdArgs &a, int group, hipStream_t st) {
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
        hipLaunchKernelGGL((k_fwd_batch<IT, VT>), dim3((a.m + 3) / 4, (a.B + 63) / 64), dim3(256),
                           0, st, a);
    }
    return hipGetLastError();
}

template <typename IT, int VT>
hipError_t step_dispatch_g(const StepArgs &a, int group, hipStream_t st) {
    const int tiles = ((a.n + 3) / 4) * ((a.n + 3) / 4);
    if (a.B == 1) {
        switch (group) {
#define APPGA_STEP_CASE(GG)                                                                   \
    case GG:                                                                                  \
        hipLaunchKernelGGL((k_step_single<IT, VT, GG>), dim3(tiles), dim3(256), 0, st, a);    \
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
        hipLaunchKernelGGL((k_step_batch<IT, VT>), dim3(tiles, (a.B + 63) / 64), dim3(256), 0, st,
                           a);
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

}  // namespace

hipError_t launch_forward(const DevCsr &A, const FwdArgs &args, int group, hipStream_t st) {
    return by_type(A.idx16, A.vtype, [&](auto it, auto vt) {
        return fwd_dispatch_g<decltype(it), decltype(vt)::value>(args, group, st);
    });
}

hipError_t launch_step(const DevCsr &AT, const StepArgs &args, int group, hipStream_t st) {
    return by_type(AT.idx16, AT.vtype, [&](auto it, auto vt) {
        return step_dispatch_g<decltype(it), decltype(vt)::value>(args, group, st);
    });
}

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
                       m, B, y, g, gamma, gamma_lane, part);
    return hipGetLastError();
}

hipError_t launch_reg_value(int n, int B, const float *x, const LaneParams *lp, double *part,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_reg_value, dim3(reg_value_blocks(n), (B + 63) / 64), dim3(256), 0, st, n,
                       B, x, lp, part);
    return hipGetLastError();
}

hipError_t launch_sum_g_minus_gamma(int m, int B, const float *g, const float *gamma,
                                    const float *gamma_lane, double *part, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_g_minus_gamma, dim3(sum_blocks(m), (B + 63) / 64), dim3(256), 0, st,
                       m, B, g, gamma, gamma_lane, part);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const double *part, int nblocks, int B, int ncomp, double *out,
                                  hipStream_t st) {
    const int t = B * ncomp;
    hipLaunchKernelGGL(k_reduce_partials, dim3((t + 127) / 128), dim3(128), 0, st, part, nblocks,
                       B, ncomp, out);
    return hipGetLastError();
}

hipError_t launch_transpose(const float *in, float *out, int rows, int cols, hipStream_t st) {
    hipLaunchKernelGGL(k_transpose, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, st, in,
                       out, rows, cols);
    return hipGetLastError();
}

hipError_t launch_disk_init(int n, int B, const double *tmc, float *f, float *ft, hipStream_t st) {
    const size_t total = static_cast<size_t>(n) * n * B;
    hipLaunchKernelGGL(k_disk_init, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0,
                       st, n, B, tmc, f, ft);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, size_t n, float v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, p, n,
                       v);
    return hipGetLastError();
}

hipError_t launch_scale_rows(float *e, const float *scale, int m, int B, hipStream_t st) {
    const size_t n = static_cast<size_t>(m) * B;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_rows, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st,
                       e, scale, m, B);
    return hipGetLastError();
}

hipError_t launch_copy(float *dst, const float *src, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, dst,
                       src, n);
    return hipGetLastError();
}

}  // namespace appga
