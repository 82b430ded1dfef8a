// Internal types shared by the HIP kernels (kernels.hip) and the host side of
// the library (appga_api.cpp, server.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace appga {

// Storage types of matrix values (same numbering as appga_dtype).
enum ValType : int { VT_F32 = 1, VT_BF16 = 2, VT_F16 = 3, VT_FP8 = 4 };

// Entries per chunk read by one lane of the B = 1 kernels (16-byte loads).
constexpr int kChunk = 8;
// Every stored row is padded with zero entries to a multiple of this (two
// chunks: the B > 1 kernels stream rows in groups of 16 entries).
constexpr int kRowPad = 16;

// One stored sparse operator (A, or the transpose used for A^T), CSR with
// rows padded to kChunk entries.  Device pointers.
struct DevCsr {
    int32_t n_rows = 0, n_cols = 0;
    int64_t nnz = 0;          // real entries
    int64_t nnz_padded = 0;   // stored entries
    int32_t *row_ptr = nullptr;  // n_rows + 1, multiples of kRowPad
    void *col = nullptr;         // uint16_t when idx16, else uint32_t (B = 1 kernels)
    uint32_t *col32 = nullptr;   // byte offset col * 256 of each entry's 64-lane record (B > 1 kernels)
    void *val = nullptr;         // float / bf16 / f16 / fp8 (uint8)
    float *row_scale = nullptr;  // FP8 only: value = scale[row] * decode(q)
    int idx16 = 1;
    int vtype = VT_F32;
    int max_row_len = 0;
    double mean_row_len = 0.0;
    int64_t bytes = 0;           // stored bytes (values + indices + row_ptr + scales)
};

// Back projection over pixel tiles for B > 1 (built from the transpose at load
// time).  The image is cut into kBackTile x kBackTile tiles; the angles into
// groups of `group_angles` consecutive angles (rays i with
// i / (n_bins * group_angles) == g).  For tile t and group g, the distinct
// rays that cross the tile, ascending, are the slots of the residual window
// staged in LDS: rays[ray_off[t*G + g] + s] is the ray in slot s (at most
// kBackSlots slots).  The entries of tile-local pixel p (row-major within the
// tile) in group g are entries [rp[(t*G + g)*64 + p], rp[... + 1]) (at most 64),
// in ray order: word = slot*256 | code << 16 for 16- and 8-bit values (the
// stored value code); for FP32 values each entry is two words, slot*256 and
// the value's bits, and the offsets count words.  The lists of the pixel pair
// (2i, 2i+1) are padded to one common multiple of 4 entries with zero-valued
// entries whose slot is kBackSlots (a record of zeros the kernel keeps in
// LDS).  Device pointers.
constexpr int kBackTile = 8;
constexpr int kBackSlots = 96;       // records per window (slot kBackSlots is the zero record)
constexpr int kBackMaxGroups = 48;
constexpr int kBackMaxWords = 2048;  // entries of one tile in one group (padded)

struct DevBackTiles {
    int valid = 0;
    int tiles_x = 0, n_groups = 0, group_angles = 0;
    uint32_t *rp = nullptr;
    uint32_t *word = nullptr;
    uint32_t *ray_off = nullptr;
    uint32_t *rays = nullptr;
    int64_t n_entries = 0, n_rays = 0;
    int64_t bytes = 0;
};

struct BackTileArgs {
    const uint32_t *rp;
    const uint32_t *word;
    const uint32_t *ray_off;
    const uint32_t *rays;
    uint32_t n_entries;     // length of word
    uint32_t n_rays;        // length of rays
    int n;                  // image side
    int tiles_x;            // tiles per image row
    int n_groups;
    int m;                  // rays (length of e per solve)
    int xcd_remap;
    int split;              // workgroups per tile; workgroup s sums groups [s G / split, (s+1) G / split)
    const float *e;         // [m] lane layout, chunk blockIdx.y
    float *out;             // [split][d] lane layout: the partial sums of A^T e
};

// Per-solve (per batch lane) parameters, FP32 copies of the FP64 host values.
struct LaneParams {
    float lambda1, lambda2, eps, beta, fixed_p, pad0, pad1, pad2;
};

// Preconditioner handling inside the fused step kernel.
enum PMode : int {
    PM_EM = 0,          // P = beta f^k / Lambda
    PM_EM_STORE = 1,    // as PM_EM, and store P into pbuf (frozen mode, k <= freeze)
    PM_STORED = 2,      // P = pbuf (frozen mode, k > freeze)
    PM_FIXED = 3        // P = fixed_p
};

// What the fused back-projection / stencil / update kernel writes.
enum StepOut : int {
    SO_STEP = 0,        // f^{k+1} into f, f~^{k+1} into ft_next
    SO_BACK = 1,        // out = A^T e
    SO_REG = 2          // out = B^T grad phi~(B ft)
};

// Forward projection epilogue.
enum FwdMode : int {
    FM_RATIO = 0,       // out = 1 - g / max(A x + gamma, tau)
    FM_PROJ = 1         // out = A x + gamma  (gamma = 0 when absent)
};

struct FwdArgs {
    const int32_t *row_ptr;
    const void *col;
    const uint32_t *col32;
    int64_t nnz_padded;
    const void *val;
    const float *row_scale;
    int m;                  // rows
    int n_x;                // columns (length of x per solve)
    int B;                  // solves
    int Bp;                 // padded lanes: 1 for B = 1, else a multiple of 64
    const float *x;         // [d][B]
    const float *g;         // [m][B]
    const float *gamma;     // [m][B] or null (then gamma_lane)
    const float *gamma_lane;// [B] or null (then 0)
    float *out;             // [m][B]
    int mode;               // FwdMode
    int scale_out;          // FM_RATIO with FP8: write row_scale[i] * e_i (the transpose has no scales)
    int fwd_wgs;            // B > 1: workgroups of the row-strided grid (0 = default)
    unsigned long long *clamps;  // floored-bin counter (may be null)
};

struct StepArgs {
    const int32_t *row_ptr;  // transpose (rows = pixels)
    const void *col;
    const uint32_t *col32;
    int64_t nnz_padded;
    const void *val;
    const float *row_scale;  // unused: FP8 transposes carry A's row scales in e
    int n;                   // image side N
    int m;                   // detector bins (length of e per solve)
    int B;                   // solves
    int Bp;                  // padded lanes: 1 for B = 1, else a multiple of 64
    const float *e;          // [m][B] ratio residual 1 - g / y
    const float *ft;         // [d][B] extrapolated point f~^k
    float *f;                // [d][B] f^k in, f^{k+1} out
    float *ft_next;          // [d][B] f~^{k+1}
    const float *lam;        // [d] Lambda
    const LaneParams *lp;    // [B]
    const float *theta_next; // [B] theta_{k+1}
    float *pbuf;             // [d][B] frozen preconditioner (or null)
    const float *gf_in;      // B > 1: A^T e from the tile kernel as gf_split partial sums (or null: gather here)
    int gf_split;            // number of partial sums in gf_in ([gf_split][d][Bp], added in order)
    int pmode;               // PMode
    int out_mode;            // StepOut
    float *out;              // [d][B] for SO_BACK / SO_REG
    double *re_part;         // [blocks][B][2] sum (f^{k+1}-f^k)^2, sum (f^{k+1})^2 (or null)
    int tiles_x;             // tiles per image row
    int xcd_remap;           // 1: map workgroups to spatially compact tile blocks per XCD
};

// Serving helpers (kernels.hip).
// B > 1 back projection out = A^T e over the tiles (lane layout, Bp / 64 chunks).
hipError_t launch_back_tiles(const DevBackTiles &bt, int vtype, int n, int m, int Bp, int xcd_remap,
                             int split, const float *e, float *out, hipStream_t st);
// Workgroups per tile for the back projection of an n x n image (enough
// workgroups to put two on every CU).
int back_tiles_split(const DevBackTiles &bt);

// Serving: advances the 64 per-lane iteration counters k by one and writes
// theta_{k+1} (eq. GNtheta, FP64) per lane; mom holds {a, b, omega, momentum_none}.
hipError_t launch_lane_theta(int *lane_k, const double *mom, float *theta, hipStream_t st);
hipError_t launch_lane_scatter(const float *src, float *dst, int n, int lane, hipStream_t st);
hipError_t launch_lane_fill(float *dst, int n, int lane, float v, hipStream_t st);
hipError_t launch_lane_gather(const float *src, float *dst, int n, int lane, hipStream_t st);
hipError_t launch_lane_disk_init(int n, int lane, double tmc, float *f, float *ft, hipStream_t st);

// Kernel launch helpers (kernels.hip).  Each returns hipSuccess or the launch error.
hipError_t launch_forward(const DevCsr &A, const FwdArgs &args, int group, hipStream_t st);
hipError_t launch_step(const DevCsr &AT, const StepArgs &args, int group, hipStream_t st);
int step_blocks(int n, int B);
hipError_t launch_fidelity_terms(int m, int B, const float *y, const float *g, const float *gamma,
                                 const float *gamma_lane, double *part, hipStream_t st);
int fidelity_blocks(int m);
hipError_t launch_reg_value(int n, int B, const float *x, const LaneParams *lp, double *part,
                            hipStream_t st);
int reg_value_blocks(int n);
hipError_t launch_reduce_partials(const double *part, int nblocks, int B, int ncomp, double *out,
                                  hipStream_t st);
int pad_lanes(int B);
hipError_t launch_to_lanes(const float *in, float *out, int n, int B, hipStream_t st);
hipError_t launch_from_lanes(const float *in, float *out, int n, int B, hipStream_t st);
hipError_t launch_disk_init(int n, int B, const double *tmc, float *f, float *ft, hipStream_t st);
hipError_t launch_sum_g_minus_gamma(int m, int B, const float *g, const float *gamma,
                                    const float *gamma_lane, double *part, hipStream_t st);
int sum_blocks(int m);
hipError_t launch_fill(float *p, size_t n, float v, hipStream_t st);
hipError_t launch_scale_rows(float *e, const float *scale, int m, int B, hipStream_t st);
hipError_t launch_copy(float *dst, const float *src, size_t n, hipStream_t st);

}  // namespace appga
