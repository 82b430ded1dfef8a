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

// Tile form of a sparse operator for batches (B > 1).  The outputs are cut
// into tiles of 64; a tile's sums run over windows, each a list of at most
// kBackSlots input records (records[rec_off[w] + s] is the input in slot s)
// that the kernel stages in LDS.  For window w the entries of tile slot o are
// words [rp[w*64 + o], rp[w*64 + o + 1]): pairs (slot * 256, FP32 value),
// where slot kBackSlots is a record of zeros the kernel keeps in LDS.  The
// lists of slots 4i .. 4i+3 (a quad) have equal lengths (padded with zero
// entries).  Tile t owns windows [win_off[t], win_off[t+1]) and its slot o
// is output outs[t*64 + o] (-1: none).
//  - Back projection A^T e: tiles of kBackTile x kBackTile pixels (slot =
//    row-major position in the tile, outputs = pixels r*N + c), windows = the
//    groups of `group_angles` consecutive angles (records = the rays that
//    cross the tile), every tile has n_groups windows.
//  - Forward projection A x: tiles of kFwdTileAngles angles x kFwdTileBins
//    bins (slot = angle * kFwdTileBins + bin within the tile, outputs = rays),
//    windows = runs of the pixels the tile's rays cross, ordered along the
//    tile's mean ray direction (records = pixels).
// Each output's entries keep their stored order within a window.  Device
// pointers.
constexpr int kBackTile = 8;
constexpr int kFwdTileAngles = 8;
constexpr int kFwdTileBins = 8;
constexpr int kFwdSlots = 512;       // tile workgroups resident at once (two per CU on 256 CUs)
constexpr int kBackSlots = 96;       // records per window (slot kBackSlots is the zero record)
constexpr int kBackMaxWords = 2048;  // words of one tile in one window (padded)

struct DevGatherTiles {
    int valid = 0;
    int n_tiles = 0;
    int tiles_x = 0;                 // pixel tiles per image row (back projection), else 0
    int n_groups = 0, group_angles = 0;  // back projection: windows per tile, angles per window
    int max_windows = 0;             // most windows of one tile
    uint32_t *win_off = nullptr;     // [n_tiles + 1]
    uint32_t *rec_off = nullptr;     // [n_windows + 1]
    uint32_t *records = nullptr;     // [n_records]
    uint32_t *rp = nullptr;          // [n_windows * 64 + 1]
    uint32_t *word = nullptr;        // [n_words]
    int32_t *outs = nullptr;         // [n_tiles * 64]
    // forward: the workgroups' parts {tile, first window, end window, partial
    // slot or kNoSlot}; a tile whose windows are split between several parts
    // gets one partial-sum slot per part (consecutive), and reds lists those
    // tiles {tile, first slot, parts, 0} for the reduction that finishes them
    uint4 *parts = nullptr;
    uint4 *reds = nullptr;
    int n_parts = 0, n_reds = 0, n_pslots = 0;
    int64_t n_windows = 0, n_records = 0, n_words = 0;
    int64_t bytes = 0;
};
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

enum GatherMode { GM_BACK = 0, GM_FWD = 1 };

struct GatherTileArgs {
    const uint32_t *win_off;
    const uint32_t *rec_off;
    const uint32_t *records;
    const uint32_t *rp;
    const uint32_t *word;
    const int32_t *outs;
    uint32_t n_records;     // length of records
    uint32_t n_words;       // length of word
    int n_tiles;
    int tiles_x;            // > 0: square grid of pixel tiles (the XCD remap applies)
    int xcd_remap;
    int split;              // GM_BACK: workgroups per tile; workgroup s sums windows [s W / split, (s+1) W / split)
    int n_in;               // input records per chunk (rays for A^T e, pixels for A x)
    int n_out;              // outputs per chunk
    const float *in;        // [chunk][n_in][64] (lane layout)
    float *out;             // GM_BACK: [split][chunk][n_out][64] partial sums
    const uint4 *parts;     // GM_FWD: workgroup parts (then blockIdx.x is a part), or null
    const uint4 *reds;      // GM_FWD: tiles finished by the reduction
    int n_pslots;           // GM_FWD: partial-sum slots (64 x 64 values per chunk each)
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
    float *tile_part;       // forward tiles with split tiles: [chunks][n_pslots][64][64] scratch
    // B = 1 with a half-stored matrix (quarter-turn symmetry): rows i >= sym_half
    // are stored row i - sym_half with every column j mapped to rho(j),
    // rho(r, c) = (c, N - 1 - r), N = img_n; 0 = the full matrix is stored
    int sym_half;
    int img_n;
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
    // B = 1 with a half-stored transpose (quarter-turn symmetry): A^T e at pixel j
    // is stored row j with e, plus stored row rho^{-1}(j) with e shifted by sym_half
    // (rho^{-1}(r, c) = (N - 1 - c, r)); 0 = the full transpose is stored
    int sym_half;
};

// One AFPPA iteration after the ratio forward projection and the back
// projection (Section 4.3).  The duals (b, c) are one vector of 6 components
// per pixel and solve: b as components 0, 1 ((I (x) D) and (D (x) I) groups),
// c as components 2..5 (the four blocks of B2), each component a plane of d
// values (component-major: index k * d + j), in the layout of Bp (plain for
// Bp == 1, else the lane layout of a vector of length 6 d).
struct AfppaArgs {
    int n;                     // image side N (d = N * N)
    int B;                     // solves
    int Bp;                    // 1, or the padded lane count (multiple of 64)
    const float *gf;           // A^T e as gf_split partial sums [gf_split][d][Bp], added in order
    int gf_split;
    float *f;                  // [d] f^k in, f^{k+1} out
    const float *ft;           // [d] f~^k
    float *ft_next;            // [d] f~^{k+1}
    float *w;                  // [d] 2 f^{k+1} - f~^k (primal writes, dual reads)
    float *y;                  // [6 d] duals (b^k, c^k) in, (b^{k+1}, c^{k+1}) out (dual)
    float *ybar;               // [6 d] extrapolated duals: read by the primal, rewritten by the dual
    const float *lam;          // [d] Lambda
    const LaneParams *lp;      // [Bp]
    const float *theta_next;   // [Bp] theta_{k+1}
    int pmode;                 // PM_EM or PM_FIXED
    // max of P at f^k per solve as kAfppaPmSlots partial maxima [slot][Bp] (FP32 bits
    // of values >= 0): the primal accumulates them, the dual reads them and clears
    // the set of the next iteration
    unsigned *pmax_acc;
    const unsigned *pmax_in;
    unsigned *pmax_clear;
    double *re_part;           // primal: [blocks][Bp][2] sum (f^{k+1} - f^k)^2, sum (f^{k+1})^2 (or null)
};

// Space-invariant Gaussian PSF H (Section 4.1): one separable pass along the
// image columns (axis 0: out(r, c) = sum_t w_t in(r, c + t - R)) or rows (axis 1),
// zero outside the image.  `in` holds n_parts partial sums [n_parts][d][Bp]
// added in order before the blur (n_parts = 1 for a plain image).  Layout of Bp.
constexpr int kPsfMaxTaps = 65;
hipError_t launch_psf_pass(const float *in, int n_parts, float *out, int n, int B, int Bp, int axis,
                           const float *taps, int R, hipStream_t st);
// H applied to the sum of n_parts partial sums: the pass along axis 0 into tmp,
// then along axis 1 into out; for batches with R <= 4 both passes run in one
// launch with the same arithmetic (tmp unused).
hipError_t launch_psf_blur(const float *in, int n_parts, float *tmp, float *out, int n, int B, int Bp,
                           const float *taps, int R, hipStream_t st);

constexpr int kAfppaPmSlots = 32;

// Workgroups of the AFPPA kernels (RE partial sums per workgroup).
int afppa_blocks(int n, int Bp);
hipError_t launch_afppa_primal(const AfppaArgs &a, hipStream_t st);
hipError_t launch_afppa_dual(const AfppaArgs &a, hipStream_t st);

// B > 1 back projection out = A^T e over the pixel tiles (lane layout, Bp / 64
// chunks, `split` partial sums).
hipError_t launch_back_tiles(const DevGatherTiles &bt, int vtype, int n, int m, int Bp, int xcd_remap,
                             int split, const float *e, float *out, hipStream_t st);
// Workgroups per tile for the back projection (enough workgroups to put two
// on every CU).
int back_tiles_split(const DevGatherTiles &bt);
// B > 1 forward projection over the ray tiles with the epilogue of `fa`
// (FM_PROJ or FM_RATIO), fa.Bp / 64 chunks; fa.tile_part must hold
// fwd_tile_part_floats(ft, fa.Bp) floats when the tile form splits tiles.
hipError_t launch_fwd_tiles(const DevGatherTiles &ft, int vtype, const FwdArgs &fa, hipStream_t st);
inline size_t fwd_tile_part_floats(const DevGatherTiles &ft, int Bp) {
    return static_cast<size_t>(ft.n_pslots) * 64 * static_cast<size_t>(Bp);
}

// Serving helpers (kernels.hip).

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
