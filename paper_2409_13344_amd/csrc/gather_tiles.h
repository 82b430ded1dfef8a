// Host-side construction of the tile forms of A (forward projection) and of
// its transpose (back projection) used by the B > 1 tile kernel
// (k_gather_tiles).  Host code only.
#pragma once

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <cstdint>
#include <vector>

#include "appga_internal.h"

namespace appga {

// Host copy of a DevGatherTiles.
struct HostGatherTiles {
    int n_tiles = 0, tiles_x = 0, n_groups = 0, group_angles = 0, max_windows = 0, n_pslots = 0;
    std::vector<uint32_t> win_off, rec_off, records, rp, word;
    std::vector<int32_t> outs;
    std::vector<uint32_t> parts, reds;   // 4 words each (DevGatherTiles::parts / reds)
};

// Tile form of the transpose for the B > 1 back projection:
// built from the transpose in its stored entry order (pixel rows, rays
// ascending), so each pixel's sum keeps that order.  Every entry becomes a
// pair of words (LDS byte offset of its ray's record in the window, FP32
// value); tv32[k] is the value of transpose entry k exactly as the stored
// type decodes it, so products equal the row kernel's.  The pixels of a tile
// row form two quads (columns 0-3 and 4-7) whose four lists in a group are
// padded to the longest of them with entries of value 0 on the zero record.
// Returns false when no angle grouping fits the kernel's limits (then the
// row kernel is used).
inline bool build_back_tiles(int n, int n_angles, int n_bins, const int64_t *trp, const int32_t *tcol,
                             const float *tv32, HostGatherTiles &bt) {
    const int T = kBackTile;
    const int tx = (n + T - 1) / T;
    const int64_t ntiles = static_cast<int64_t>(tx) * tx;
    const int64_t m = static_cast<int64_t>(n_angles) * n_bins;
    auto pixels_of = [&](int64_t t, std::vector<int> &pix) {
        pix.assign(T * T, -1);
        const int r0 = static_cast<int>(t / tx) * T, c0 = static_cast<int>(t % tx) * T;
        for (int p = 0; p < T * T; ++p) {
            const int r = r0 + p / T, c = c0 + p % T;
            if (r < n && c < n) pix[p] = r * n + c;
        }
    };
    // distinct rays per (tile, angle); most entries of one pixel at one angle
    std::vector<int64_t> stamp(m, -1);
    std::vector<int32_t> cnt(ntiles * n_angles, 0);
    std::vector<int32_t> cpa(static_cast<size_t>(n) * n * n_angles, 0);   // entries per (pixel, angle)
    std::vector<int> pix;
    for (int64_t t = 0; t < ntiles; ++t) {
        pixels_of(t, pix);
        for (int p = 0; p < T * T; ++p) {
            if (pix[p] < 0) continue;
            for (int64_t k = trp[pix[p]]; k < trp[pix[p] + 1]; ++k) {
                const int32_t i = tcol[k];
                const int a = i / n_bins;
                cpa[static_cast<size_t>(pix[p]) * n_angles + a] += 1;
                if (stamp[i] != t) {
                    stamp[i] = t;
                    cnt[t * n_angles + a] += 1;
                }
            }
        }
    }
    // largest angle group whose windows fit kBackSlots and whose word lists
    // (after the quad padding) fit kBackMaxWords per tile and group
    auto max_words = [&](int cand, int ng) {
        int64_t wmax = 0;
        for (int64_t t = 0; t < ntiles; ++t) {
            pixels_of(t, pix);
            for (int g = 0; g < ng; ++g) {
                int64_t wsum = 0;
                for (int qd = 0; qd < T * T / 4; ++qd) {
                    int64_t l = 0;
                    for (int p = 4 * qd; p < 4 * qd + 4; ++p) {
                        if (pix[p] < 0) continue;
                        int64_t c = 0;
                        for (int a = g * cand; a < std::min(n_angles, (g + 1) * cand); ++a)
                            c += cpa[static_cast<size_t>(pix[p]) * n_angles + a];
                        l = std::max(l, c);
                    }
                    wsum += 4 * l * 2;
                }
                wmax = std::max(wmax, wsum);
            }
        }
        return wmax;
    };
    int G = 0;
    for (int cand = n_angles; cand >= 1; --cand) {
        const int ng = (n_angles + cand - 1) / cand;
        int64_t smax = 0;
        for (int64_t t = 0; t < ntiles && smax <= kBackSlots; ++t)
            for (int g = 0; g < ng; ++g) {
                int64_t s = 0;
                for (int a = g * cand; a < std::min(n_angles, (g + 1) * cand); ++a) s += cnt[t * n_angles + a];
                smax = std::max(smax, s);
            }
        if (smax <= kBackSlots && max_words(cand, ng) <= kBackMaxWords) {
            G = cand;
            break;
        }
    }
    if (G == 0) return false;
    const int NG = (n_angles + G - 1) / G;
    bt.n_tiles = static_cast<int>(ntiles);
    bt.tiles_x = tx;
    bt.n_groups = NG;
    bt.group_angles = G;
    bt.max_windows = NG;
    bt.win_off.resize(ntiles + 1);
    for (int64_t t = 0; t <= ntiles; ++t) bt.win_off[t] = static_cast<uint32_t>(t * NG);
    bt.outs.resize(ntiles * 64);
    for (int64_t t = 0; t < ntiles; ++t) {
        pixels_of(t, pix);
        for (int p = 0; p < 64; ++p) bt.outs[t * 64 + p] = pix[p];
    }
    bt.rp.assign(static_cast<size_t>(ntiles) * NG * 64 + 1, 0);
    bt.rec_off.assign(static_cast<size_t>(ntiles) * NG + 1, 0);
    bt.records.clear();
    bt.word.clear();
    std::vector<int32_t> slot_of(m, -1);
    std::vector<int64_t> cur(T * T);
    std::vector<uint32_t> tr;
    const uint32_t pad_word = static_cast<uint32_t>(kBackSlots) * 256u;
    for (int64_t t = 0; t < ntiles; ++t) {
        pixels_of(t, pix);
        tr.clear();
        for (int p = 0; p < T * T; ++p) {
            if (pix[p] < 0) continue;
            for (int64_t k = trp[pix[p]]; k < trp[pix[p] + 1]; ++k)
                if (stamp[tcol[k]] != -2 - t) {
                    stamp[tcol[k]] = -2 - t;
                    tr.push_back(static_cast<uint32_t>(tcol[k]));
                }
        }
        std::sort(tr.begin(), tr.end());
        size_t q = 0;
        for (int g = 0; g < NG; ++g) {
            bt.rec_off[t * NG + g] = static_cast<uint32_t>(bt.records.size());
            int slot = 0;
            while (q < tr.size() && static_cast<int>(tr[q] / n_bins) / G == g) {
                slot_of[tr[q]] = slot++;
                bt.records.push_back(tr[q++]);
            }
        }
        for (int p = 0; p < T * T; ++p) cur[p] = pix[p] < 0 ? 0 : trp[pix[p]];
        for (int g = 0; g < NG; ++g) {
            // entries of pixel p in group g; the four lists of a quad are
            // padded to the same length (the kernel sums a quad in one loop)
            int64_t cntg[T * T];
            std::vector<int64_t> kbeg(T * T);
            for (int p = 0; p < T * T; ++p) {
                kbeg[p] = cur[p];
                int64_t c = 0;
                if (pix[p] >= 0) {
                    const int64_t end = trp[pix[p] + 1];
                    while (cur[p] < end && (tcol[cur[p]] / n_bins) / G == g) {
                        ++cur[p];
                        ++c;
                    }
                }
                cntg[p] = c;
            }
            for (int p = 0; p < T * T; ++p) {
                bt.rp[(t * NG + g) * 64 + p] = static_cast<uint32_t>(bt.word.size());
                const int q0 = p & ~3;
                const int64_t len = std::max(std::max(cntg[q0], cntg[q0 + 1]), std::max(cntg[q0 + 2], cntg[q0 + 3]));
                for (int64_t q = 0; q < len; ++q) {
                    if (q < cntg[p]) {
                        const int64_t k = kbeg[p] + q;
                        uint32_t bits;
                        std::memcpy(&bits, &tv32[k], 4);
                        bt.word.push_back(static_cast<uint32_t>(slot_of[tcol[k]]) * 256u);
                        bt.word.push_back(bits);
                    } else {
                        bt.word.push_back(pad_word);
                        bt.word.push_back(0u);
                    }
                }
            }
        }
    }
    bt.rp.back() = static_cast<uint32_t>(bt.word.size());
    bt.rec_off.back() = static_cast<uint32_t>(bt.records.size());
    return bt.word.size() < (1ull << 31);
}

// Tile form of A for the B > 1 forward projection (rows i = angle * n_bins +
// bin): blocks of kFwdTileAngles consecutive angles x kFwdTileBins
// consecutive bins (slot o = angle offset * kFwdTileBins + bin offset, so a
// quad is four neighbouring bins of one angle).  Blocks whose rays all cross
// no pixel are not tiles: their rays go, 64 to a tile, into tiles without
// windows (sums 0).  Workgroups take parts (a tile or a run of its windows)
// longest first.  A tile's windows partition the pixels its rays cross, taken in
// order along the tile's mean ray direction (estimated from each ray's first
// and last stored pixel) in runs of at most kBackSlots (fewer if a window's
// padded word lists would not fit kBackMaxWords).  Each ray's entries are
// kept in stored order within a window.  v32[k] is the value of entry k
// exactly as the stored type decodes it (FP8: without the row scale, which
// the epilogue applies).  Returns false when a tile fits no window size within
// the kernel's limits.
inline bool build_fwd_tiles(int n, int n_angles, int n_bins, const int64_t *row_ptr, const int32_t *col,
                            const float *v32, HostGatherTiles &ft, int64_t part_windows = -1) {
    const int TA = kFwdTileAngles, TB = kFwdTileBins;
    static_assert(kFwdTileAngles * kFwdTileBins == 64, "64 slots per tile");
    const int64_t d = static_cast<int64_t>(n) * n;
    // the tiles' rays
    std::vector<std::array<int64_t, 64>> tiles, blocks;
    {
        std::vector<int64_t> empty;
        for (int a0 = 0; a0 < n_angles; a0 += TA)
            for (int b0 = 0; b0 < n_bins; b0 += TB) {
                std::array<int64_t, 64> blk;
                bool any = false;
                for (int o = 0; o < 64; ++o) {
                    const int a = a0 + o / TB, b = b0 + o % TB;
                    blk[o] = (a < n_angles && b < n_bins) ? static_cast<int64_t>(a) * n_bins + b : -1;
                    if (blk[o] >= 0 && row_ptr[blk[o] + 1] > row_ptr[blk[o]]) any = true;
                }
                if (any) {
                    blocks.push_back(blk);
                } else {
                    for (int o = 0; o < 64; ++o)
                        if (blk[o] >= 0) empty.push_back(blk[o]);
                }
            }
        for (size_t i = 0; i < empty.size(); i += 64) {
            std::array<int64_t, 64> t;
            t.fill(-1);
            for (size_t o = 0; o < 64 && i + o < empty.size(); ++o) t[o] = empty[i + o];
            tiles.push_back(t);
        }
        tiles.insert(tiles.end(), blocks.begin(), blocks.end());
    }
    const int64_t ntiles = static_cast<int64_t>(tiles.size());
    ft = HostGatherTiles();
    ft.n_tiles = static_cast<int>(ntiles);
    ft.win_off.assign(ntiles + 1, 0);
    ft.outs.assign(ntiles * 64, -1);
    ft.rec_off.push_back(0);
    const uint32_t pad_word = static_cast<uint32_t>(kBackSlots) * 256u;
    std::vector<int64_t> stamp(d, -1);
    std::vector<int32_t> win_of(d, -1), slot_of(d, -1);
    std::vector<int32_t> pixels;
    std::vector<double> key;
    std::vector<int32_t> order;
    for (int64_t t = 0; t < ntiles; ++t) {
        const int64_t *ray = tiles[t].data();
        for (int o = 0; o < 64; ++o) ft.outs[t * 64 + o] = ray[o] < 0 ? -1 : static_cast<int32_t>(ray[o]);
        // mean direction and the pixels the tile's rays cross
        double dy = 0.0, dx = 0.0, ry = 0.0, rx = 0.0;
        pixels.clear();
        for (int o = 0; o < 64; ++o) {
            if (ray[o] < 0) continue;
            const int64_t k0 = row_ptr[ray[o]], k1 = row_ptr[ray[o] + 1];
            for (int64_t k = k0; k < k1; ++k)
                if (stamp[col[k]] != t) {
                    stamp[col[k]] = t;
                    pixels.push_back(col[k]);
                }
            if (k1 - k0 >= 2) {
                double vy = col[k1 - 1] / n - col[k0] / n, vx = col[k1 - 1] % n - col[k0] % n;
                const double len = std::sqrt(vy * vy + vx * vx);
                if (len == 0.0) continue;
                vy /= len;
                vx /= len;
                if (ry == 0.0 && rx == 0.0) {
                    ry = vy;
                    rx = vx;
                }
                if (vy * ry + vx * rx < 0.0) {
                    vy = -vy;
                    vx = -vx;
                }
                dy += vy;
                dx += vx;
            }
        }
        if (dy == 0.0 && dx == 0.0) dx = 1.0;
        const int64_t P = static_cast<int64_t>(pixels.size());
        key.resize(P);
        order.resize(P);
        for (int64_t i = 0; i < P; ++i) {
            key[i] = (pixels[i] / n) * dy + (pixels[i] % n) * dx;
            order[i] = static_cast<int32_t>(i);
        }
        std::sort(order.begin(), order.end(), [&](int32_t u, int32_t v) {
            return key[u] != key[v] ? key[u] < key[v] : pixels[u] < pixels[v];
        });
        // largest window size whose windows fit the limits
        int S = kBackSlots, nw = 0;
        std::vector<int64_t> cntw;
        for (; S >= 8; S -= 8) {
            nw = static_cast<int>((P + S - 1) / S);
            for (int64_t i = 0; i < P; ++i) win_of[pixels[order[i]]] = static_cast<int32_t>(i / S);
            cntw.assign(static_cast<size_t>(nw) * 64, 0);
            for (int o = 0; o < 64; ++o) {
                if (ray[o] < 0) continue;
                for (int64_t k = row_ptr[ray[o]]; k < row_ptr[ray[o] + 1]; ++k) cntw[win_of[col[k]] * 64 + o] += 1;
            }
            bool fits = true;
            for (int wi = 0; wi < nw && fits; ++wi) {
                int64_t words = 0;
                for (int q0 = 0; q0 < 64; q0 += 4) {
                    int64_t l = 0;
                    for (int o = q0; o < q0 + 4; ++o) l = std::max(l, cntw[wi * 64 + o]);
                    words += 4 * l * 2;
                }
                fits = words <= kBackMaxWords;
            }
            if (fits) break;
        }
        if (S < 8) return false;
        ft.max_windows = std::max(ft.max_windows, nw);
        ft.win_off[t] = static_cast<uint32_t>(ft.rec_off.size() - 1);
        for (int wi = 0; wi < nw; ++wi) {
            const int64_t p0 = static_cast<int64_t>(wi) * S, p1 = std::min<int64_t>(P, p0 + S);
            for (int64_t i = p0; i < p1; ++i) {
                slot_of[pixels[order[i]]] = static_cast<int32_t>(i - p0);
                ft.records.push_back(static_cast<uint32_t>(pixels[order[i]]));
            }
            ft.rec_off.push_back(static_cast<uint32_t>(ft.records.size()));
            for (int o = 0; o < 64; ++o) {
                ft.rp.push_back(static_cast<uint32_t>(ft.word.size()));
                const int q0 = o & ~3;
                int64_t len = 0;
                for (int u = q0; u < q0 + 4; ++u) len = std::max(len, cntw[wi * 64 + u]);
                int64_t c = 0;
                if (ray[o] >= 0)
                    for (int64_t k = row_ptr[ray[o]]; k < row_ptr[ray[o] + 1]; ++k) {
                        if (win_of[col[k]] != wi) continue;
                        uint32_t bits;
                        std::memcpy(&bits, &v32[k], 4);
                        ft.word.push_back(static_cast<uint32_t>(slot_of[col[k]]) * 256u);
                        ft.word.push_back(bits);
                        ++c;
                    }
                for (; c < len; ++c) {
                    ft.word.push_back(pad_word);
                    ft.word.push_back(0u);
                }
            }
        }
    }
    ft.win_off[ntiles] = static_cast<uint32_t>(ft.rec_off.size() - 1);
    ft.rp.push_back(static_cast<uint32_t>(ft.word.size()));
    // Workgroup parts: one workgroup sums a tile unless the tile has more than
    // K windows; then its windows are split into near-equal runs (partial sums
    // added by a reduction).  part_windows < 0: K about the mean windows per
    // workgroup slot of the device (two per CU); 0: no splitting; else K.
    const int64_t nwin = static_cast<int64_t>(ft.rec_off.size()) - 1;
    const int64_t K = part_windows < 0 ? std::max<int64_t>(4, (nwin + kFwdSlots - 1) / kFwdSlots + 1)
                      : part_windows == 0 ? std::numeric_limits<int64_t>::max() : part_windows;
    for (int64_t t = 0; t < ntiles; ++t) {
        const int64_t w0 = ft.win_off[t], nw = ft.win_off[t + 1] - w0;
        const int64_t np = std::max<int64_t>(1, (nw + K - 1) / K);
        if (np > 1) {
            ft.reds.insert(ft.reds.end(), {static_cast<uint32_t>(t), static_cast<uint32_t>(ft.n_pslots),
                                           static_cast<uint32_t>(np), 0u});
        }
        for (int64_t p = 0; p < np; ++p) {
            const uint32_t slot = np > 1 ? static_cast<uint32_t>(ft.n_pslots + p) : kNoSlot;
            ft.parts.insert(ft.parts.end(), {static_cast<uint32_t>(t), static_cast<uint32_t>(w0 + p * nw / np),
                                             static_cast<uint32_t>(w0 + (p + 1) * nw / np), slot});
        }
        if (np > 1) ft.n_pslots += static_cast<int>(np);
    }
    // dispatch order: longest parts first (the device starts workgroups in
    // index order), so that short parts fill the slots the long ones free
    {
        const size_t np = ft.parts.size() / 4;
        std::vector<size_t> ord(np);
        std::iota(ord.begin(), ord.end(), size_t{0});
        std::stable_sort(ord.begin(), ord.end(), [&](size_t u, size_t v) {
            return ft.parts[4 * u + 2] - ft.parts[4 * u + 1] > ft.parts[4 * v + 2] - ft.parts[4 * v + 1];
        });
        std::vector<uint32_t> sorted(ft.parts.size());
        for (size_t i = 0; i < np; ++i)
            for (int k = 0; k < 4; ++k) sorted[4 * i + k] = ft.parts[4 * ord[i] + k];
        ft.parts.swap(sorted);
    }
    return ft.word.size() < (1ull << 31);
}

}  // namespace appga
