// Host-side construction of the tile form of the stored transpose used by the
// B > 1 back projection kernel (k_back_tiles).  Host code only.
#pragma once

#include <algorithm>
#include <cstring>
#include <cstdint>
#include <vector>

#include "appga_internal.h"

namespace appga {

// Tile form of the transpose for the B > 1 back projection (DevBackTiles):
// built from the transpose in its stored entry order (pixel rows, rays
// ascending), so each pixel's sum keeps that order.  tcode[k] is the stored
// value code of transpose entry k (16- and 8-bit types), tv32[k] its FP32
// value (f32).  Returns false when no angle grouping fits the kernel's limits
// (then the row kernel is used).
struct HostBackTiles {
    int tiles_x = 0, n_groups = 0, group_angles = 0;
    std::vector<uint32_t> rp, word, ray_off, rays;
};

inline bool build_back_tiles(int n, int n_angles, int n_bins, const int64_t *trp, const int32_t *tcol,
                             const uint32_t *tcode, const float *tv32, bool f32, HostBackTiles &bt) {
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
    int max_pa = 1;
    std::vector<int> pix;
    for (int64_t t = 0; t < ntiles; ++t) {
        pixels_of(t, pix);
        for (int p = 0; p < T * T; ++p) {
            if (pix[p] < 0) continue;
            int prev = -1, run = 0;
            for (int64_t k = trp[pix[p]]; k < trp[pix[p] + 1]; ++k) {
                const int32_t i = tcol[k];
                const int a = i / n_bins;
                run = (a == prev) ? run + 1 : 1;
                prev = a;
                max_pa = std::max(max_pa, run);
                if (stamp[i] != t) {
                    stamp[i] = t;
                    cnt[t * n_angles + a] += 1;
                }
            }
        }
    }
    // largest angle group whose windows fit kBackSlots, with at most 64 (padded)
    // entries per pixel and group, at most kBackMaxWords entries per tile and
    // group (bounded by 64 pixels x (G max_pa + 3) after the pair padding) and
    // at most kBackMaxGroups groups
    int G = 0;
    for (int cand = std::min(n_angles, (64 - 3) / max_pa); cand >= 1; --cand) {
        const int ng = (n_angles + cand - 1) / cand;
        if (ng > kBackMaxGroups) break;
        if (64 * (cand * max_pa + 3) * (f32 ? 2 : 1) > kBackMaxWords) continue;
        int64_t smax = 0;
        for (int64_t t = 0; t < ntiles && smax <= kBackSlots; ++t)
            for (int g = 0; g < ng; ++g) {
                int64_t s = 0;
                for (int a = g * cand; a < std::min(n_angles, (g + 1) * cand); ++a) s += cnt[t * n_angles + a];
                smax = std::max(smax, s);
            }
        if (smax <= kBackSlots) {
            G = cand;
            break;
        }
    }
    if (G == 0) return false;
    const int NG = (n_angles + G - 1) / G;
    bt.tiles_x = tx;
    bt.n_groups = NG;
    bt.group_angles = G;
    bt.rp.assign(static_cast<size_t>(ntiles) * NG * 64 + 1, 0);
    bt.ray_off.assign(static_cast<size_t>(ntiles) * NG + 1, 0);
    bt.rays.clear();
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
            bt.ray_off[t * NG + g] = static_cast<uint32_t>(bt.rays.size());
            int slot = 0;
            while (q < tr.size() && static_cast<int>(tr[q] / n_bins) / G == g) {
                slot_of[tr[q]] = slot++;
                bt.rays.push_back(tr[q++]);
            }
        }
        for (int p = 0; p < T * T; ++p) cur[p] = pix[p] < 0 ? 0 : trp[pix[p]];
        for (int g = 0; g < NG; ++g) {
            // entries of pixel p in group g; the two pixels of a pair (2i, 2i+1)
            // are padded to the same multiple of 4 (the kernel sums a pair in one loop)
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
                const int64_t padded = (std::max(cntg[p], cntg[p ^ 1]) + 3) / 4 * 4;
                for (int64_t q = 0; q < padded; ++q) {
                    if (q < cntg[p]) {
                        const int64_t k = kbeg[p] + q;
                        const uint32_t code = f32 ? 0u : tcode[k];
                        bt.word.push_back(static_cast<uint32_t>(slot_of[tcol[k]]) * 256u | code << 16);
                        if (f32) {
                            uint32_t bits;
                            std::memcpy(&bits, &tv32[k], 4);
                            bt.word.push_back(bits);
                        }
                    } else {
                        bt.word.push_back(pad_word);
                        if (f32) bt.word.push_back(0u);
                    }
                }
            }
        }
    }
    bt.rp.back() = static_cast<uint32_t>(bt.word.size());
    bt.ray_off.back() = static_cast<uint32_t>(bt.rays.size());
    return bt.word.size() < (1ull << 31);
}

}  // namespace appga
