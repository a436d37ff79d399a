// bz_host.hpp -- host-side argument checks and decision constants shared by
// every entry point of libbinarize.  Plain C++ with no HIP dependency, so the
// CPU test suite can build it with g++ under AddressSanitizer and UBSan.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <cmath>

#include "binarize.h"
#include "bz_common.hpp"

namespace bz {

// ------------------------------------------------------------ parameters
//
// Accepted threshold parameters (Sec. 1, Eq. 4 and the Niblack rule).  The
// kernels take sqrt(D) in fp32 (relative error below 1.35e-7: the rounding
// of D to fp32 plus one ulp of the hardware square root) and everything
// else that can move the Sauvola threshold in fp64, so the only sizeable
// error in t is m |k| s / R * 1.35e-7 <= (|k| / R) * 2.9e-3, with
// m s <= 21117 for 8-bit data (s^2 <= m (255 - m)).  With |k| <= 1 and
// R >= 64 that stays below 4.5e-5, and |t| stays below 1024, where the fp32
// t plane adds at most 3.1e-5 of rounding.  The Niblack decision
// n f - S1 < k sqrt(D) is fp32 with an exact left side; its error is below
// |k| s * 1.9e-7 <= 2.5e-5.  Outside this range the 1e-4 bar would no longer
// hold, so such parameters are refused with BZ_ERR_PARAM.
constexpr float kMaxAbsK = 1.0f;
constexpr float kMinSauvolaR = 64.0f;

inline int check_params(int rule, float k, float R) {
    if (rule != BZ_SAUVOLA && rule != BZ_NIBLACK) return BZ_ERR_RULE;
    if (!std::isfinite(k) || !(std::fabs(k) <= kMaxAbsK)) return BZ_ERR_PARAM;
    if (!std::isfinite(R) || !(R > 0.0f)) return BZ_ERR_PARAM;
    if (rule == BZ_SAUVOLA && !(R >= kMinSauvolaR)) return BZ_ERR_PARAM;
    return BZ_OK;
}

inline int check_window(int win) { return (win < 1 || win > 255) ? BZ_ERR_WINDOW : BZ_OK; }

// Constants of the decision forms, in the precision the kernels use.
struct Decision {
    int rule;          // BZ_SAUVOLA, or BZ_NIBLACK (also for Sauvola with k == 0)
    float k;           // Niblack: t = m + k s
    double c1, c2;     // Sauvola: t = m (c1 + c2 s), c1 = 1 - k, c2 = k / R
    double c1n, c2n2;  // whole windows (n = win^2): c1 / n and c2 / n^2
};

inline Decision make_decision(int rule, float k, float R, int win) {
    Decision d;
    // Sauvola with k = 0 is t = m, the Niblack rule with k = 0, whose form
    // decides exact ties exactly.
    d.rule = (rule == BZ_SAUVOLA && k == 0.0f) ? BZ_NIBLACK : rule;
    d.k = k;
    d.c1 = 1.0 - (double)k;
    d.c2 = (double)k / (double)R;
    const double n = (double)win * (double)win;
    d.c1n = d.c1 / n;
    d.c2n2 = d.c2 / (n * n);
    return d;
}

// ------------------------------------------------------------ memory regions

// H rows of `len` bytes, `pitch` bytes apart, starting at `base`.
struct Region {
    uintptr_t base;
    int64_t rows;
    int64_t pitch;
    int64_t len;
};

inline uintptr_t region_end(const Region &r) {
    return r.rows < 1 ? r.base : r.base + (uintptr_t)((r.rows - 1) * r.pitch + r.len);
}

// Floor division for a positive divisor.
inline int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// True if some byte lies in both regions (each region's own rows are
// disjoint: pitch >= len, or a single row).  Exact for strided layouts, so
// two crops of one buffer whose rows interleave without touching are
// accepted.  Linear in the rows of the shorter region.
inline bool regions_overlap(const Region &a, const Region &b) {
    if (a.rows < 1 || b.rows < 1 || a.len < 1 || b.len < 1) return false;
    if (!(a.base < region_end(b) && b.base < region_end(a))) return false;
    const Region &s = a.rows <= b.rows ? a : b;  // walk the shorter one
    const Region &t = a.rows <= b.rows ? b : a;
    const int64_t tp = t.rows > 1 ? t.pitch : t.len;
    for (int64_t i = 0; i < s.rows; ++i) {
        // row i of s covers [x0, x0 + s.len) relative to t.base
        const int64_t x0 = (int64_t)(s.base - t.base) + i * s.pitch;
        // rows j of t with j tp < x0 + s.len and x0 < j tp + t.len
        int64_t jlo = floor_div(x0 - t.len, tp) + 1;
        int64_t jhi = floor_div(x0 + s.len - 1, tp);
        if (jlo < 0) jlo = 0;
        if (jhi > t.rows - 1) jhi = t.rows - 1;
        if (jlo <= jhi) return true;
    }
    return false;
}

// ------------------------------------------------------------ images

// One page as the caller describes it; pitches are bytes between rows.
struct ImageDesc {
    const uint8_t *img;
    uint8_t *out;
    int H, W, C;
    int64_t pitch_in, pitch_out;
};

inline Region input_region(const ImageDesc &d) {
    return Region{(uintptr_t)d.img, d.H, d.pitch_in, (int64_t)d.W * d.C};
}
inline Region output_region(const ImageDesc &d) { return Region{(uintptr_t)d.out, d.H, d.pitch_out, d.W}; }

// Shape, channels, pitches and size of a page, and its output must not
// overlap its input.  A pitch of 0 means rows are contiguous; it is replaced
// by W * C (input) or W (output).
inline int check_image(ImageDesc &d) {
    if (!d.img || !d.out) return BZ_ERR_NULL;
    if (d.H < 1 || d.W < 1) return BZ_ERR_SHAPE;
    if (d.C != 1 && d.C != 3) return BZ_ERR_CHANNELS;
    if ((int64_t)d.H * d.W * d.C >= ((int64_t)1 << 31)) return BZ_ERR_SHAPE;
    if (d.pitch_in == 0) d.pitch_in = (int64_t)d.W * d.C;
    if (d.pitch_out == 0) d.pitch_out = d.W;
    if (d.pitch_in < (int64_t)d.W * d.C || d.pitch_out < d.W) return BZ_ERR_SHAPE;
    if (d.pitch_in >= ((int64_t)1 << 40) || d.pitch_out >= ((int64_t)1 << 40)) return BZ_ERR_SHAPE;
    if (regions_overlap(input_region(d), output_region(d))) return BZ_ERR_ALIAS;
    return BZ_OK;
}

// Everything one page of the tile kernel needs checked before a launch.
inline int check_page(ImageDesc &d, int win, float k, float R, int rule) {
    int rc = check_image(d);
    if (rc) return rc;
    if ((rc = check_window(win))) return rc;
    return check_params(rule, k, R);
}

// ------------------------------------------------------------ tile plans

// Default tile for a page on a GPU with `cus` compute units: 256 columns
// when the window fits, and a height that gives every CU as many tiles as
// the LDS footprint lets it run at once, at least 64 rows so the win
// start-up rows stay a modest share of a tile.  A page too small to give
// every CU one 64-row tile gets shorter tiles instead (down to 8 rows, about
// one per CU): its launch is then bound by one workgroup's latency, which
// shorter tiles cut.
inline void pick_default_tile(int H, int W, int C, int win, int cus, int *tw, int *th) {
    const int w = tile_fits(256, win, C) ? 256 : 128;
    int per_cu = kMaxLds / tile_lds_bytes(w, win, C);
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 8) per_cu = 8;  // 8 x 4 waves fill a CU
    const long target = (long)cus * per_cu;
    const long tiles_x = (W + w - 1) / w;
    const long rows = (long)H * tiles_x;  // tile rows of the page, all columns of tiles
    auto r8 = [](long v) { return (v + kRowsPerStep - 1) / kRowsPerStep * kRowsPerStep; };
    long h = r8((rows + target - 1) / target);
    const long hmin = 64;
    if (h < hmin) h = hmin;
    if (tiles_x * ((H + hmin - 1) / hmin) < cus) h = r8((rows + cus - 1) / cus);  // small page
    if (h > 4096) h = 4096;
    *tw = w;
    *th = (int)h;
}

// Whether a single-page launch of this tile shape takes the blocks layout:
// the window makes it eligible (gray_blocks) and the page has more tiles than
// the ring layout's occupancy runs at once on `cus` CUs.  With fewer tiles
// the ring's occupancy costs nothing and its start-up (one pass over the
// first win rows, no barriers between blocks) is the cheaper one.
inline bool use_blocks(int H, int W, int C, int win, int tile_w, int tile_h, int cus) {
    if (!gray_blocks(tile_w, win, C)) return false;
    const long tiles = (long)((W + tile_w - 1) / tile_w) * ((H + tile_h - 1) / tile_h);
    const long ring_slots = (long)cus * (kMaxLds / ring_layout_lds(tile_w, win));
    return tiles > ring_slots;
}

inline int check_tile(int tile_w, int tile_h, int win, int C) {
    if (tile_w != 128 && tile_w != 256) return BZ_ERR_TILE;
    if (tile_h < kRowsPerStep || tile_h > 4096 || tile_h % kRowsPerStep) return BZ_ERR_TILE;
    if (!tile_fits(tile_w, win, C)) return BZ_ERR_TILE;
    return BZ_OK;
}

// Kernel arguments of one checked page for a given tile shape.  The page
// must have passed check_page (pitches filled in) and the tile check_tile
// (or the batch's own tile check, with allow_blocks false).
inline PageArgs page_args(const ImageDesc &d, int win, float k, float R, int rule, int tile_w, int tile_h,
                          bool allow_blocks = true) {
    const Decision q = make_decision(rule, k, R, win);
    PageArgs a;
    a.img = d.img;
    a.out = d.out;
    a.gray = nullptr;
    a.s1 = a.s2 = a.n = nullptr;
    a.t = nullptr;
    a.pitch_in = d.pitch_in;
    a.pitch_out = d.pitch_out;
    a.c1 = q.c1;
    a.c2 = q.c2;
    a.c1n = q.c1n;
    a.c2n2 = q.c2n2;
    a.H = d.H;
    a.W = d.W;
    a.win = win;
    a.lo = win / 2;
    a.hi = win - 1 - a.lo;
    a.k = q.k;
    a.tile_h = tile_h;
    a.tiles_x = (d.W + tile_w - 1) / tile_w;
    a.n_tiles = a.tiles_x * ((d.H + tile_h - 1) / tile_h);
    a.rp = ring_pitch(tile_w, win);
    a.depth = ring_rows(tile_w, win, d.C, allow_blocks);
    a.blocks = gray_blocks(tile_w, win, d.C, allow_blocks) ? 1 : 0;
    // (pitches below 2^28 keep the per-thread offsets of the aligned and
    // wide bodies from a step's first row, at most 8 rows plus a row's bytes,
    // in 32 bits)
    a.small_pitch = (d.pitch_in < ((int64_t)1 << 28) && d.pitch_out < ((int64_t)1 << 28)) ? 1 : 0;
    a.row_aligned = (a.small_pitch && ((uintptr_t)d.img & 15) == 0 && d.pitch_in % 16 == 0 &&
                     ((int64_t)d.W * d.C) % 16 == 0 && ((uintptr_t)d.out & 7) == 0 && d.pitch_out % 8 == 0)
                        ? 1
                        : 0;
    return a;
}

// ------------------------------------------------------------ batch plans
//
// Pages run in launches keyed by kernel group and occupancy class, launched
// one after another on the caller's stream.  Groups 0 and 1 hold the pages
// in the ring layout with 256- and 128-column tiles, groups 2..5 the gray
// pages in the blocks layout (those whose ring would exceed a quarter of
// the CU's LDS), one group per tile variant: 2 + (tile_w == 256) * 2 + rule.
// Tile variant of a ring page within its group, 0..3:
// (channels == 3) * 2 + rule.  The class of a page is the highest number of
// workgroups per CU (4, 3, 2, 1) whose share of the LDS holds its tile; a
// launch reserves that share per workgroup, so pages of narrow windows run
// at four workgroups per CU even when wider ones share the batch.
constexpr int kGroups = 6;
constexpr int kClasses = 4;
constexpr int kLaunches = kGroups * kClasses;  // launch key: group * kClasses + class
inline int kind_of(int channels, int rule) { return (channels == 3) * 2 + rule; }
inline bool blk_group(int g) { return g >= 2; }
inline int group_of(int tile_w, int rule, bool blocks) {
    return blocks ? 2 + (tile_w == 256) * 2 + rule : (tile_w == 256 ? 0 : 1);
}

// LDS the batch kernels declare statically (the item slot), rounded up.
constexpr int kStaticLds = 64;
// Dynamic LDS of a workgroup of class c (kClasses - c workgroups per CU),
// a multiple of 16 bytes.
inline int class_lds(int c) { return (kMaxLds / (kClasses - c) - kStaticLds) & ~15; }
// Class of a tile that needs `lds` bytes (-1: more than one CU holds).
inline int class_of(int lds) {
    for (int c = 0; c < kClasses; ++c)
        if (lds <= class_lds(c)) return c;
    return -1;
}

// Tile, layout and LDS need of one page within the batch's LDS cap: the
// caller's width if it fits, else 256 columns when the window allows, else
// 128; tile_h 128 unless given.  Gray pages whose ring would exceed a
// quarter of the CU's LDS take the blocks layout (as in the single-page
// kernel, which also weighs the page's tile count: in a batch the pages share
// the GPU, so occupancy always counts), every other page the ring.
inline int page_tile(const bz_page &p, int lds_cap, int *tw, int *th, bool *blk, int *lds) {
    auto fits = [&](int w) {
        return tile_fits(w, p.win, p.channels) && tile_lds_bytes(w, p.win, p.channels) <= lds_cap;
    };
    int w = p.tile_w, h = p.tile_h;
    if (w == 0) w = fits(256) ? 256 : 128;
    if (h == 0) h = 128;
    if (w != 128 && w != 256) return BZ_ERR_TILE;
    if (h < kRowsPerStep || h > 4096 || h % kRowsPerStep) return BZ_ERR_TILE;
    if (!fits(w)) return BZ_ERR_TILE;
    *tw = w;
    *th = h;
    *blk = gray_blocks(w, p.win, p.channels);
    *lds = tile_lds_bytes(w, p.win, p.channels);
    return BZ_OK;
}

}  // namespace bz
