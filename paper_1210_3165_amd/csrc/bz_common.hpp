// bz_common.hpp -- launch arguments shared by the host dispatcher and the
// gfx950 kernels of libbinarize.
#pragma once
#include <stdint.h>

namespace bz {

// Workgroup shape of the tile kernel: 512 threads (8 wave64s).  The vertical
// pass gives every thread one LDS column; the horizontal pass gives each of
// the RB output rows of a step TPR = 32 threads.
constexpr int kThreads = 512;
constexpr int kRowsPerStep = 16;                   // RB
constexpr int kThreadsPerRow = kThreads / kRowsPerStep;  // TPR = 32
constexpr int kMaxCols = kThreads;                 // LDS columns per tile
constexpr int kMaxLds = 160 * 1024;                // gfx950 LDS per workgroup

// One page as the tile kernel sees it.  All geometry that depends only on the
// page and the tile shape is computed once on the host.
struct PageArgs {
    const uint8_t *img;  // H x W x C, row pitch W*C
    uint8_t *out;        // H x W
    // verification planes (only written by the stats variant; may be null)
    uint8_t *gray;
    uint32_t *s1;
    uint32_t *s2;
    uint32_t *n;
    float *t;
    int H, W;
    int win, lo, hi;     // window side and its extent above/left (lo) and below/right (hi)
    float k;             // Niblack k
    float c1, c2;        // Sauvola: c1 = 1 - k, c2 = k / R
    int tile_h;          // output rows per workgroup (multiple of kRowsPerStep)
    int tiles_x;         // tiles per image row
    int n_tiles;         // tiles_x * tiles_y
    int rp;              // LDS ring row pitch in bytes (multiple of 16)
    int depth;           // ring depth in rows = win + kRowsPerStep
    int vp;              // swizzle class pitch of the window-sum rows
    int off_v1, off_v2;  // byte offsets of the V1 / V2 row blocks in LDS
};

// LDS footprint and swizzle pitch of one tile configuration.
struct LdsPlan {
    int rp, depth, vp, off_v1, off_v2, bytes;
};

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// tile_w output columns, window win.  Returns false if it cannot fit.
inline bool plan_lds(int tile_w, int win, LdsPlan *p) {
    const int opt = tile_w / kThreadsPerRow;  // outputs per thread per row
    const int rp = round_up(tile_w + win + 15, 16);
    if (rp > kMaxCols) return false;
    const int depth = win + kRowsPerStep;
    // class pitch vp: every class holds rp/opt columns; opt*vp = 16 (mod 64)
    // keeps the 4 rows of a wave on different LDS banks.
    int vp = (rp + opt - 1) / opt;
    while ((opt * vp) % 64 != 16) ++vp;
    const int ring = round_up(depth * rp + 16, 16);
    const int v1 = round_up(kRowsPerStep * opt * vp * 2, 16);
    const int v2 = kRowsPerStep * opt * vp * 4;
    p->rp = rp;
    p->depth = depth;
    p->vp = vp;
    p->off_v1 = ring;
    p->off_v2 = ring + v1;
    p->bytes = ring + v1 + v2;
    return p->bytes <= kMaxLds;
}

}  // namespace bz
