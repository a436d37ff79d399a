// bz_common.hpp -- launch arguments and LDS plan shared by the host
// dispatcher and the gfx950 kernels of libbinarize.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>

#include <mutex>
#include <utility>
#endif

#if defined(__HIPCC__)
#define BZ_HD __host__ __device__
#else
#define BZ_HD
#endif

namespace bz {

// Workgroup shape of the tile kernel: 256 threads (4 wave64s).  The vertical
// pass gives every thread two adjacent LDS columns; the horizontal pass gives
// each of the RB output rows of a step TPR = 32 threads.
constexpr int kThreads = 256;
constexpr int kRowsPerStep = 8;                          // RB
constexpr int kThreadsPerRow = kThreads / kRowsPerStep;  // TPR = 32
constexpr int kMaxCols = 2 * kThreads;                   // LDS columns per tile
constexpr int kMaxLds = 160 * 1024;                      // gfx950 LDS per workgroup

// One page as the tile kernel sees it.  All geometry that depends only on the
// page and the tile shape is computed once on the host.
struct PageArgs {
    const uint8_t *img;  // H rows of W * C bytes, pitch_in bytes apart
    uint8_t *out;        // H rows of W bytes, pitch_out bytes apart
    // verification planes (only written by the stats variant; may be null),
    // each H x W with rows W entries apart
    uint8_t *gray;
    uint32_t *s1;
    uint32_t *s2;
    uint32_t *n;
    float *t;
    int64_t pitch_in, pitch_out;
    double c1, c2;     // Sauvola: t = m (c1 + c2 s), c1 = 1 - k, c2 = k / R
    double c1n, c2n2;  // whole windows (n = win^2): c1 / n, c2 / n^2
    int H, W;
    int win, lo, hi;  // window side and its extent above/left (lo) and below/right (hi)
    float k;          // Niblack k
    int tile_h;       // output rows per workgroup (multiple of kRowsPerStep)
    int tiles_x;      // tiles per image row
    int n_tiles;      // tiles_x * tiles_y
    int rp;           // LDS ring row pitch in bytes (multiple of 16)
    int depth;        // ring depth in rows
    int row_aligned;  // input rows 16-byte aligned and a multiple of 16 pixels, output rows 8-byte
                      // aligned, both pitches below 2^28
    int blocks;       // gray page in the blocks layout (see gray_blocks)
    int small_pitch;  // both pitches below 2^28 (per-thread offsets of 8 rows fit 32 bits)
};

BZ_HD inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Ring geometry.  rp covers the tile, its halo and up to 16 columns of
// alignment slack.  depth holds every row one step touches (win + RB).  The
// next step's rows are written while this step's horizontal pass still reads
// its window centres; they replace rows at least depth rows older, which must
// be rows the vertical pass has finished with and not centres: with
// depth = win + RB they are this step's leaving rows, and when the window
// reaches less than RB rows down depth >= hi + 2 RB keeps them above the
// centres.
BZ_HD inline int ring_pitch(int tile_w, int win) { return round_up(tile_w + win + 15, 16); }
BZ_HD inline int ring_depth(int win) {
    const int hi = win - 1 - win / 2;
    return (win + kRowsPerStep > hi + 2 * kRowsPerStep) ? win + kRowsPerStep : hi + 2 * kRowsPerStep;
}
// Width of the Vb rows: the tile, or the whole first window if that is wider.
BZ_HD inline int vb_width(int tile_w, int win) { return round_up(win > tile_w ? win : tile_w, 32); }
// Row pitches of the V arrays: the entries a row needs, then kTrash trash
// entries that take the writes of the columns the row does not need, so every
// column writes at one fixed offset per row (the few lanes that write trash
// share an entry at most four to a wave).  For 256-column tiles vb_width is
// always 256.
constexpr int kTrash = 16;
BZ_HD inline int va_pitch(int tile_w) { return tile_w + kTrash; }
BZ_HD inline int vb_pitch(int tile_w, int win) { return vb_width(tile_w, win) + kTrash; }
BZ_HD inline int v_bytes(int tile_w, int win) {
    const int pa = va_pitch(tile_w), pb = vb_pitch(tile_w, win);
    return kRowsPerStep * (pa * 2 + pb * 2 + pa * 4 + pb * 4);
}
BZ_HD inline int rows_bytes(int rows, int tile_w, int win) { return round_up(rows * ring_pitch(tile_w, win) + 16, 16); }

// Two layouts of the input rows in LDS.  The ring holds every row the
// window spans (depth rows), so each input byte is staged once per tile (and
// converted to gray once); its footprint grows with the window.  The blocks
// layout of a gray page holds three blocks of RB rows: the step's entering
// rows, its leaving rows and its window centres, each staged from global
// memory (an input row is read up to three times per tile, the second and
// third time from L2), so the footprint does not depend on the window; at
// start-up the first win rows are staged kStartRows at a time into the whole
// of the tile's LDS and summed.  A gray tile takes the blocks layout when the
// ring would allow fewer than four workgroups per CU (the occupancy of the
// narrow windows): staging three blocks costs more than staging one row set,
// so the ring is kept where it does not limit occupancy.  Both layouts give
// identical bytes.  `allow_blocks` false keeps the ring (a single-page
// launch with few tiles; a ring page of the batched launch).
constexpr int kGrayBlocks = 3;
constexpr int kStartRows = 4 * kRowsPerStep;
BZ_HD inline int ring_layout_lds(int tile_w, int win) { return rows_bytes(ring_depth(win), tile_w, win) + v_bytes(tile_w, win); }
BZ_HD inline bool gray_blocks(int tile_w, int win, int channels, bool allow_blocks = true) {
    return allow_blocks && channels == 1 && ring_layout_lds(tile_w, win) > kMaxLds / 4;
}
BZ_HD inline int ring_rows(int tile_w, int win, int channels, bool allow_blocks = true) {
    return gray_blocks(tile_w, win, channels, allow_blocks) ? kGrayBlocks * kRowsPerStep : ring_depth(win);
}
// LDS layout: rows (ring or blocks) | Va1 [RB][va_pitch] u16 |
// Vb1 [RB][vb_pitch] u16 | Va2 [RB][va_pitch] u32 | Vb2 [RB][vb_pitch] u32,
// and in the blocks layout at least 2 kStartRows rows of the row pitch (the
// start-up's two staging halves).
BZ_HD inline int tile_lds_bytes(int tile_w, int win, int channels, bool allow_blocks = true) {
    if (!gray_blocks(tile_w, win, channels, allow_blocks)) return ring_layout_lds(tile_w, win);
    const int b = rows_bytes(kGrayBlocks * kRowsPerStep, tile_w, win) + v_bytes(tile_w, win);
    const int s = rows_bytes(2 * kStartRows, tile_w, win);
    return b > s ? b : s;
}

// Position of entry x in a V2 row of `width` entries.  Thread h of a row group
// reads entries 8h .. 8h+7 as two 16-byte quads; quads 8h..8h+3 of all threads
// are packed first and quads 8h+4..8h+7 after width/2, so each 128-bit read of
// a wave covers consecutive addresses.  With SW (256-column tiles), inside the
// second quad neighbouring entries trade places (8h+4..8h+7 stored as
// 5 4 7 6).  The vertical pass writes every other entry in one instruction;
// without the swap the entries of both quads would fall on even banks only
// (quads start on multiples of four words), two lanes to a bank, and with it
// the second quad's entries take the odd banks.  128-column tiles, whose
// threads read one quad each, keep the plain order: there the swap would cost
// a per-lane select on every read.
BZ_HD inline int v2_quad(int x, int width) { return ((x >> 3) << 2) + (((x >> 2) & 1) ? width / 2 : 0); }
template <bool SW>
BZ_HD inline int v2_pos(int x, int width) {
    return v2_quad(x, width) + (SW ? ((x & 3) ^ ((x >> 2) & 1)) : (x & 3));
}

// HIP error of the last failed runtime call on this thread (kept by the
// single-page entry points and the batch entry points alike).
void set_last_hip_error(int e);

#if defined(__HIPCC__)
// Runs f once per device id (the current device): function attributes such
// as the dynamic LDS limit belong to a device, so each device a process
// launches on needs its own first call.
constexpr int kMaxDevices = 64;
template <class F>
inline void once_per_device(std::once_flag (&flags)[kMaxDevices], F &&f) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        f();
        return;
    }
    std::call_once(flags[dev], std::forward<F>(f));
}
#endif

// Does this tile configuration fit the hardware?
inline bool tile_fits(int tile_w, int win, int channels, bool allow_blocks = true) {
    if (tile_w != 128 && tile_w != 256) return false;
    if (ring_pitch(tile_w, win) > kMaxCols) return false;
    return tile_lds_bytes(tile_w, win, channels, allow_blocks) <= kMaxLds;
}

}  // namespace bz
