// Host-side argument checks and planning of libbinarize (bz_host.hpp), built
// with g++ under AddressSanitizer and UBSan by the CPU test suite.  Exits 0
// when every check holds; prints the first failure otherwise.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "bz_host.hpp"

using namespace bz;

static int g_fail = 0;
#define CHECK(cond, ...)                                           \
    do {                                                           \
        if (!(cond)) {                                             \
            if (g_fail++ < 20) {                                   \
                std::printf("FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond); \
                std::printf(__VA_ARGS__);                          \
                std::printf("\n");                                 \
            }                                                      \
        }                                                          \
    } while (0)

// Brute force: mark every byte of a, look for one of b.
static bool brute_overlap(const Region &a, const Region &b, size_t space) {
    std::vector<unsigned char> mark(space, 0);
    for (int64_t i = 0; i < a.rows; ++i)
        for (int64_t j = 0; j < a.len; ++j) mark[(size_t)(a.base + i * a.pitch + j)] = 1;
    for (int64_t i = 0; i < b.rows; ++i)
        for (int64_t j = 0; j < b.len; ++j)
            if (mark[(size_t)(b.base + i * b.pitch + j)]) return true;
    return false;
}

static void check_regions() {
    std::mt19937_64 rng(12345);
    const size_t space = 8192;
    auto rnd = [&](int lo, int hi) { return (int64_t)(lo + (int)(rng() % (uint64_t)(hi - lo + 1))); };
    for (int trial = 0; trial < 200000; ++trial) {
        Region r[2];
        for (auto &x : r) {
            x.rows = rnd(1, 9);
            x.len = rnd(1, 48);
            x.pitch = x.rows > 1 ? x.len + rnd(0, 64) : rnd(0, 3) * x.len;
            const int64_t span = (x.rows - 1) * (x.rows > 1 ? x.pitch : 0) + x.len;
            x.base = (uintptr_t)rnd(0, (int)(space - span - 1));
        }
        const bool want = brute_overlap(r[0], r[1], space);
        CHECK(regions_overlap(r[0], r[1]) == want, "trial %d", trial);
        CHECK(regions_overlap(r[1], r[0]) == want, "trial %d swapped", trial);
    }
}

static void check_parameter_range() {
    CHECK(check_params(BZ_SAUVOLA, 0.5f, 128.0f) == BZ_OK, "typical Sauvola");
    CHECK(check_params(BZ_SAUVOLA, 1.0f, 64.0f) == BZ_OK, "Sauvola limits");
    CHECK(check_params(BZ_SAUVOLA, -1.0f, 64.0f) == BZ_OK, "Sauvola limits, negative k");
    CHECK(check_params(BZ_SAUVOLA, std::nextafter(1.0f, 2.0f), 128.0f) == BZ_ERR_PARAM, "k just above 1");
    CHECK(check_params(BZ_SAUVOLA, 0.5f, std::nextafter(64.0f, 0.0f)) == BZ_ERR_PARAM, "R just below 64");
    CHECK(check_params(BZ_NIBLACK, -1.0f, 0.25f) == BZ_OK, "Niblack ignores R's size");
    CHECK(check_params(BZ_NIBLACK, 0.2f, 0.0f) == BZ_ERR_PARAM, "R must be positive");
    CHECK(check_params(BZ_NIBLACK, NAN, 128.0f) == BZ_ERR_PARAM, "NaN k");
    CHECK(check_params(BZ_SAUVOLA, 0.5f, INFINITY) == BZ_ERR_PARAM, "infinite R");
    CHECK(check_params(2, 0.5f, 128.0f) == BZ_ERR_RULE, "rule");
    CHECK(check_window(0) == BZ_ERR_WINDOW && check_window(256) == BZ_ERR_WINDOW, "window");
    CHECK(check_window(1) == BZ_OK && check_window(255) == BZ_OK, "window limits");
}

static void check_decision() {
    for (int win = 1; win <= 255; win += 2) {
        const Decision d = make_decision(BZ_SAUVOLA, 0.34f, 128.0f, win);
        const double n = (double)win * win;
        CHECK(d.rule == BZ_SAUVOLA, "rule");
        CHECK(std::fabs(d.c1n * n - d.c1) <= 1e-15 * std::fabs(d.c1), "c1n win %d", win);
        CHECK(std::fabs(d.c2n2 * n * n - d.c2) <= 1e-15 * std::fabs(d.c2), "c2n2 win %d", win);
        CHECK(d.c1 == 1.0 - (double)0.34f && d.c2 == (double)0.34f / 128.0, "c1 c2");
    }
    CHECK(make_decision(BZ_SAUVOLA, 0.0f, 128.0f, 15).rule == BZ_NIBLACK, "k = 0 routes to Niblack");
    CHECK(make_decision(BZ_NIBLACK, -0.2f, 128.0f, 15).rule == BZ_NIBLACK, "Niblack stays");
}

static void check_images() {
    const uint8_t *in = (const uint8_t *)(uintptr_t)0x100000;
    uint8_t *out = (uint8_t *)(uintptr_t)0x200000;
    ImageDesc d{in, out, 16, 16, 1, 0, 0};
    CHECK(check_image(d) == BZ_OK && d.pitch_in == 16 && d.pitch_out == 16, "contiguous pitches filled");
    d = ImageDesc{in, out, 16, 16, 3, 47, 0};
    CHECK(check_image(d) == BZ_ERR_SHAPE, "short input pitch");
    d = ImageDesc{in, out, 16, 16, 1, 0, 15};
    CHECK(check_image(d) == BZ_ERR_SHAPE, "short output pitch");
    d = ImageDesc{in, out, 65536, 32768, 1, 0, 0};
    CHECK(check_image(d) == BZ_ERR_SHAPE, "2^31 pixels");
    d = ImageDesc{in, out, 16, 16, 4, 0, 0};
    CHECK(check_image(d) == BZ_ERR_CHANNELS, "channels");
    d = ImageDesc{nullptr, out, 16, 16, 1, 0, 0};
    CHECK(check_image(d) == BZ_ERR_NULL, "null");
    d = ImageDesc{in, (uint8_t *)in + 32, 16, 16, 1, 64, 64};
    CHECK(check_image(d) == BZ_OK, "interleaved rows accepted");
    d = ImageDesc{in, (uint8_t *)in + 8, 16, 16, 1, 64, 64};
    CHECK(check_image(d) == BZ_ERR_ALIAS, "straddling rows refused");
    d = ImageDesc{in, out, 300, 212, 3, 0, 0};
    CHECK(check_page(d, 31, 0.34f, 128.0f, BZ_SAUVOLA) == BZ_OK, "A4-like page");
    CHECK(check_page(d, 31, 1.5f, 128.0f, BZ_SAUVOLA) == BZ_ERR_PARAM, "k out of range");
}

static void check_plans() {
    const int sizes[] = {1, 7, 16, 255, 256, 257, 300, 1024, 3508, 4096, 46340};
    for (int C : {1, 3})
        for (int win = 1; win <= 255; ++win)
            for (int H : sizes)
                for (int W : sizes) {
                    int tw = 0, th = 0;
                    pick_default_tile(H, W, C, win, 256, &tw, &th);
                    CHECK(check_tile(tw, th, win, C) == BZ_OK, "default tile %dx%dx%d win %d: %d x %d", H, W, C, win,
                          tw, th);
                    CHECK(tile_lds_bytes(tw, win, C) <= kMaxLds, "LDS");
                    // gray tiles: the start-up rounds fit in the tile's LDS
                    if (C == 1)
                        CHECK(tile_lds_bytes(tw, win, 1) >= kStartRows * ring_pitch(tw, win), "gray LDS %d win %d",
                              tw, win);
                }
    // layout choice: narrow windows keep the ring; wide windows take the
    // blocks layout on a full 4096^2 page but not on a page with few tiles
    {
        int tw = 0, th = 0;
        pick_default_tile(4096, 4096, 1, 15, 256, &tw, &th);
        CHECK(!use_blocks(4096, 4096, 1, 15, tw, th, 256), "win 15 keeps the ring");
        pick_default_tile(4096, 4096, 1, 101, 256, &tw, &th);
        CHECK(use_blocks(4096, 4096, 1, 101, tw, th, 256) && tw == 256 && th == 64, "win 101: blocks, 256x64 (%dx%d)",
              tw, th);
        CHECK(tile_lds_bytes(tw, 101, 1, true) <= kMaxLds / 4, "four tiles per CU");
        pick_default_tile(1000, 1000, 1, 101, 256, &tw, &th);
        CHECK(!use_blocks(1000, 1000, 1, 101, tw, th, 256), "few tiles: ring");
        pick_default_tile(4096, 4096, 3, 101, 256, &tw, &th);
        CHECK(!use_blocks(4096, 4096, 3, 101, tw, th, 256), "colour pages keep the ring");
    }
    // argument block of an aligned page and of a one-byte-shifted one
    alignas(16) static uint8_t buf[4096 * 2 + 64];
    ImageDesc d{buf, buf + 4096 + 32, 64, 64, 1, 0, 0};
    CHECK(check_page(d, 15, 0.5f, 128.0f, BZ_SAUVOLA) == BZ_OK, "page");
    PageArgs a = page_args(d, 15, 0.5f, 128.0f, BZ_SAUVOLA, 256, 64);
    CHECK(a.row_aligned == 1 && a.lo == 7 && a.hi == 7 && a.tiles_x == 1 && a.n_tiles == 1, "aligned args");
    d.img = buf + 1;
    a = page_args(d, 14, 0.5f, 128.0f, BZ_SAUVOLA, 256, 64);
    CHECK(a.row_aligned == 0 && a.lo == 7 && a.hi == 6, "unaligned args, even window");
    // the aligned body keeps 32-bit per-thread offsets (8 rows plus a row's
    // bytes): pitches of 2^28 or more take the general body
    d.img = buf;
    d.pitch_in = (int64_t)1 << 28;
    d.pitch_out = 64;
    a = page_args(d, 15, 0.5f, 128.0f, BZ_SAUVOLA, 256, 64);
    CHECK(a.row_aligned == 0, "input pitch 2^28: general body");
    d.pitch_in = ((int64_t)1 << 28) - 16;
    a = page_args(d, 15, 0.5f, 128.0f, BZ_SAUVOLA, 256, 64);
    CHECK(a.row_aligned == 1, "input pitch below 2^28: aligned body");
    d.pitch_out = (int64_t)1 << 28;
    a = page_args(d, 15, 0.5f, 128.0f, BZ_SAUVOLA, 256, 64);
    CHECK(a.row_aligned == 0 && a.small_pitch == 0, "output pitch 2^28: edge body only");
    d.pitch_out = 4099;
    d.img = buf + 3;
    a = page_args(d, 15, 0.5f, 128.0f, BZ_SAUVOLA, 256, 64);
    CHECK(a.row_aligned == 0 && a.small_pitch == 1, "unaligned rows, small pitches: wide interior tiles");
}

// Batch plans: occupancy classes, tile width, layout and launch group of a
// page, and the refusals.
static void check_batch_plans() {
    CHECK(class_lds(0) == 40896 && class_lds(1) == 54544 && class_lds(2) == 81856 && class_lds(3) == 163776,
          "class shares %d %d %d %d", class_lds(0), class_lds(1), class_lds(2), class_lds(3));
    for (int c = 0; c < kClasses; ++c)
        CHECK((kClasses - c) * (class_lds(c) + kStaticLds) <= kMaxLds && class_lds(c) % 16 == 0, "class %d fits", c);
    CHECK(class_of(40896) == 0 && class_of(40897) == 1 && class_of(54544) == 1 && class_of(54545) == 2 &&
              class_of(81856) == 2 && class_of(81857) == 3 && class_of(163776) == 3 && class_of(163777) == -1,
          "class boundaries");
    CHECK(group_of(256, 0, false) == 0 && group_of(128, 1, false) == 1 && group_of(128, 0, true) == 2 &&
              group_of(128, 1, true) == 3 && group_of(256, 0, true) == 4 && group_of(256, 1, true) == 5,
          "groups");
    CHECK(blk_group(2) && blk_group(5) && !blk_group(0) && !blk_group(1), "blocks groups");
    auto plan = [](int C, int win, int cap, int tw_req, int th_req, int *tw, int *th, bool *blk, int *lds) {
        bz_page p{};
        p.H = 100;
        p.W_img = 100;
        p.channels = C;
        p.win = win;
        p.tile_w = tw_req;
        p.tile_h = th_req;
        return page_tile(p, cap, tw, th, blk, lds);
    };
    int tw = 0, th = 0, lds = 0;
    bool blk = false;
    const int cap = class_lds(2);  // the default
    CHECK(plan(1, 15, cap, 0, 0, &tw, &th, &blk, &lds) == BZ_OK && tw == 256 && th == 128 && !blk && lds == 32752 &&
              class_of(lds) == 0,
          "gray 15: ring, 4 per CU");
    CHECK(plan(1, 61, cap, 0, 0, &tw, &th, &blk, &lds) == BZ_OK && tw == 256 && blk && class_of(lds) == 0,
          "gray 61: blocks, 4 per CU (%d)", lds);
    CHECK(plan(1, 255, cap, 0, 0, &tw, &th, &blk, &lds) == BZ_OK && tw == 128 && blk && class_of(lds) == 0,
          "gray 255: 128-column blocks (%d)", lds);
    CHECK(plan(3, 61, cap, 0, 0, &tw, &th, &blk, &lds) == BZ_OK && tw == 256 && !blk && class_of(lds) == 1,
          "rgb 61: ring, 3 per CU (%d)", lds);
    CHECK(plan(3, 151, cap, 0, 0, &tw, &th, &blk, &lds) == BZ_OK && tw == 128 && !blk && class_of(lds) == 2,
          "rgb 151 at the default cap: 128 columns, 2 per CU (%d)", lds);
    CHECK(plan(3, 201, class_lds(3), 0, 0, &tw, &th, &blk, &lds) == BZ_OK && tw == 256 && class_of(lds) == 3,
          "rgb 201 at the largest cap: 256 columns, 1 per CU (%d)", lds);
    CHECK(plan(3, 255, cap, 0, 0, &tw, &th, &blk, &lds) == BZ_ERR_TILE, "rgb 255 needs more than the cap");
    CHECK(plan(1, 31, cap, 128, 64, &tw, &th, &blk, &lds) == BZ_OK && tw == 128 && th == 64 && !blk,
          "caller's tile");
    CHECK(plan(1, 31, cap, 64, 0, &tw, &th, &blk, &lds) == BZ_ERR_TILE, "tile width 64 refused");
    CHECK(plan(1, 31, cap, 0, 12, &tw, &th, &blk, &lds) == BZ_ERR_TILE, "tile height 12 refused");
    CHECK(plan(1, 31, class_lds(0), 0, 0, &tw, &th, &blk, &lds) == BZ_OK && lds <= class_lds(0), "small cap");
}

int main() {
    check_regions();
    check_batch_plans();
    check_parameter_range();
    check_decision();
    check_images();
    check_plans();
    if (g_fail) {
        std::printf("%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
