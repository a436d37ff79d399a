// binarize.hip -- host side of libbinarize: argument validation, tile
// planning, kernel dispatch and the C ABI declared in include/binarize.h.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "binarize.h"
#include "bz_common.hpp"
#include "bz_tile.hpp"

using namespace bz;

namespace {
thread_local int t_last_hip = 0;
}  // namespace

void bz::set_last_hip_error(int e) { t_last_hip = e; }

namespace {

int hip_fail(hipError_t e) {
    t_last_hip = (int)e;
    return BZ_ERR_HIP;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

int validate(const uint8_t *img, int H, int W, int C, int win, float k, float R, int rule,
             const uint8_t *out) {
    if (!img || !out) return BZ_ERR_NULL;
    if (H < 1 || W < 1) return BZ_ERR_SHAPE;
    if (C != 1 && C != 3) return BZ_ERR_CHANNELS;
    if ((int64_t)H * (int64_t)W * C >= ((int64_t)1 << 31)) return BZ_ERR_SHAPE;
    if (win < 1 || win > 255) return BZ_ERR_WINDOW;
    if (rule != BZ_SAUVOLA && rule != BZ_NIBLACK) return BZ_ERR_RULE;
    if (!std::isfinite(k) || !std::isfinite(R) || !(R > 0.0f)) return BZ_ERR_PARAM;
    if (overlaps(img, (size_t)H * W * C, out, (size_t)H * W)) return BZ_ERR_ALIAS;
    return BZ_OK;
}

// Compute units of the current device (cached per device id; threads that
// race on the first query store the same value).
int device_cus() {
    static std::atomic<int> cus[64];  // zero-initialised: not yet queried
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = cus[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        cus[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

void pick_default_tile(int H, int W, int win, int cus, int *tw, int *th) {
    const int w = tile_fits(256, win) ? 256 : 128;
    int per_cu = kMaxLds / tile_lds_bytes(w, win);
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 8) per_cu = 8;  // 8 x 4 waves fill a CU
    const long target = (long)cus * per_cu;
    const long tiles_x = (W + w - 1) / w;
    long h = (H * tiles_x + target - 1) / target;
    h = (h + kRowsPerStep - 1) / kRowsPerStep * kRowsPerStep;
    const long hmin = 64;  // keep the start-up rows (win) a modest share of the tile
    if (h < hmin) h = hmin;
    if (h > 4096) h = 4096;
    *tw = w;
    *th = (int)h;
}

struct Plan {
    int tile_w, tile_h;
    int lds_bytes;
    int tiles_x, tiles_y;
};

int make_plan(int H, int W, int win, int tile_w, int tile_h, Plan *p) {
    if (tile_w != 128 && tile_w != 256) return BZ_ERR_TILE;
    if (tile_h < kRowsPerStep || tile_h > 4096 || tile_h % kRowsPerStep) return BZ_ERR_TILE;
    if (!tile_fits(tile_w, win)) return BZ_ERR_TILE;
    p->lds_bytes = tile_lds_bytes(tile_w, win);
    p->tile_w = tile_w;
    p->tile_h = tile_h;
    p->tiles_x = (W + tile_w - 1) / tile_w;
    p->tiles_y = (H + tile_h - 1) / tile_h;
    return BZ_OK;
}

void fill_args(PageArgs *a, const uint8_t *img, int H, int W, int C, int win, float k, float R,
               uint8_t *out, const Plan &p) {
    a->img = img;
    a->out = out;
    a->gray = nullptr;
    a->s1 = a->s2 = a->n = nullptr;
    a->t = nullptr;
    a->H = H;
    a->W = W;
    a->win = win;
    a->lo = win / 2;
    a->hi = win - 1 - a->lo;
    a->k = k;
    a->c1 = (float)(1.0 - (double)k);
    a->c2 = (float)((double)k / (double)R);
    a->tile_h = p.tile_h;
    a->tiles_x = p.tiles_x;
    a->n_tiles = p.tiles_x * p.tiles_y;
    a->rp = ring_pitch(p.tile_w, win);
    a->depth = ring_depth(win);
    a->row_aligned =
        (((uintptr_t)img & 15) == 0 && ((int64_t)W * C) % 16 == 0 && ((uintptr_t)out & 7) == 0) ? 1 : 0;
}

template <int TW, int C, int RULE, bool STATS>
int launch_t(const PageArgs &a, int lds, hipStream_t st) {
    auto kern = bz_page_kernel<TW, C, RULE, STATS>;
    static std::once_flag once[kMaxDevices];
    once_per_device(once, [&] {
        // allow the full 160 KB of gfx950 LDS for dynamic shared memory
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
        (void)hipGetLastError();
    });
    hipLaunchKernelGGL(kern, dim3((unsigned)a.n_tiles), dim3(kThreads), (unsigned)lds, st, a);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BZ_OK : hip_fail(e);
}

template <int TW, int C, int RULE>
int launch_s(const PageArgs &a, bool stats, int lds, hipStream_t st) {
    return stats ? launch_t<TW, C, RULE, true>(a, lds, st) : launch_t<TW, C, RULE, false>(a, lds, st);
}

template <int TW, int C>
int launch_r(const PageArgs &a, int rule, bool stats, int lds, hipStream_t st) {
    return rule == BZ_SAUVOLA ? launch_s<TW, C, BZ_SAUVOLA>(a, stats, lds, st)
                              : launch_s<TW, C, BZ_NIBLACK>(a, stats, lds, st);
}

template <int TW>
int launch_c(const PageArgs &a, int C, int rule, bool stats, int lds, hipStream_t st) {
    return C == 1 ? launch_r<TW, 1>(a, rule, stats, lds, st) : launch_r<TW, 3>(a, rule, stats, lds, st);
}

int launch(const PageArgs &a, int tile_w, int C, int rule, bool stats, int lds, hipStream_t st) {
    return tile_w == 256 ? launch_c<256>(a, C, rule, stats, lds, st)
                         : launch_c<128>(a, C, rule, stats, lds, st);
}

int run(const uint8_t *img, int H, int W, int C, int win, float k, float R, int rule, uint8_t *out,
        int tile_w, int tile_h, uint8_t *gray, uint32_t *s1, uint32_t *s2, uint32_t *n, float *t,
        bool stats, void *stream) {
    int rc = validate(img, H, W, C, win, k, R, rule, out);
    if (rc) return rc;
    if (stats) {
        const size_t npx = (size_t)H * W;
        const void *planes[5] = {gray, s1, s2, n, t};
        const size_t sizes[5] = {npx, 4 * npx, 4 * npx, 4 * npx, 4 * npx};
        for (int i = 0; i < 5; ++i) {
            if (!planes[i]) continue;
            if (overlaps(planes[i], sizes[i], img, npx * C) || overlaps(planes[i], sizes[i], out, npx))
                return BZ_ERR_ALIAS;
            for (int j = 0; j < i; ++j)
                if (planes[j] && overlaps(planes[i], sizes[i], planes[j], sizes[j])) return BZ_ERR_ALIAS;
        }
    }
    if (tile_w <= 0 || tile_h <= 0) pick_default_tile(H, W, win, device_cus(), &tile_w, &tile_h);
    Plan p;
    rc = make_plan(H, W, win, tile_w, tile_h, &p);
    if (rc) return rc;
    // Sauvola with k = 0 is t = m, exactly the Niblack rule with k = 0; the
    // Niblack form decides ties in exact integers.
    if (rule == BZ_SAUVOLA && k == 0.0f) rule = BZ_NIBLACK;
    PageArgs a;
    fill_args(&a, img, H, W, C, win, k, R, out, p);
    if (stats) {
        a.gray = gray;
        a.s1 = s1;
        a.s2 = s2;
        a.n = n;
        a.t = t;
    }
    return launch(a, p.tile_w, C, rule, stats, p.lds_bytes, (hipStream_t)stream);
}

}  // namespace

extern "C" {

int binarize(const uint8_t *img, int H, int W_img, int channels, int win, float k, float R, int rule,
             uint8_t *out) {
    return run(img, H, W_img, channels, win, k, R, rule, out, 0, 0, nullptr, nullptr, nullptr, nullptr,
               nullptr, false, nullptr);
}

int binarize_async(const uint8_t *img, int H, int W_img, int channels, int win, float k, float R,
                   int rule, uint8_t *out, void *stream) {
    return run(img, H, W_img, channels, win, k, R, rule, out, 0, 0, nullptr, nullptr, nullptr, nullptr,
               nullptr, false, stream);
}

int binarize_tuned(const uint8_t *img, int H, int W_img, int channels, int win, float k, float R,
                   int rule, uint8_t *out, int tile_w, int tile_h, void *stream) {
    if (tile_w <= 0 || tile_h <= 0) return BZ_ERR_TILE;
    return run(img, H, W_img, channels, win, k, R, rule, out, tile_w, tile_h, nullptr, nullptr, nullptr,
               nullptr, nullptr, false, stream);
}

int binarize_stats(const uint8_t *img, int H, int W_img, int channels, int win, float k, float R,
                   int rule, uint8_t *out, uint8_t *gray, uint32_t *s1, uint32_t *s2, uint32_t *n,
                   float *t, void *stream) {
    return run(img, H, W_img, channels, win, k, R, rule, out, 0, 0, gray, s1, s2, n, t, true, stream);
}

int binarize_tile_lds(int tile_w, int win) {
    if (win < 1 || win > 255) return BZ_ERR_WINDOW;
    if (!tile_fits(tile_w, win)) return BZ_ERR_TILE;
    return tile_lds_bytes(tile_w, win);
}

int binarize_default_tile(int H, int W_img, int channels, int win, int *tile_w, int *tile_h) {
    if (!tile_w || !tile_h) return BZ_ERR_NULL;
    if (H < 1 || W_img < 1) return BZ_ERR_SHAPE;
    if (channels != 1 && channels != 3) return BZ_ERR_CHANNELS;
    if (win < 1 || win > 255) return BZ_ERR_WINDOW;
    pick_default_tile(H, W_img, win, device_cus(), tile_w, tile_h);
    return BZ_OK;
}

const char *binarize_strerror(int code) {
    switch (code) {
        case BZ_OK: return "ok";
        case BZ_ERR_NULL: return "a required pointer is NULL";
        case BZ_ERR_SHAPE: return "image shape out of range (H, W_img >= 1, H*W_img*channels < 2^31)";
        case BZ_ERR_CHANNELS: return "channels must be 1 or 3";
        case BZ_ERR_WINDOW: return "window side must be in [1, 255]";
        case BZ_ERR_PARAM: return "k must be finite and R finite and positive";
        case BZ_ERR_RULE: return "rule must be BZ_SAUVOLA (0) or BZ_NIBLACK (1)";
        case BZ_ERR_ALIAS: return "output overlaps the input or another output plane";
        case BZ_ERR_HIP: return "HIP runtime error (see binarize_last_hip_error)";
        case BZ_ERR_TILE: return "unsupported tile configuration";
        case BZ_ERR_WORKSPACE: return "workspace missing or too small";
        default: return "unknown error";
    }
}

int binarize_version(void) { return BINARIZE_VERSION; }

int binarize_last_hip_error(void) { return t_last_hip; }

}  // extern "C"
