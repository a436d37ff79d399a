// binarize.hip -- host side of libbinarize: argument validation, tile
// planning, kernel dispatch and the C ABI declared in include/binarize.h.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "binarize.h"
#include "bz_common.hpp"
#include "bz_host.hpp"
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

Region plane(const void *p, size_t bytes) { return Region{(uintptr_t)p, 1, (int64_t)bytes, (int64_t)bytes}; }

template <int TW, int C, int RULE, bool STATS, bool BLK>
int launch_t(const PageArgs &a, int lds, hipStream_t st) {
    auto kern = bz_page_kernel<TW, C, RULE, STATS, BLK>;
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
    if (C == 1 && a.blocks)  // gray page in the blocks layout
        return stats ? launch_t<TW, 1, RULE, true, true>(a, lds, st) : launch_t<TW, 1, RULE, false, true>(a, lds, st);
    return stats ? launch_t<TW, C, RULE, true, false>(a, lds, st) : launch_t<TW, C, RULE, false, false>(a, lds, st);
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

int run(ImageDesc d, int win, float k, float R, int rule, int tile_w, int tile_h, uint8_t *gray, uint32_t *s1,
        uint32_t *s2, uint32_t *n, float *t, bool stats, void *stream) {
    int rc = check_page(d, win, k, R, rule);
    if (rc) return rc;
    if (stats) {
        const size_t npx = (size_t)d.H * d.W;
        const void *planes[5] = {gray, s1, s2, n, t};
        const size_t sizes[5] = {npx, 4 * npx, 4 * npx, 4 * npx, 4 * npx};
        for (int i = 0; i < 5; ++i) {
            if (!planes[i]) continue;
            const Region r = plane(planes[i], sizes[i]);
            if (regions_overlap(r, input_region(d)) || regions_overlap(r, output_region(d))) return BZ_ERR_ALIAS;
            for (int j = 0; j < i; ++j)
                if (planes[j] && regions_overlap(r, plane(planes[j], sizes[j]))) return BZ_ERR_ALIAS;
        }
    }
    const int cus = device_cus();
    if (tile_w <= 0 || tile_h <= 0) pick_default_tile(d.H, d.W, d.C, win, cus, &tile_w, &tile_h);
    if ((rc = check_tile(tile_w, tile_h, win, d.C))) return rc;
    const bool blocks = use_blocks(d.H, d.W, d.C, win, tile_w, tile_h, cus);
    PageArgs a = page_args(d, win, k, R, rule, tile_w, tile_h, blocks);
    if (stats) {
        a.gray = gray;
        a.s1 = s1;
        a.s2 = s2;
        a.n = n;
        a.t = t;
    }
    const int kernel_rule = make_decision(rule, k, R, win).rule;
    return launch(a, tile_w, d.C, kernel_rule, stats, tile_lds_bytes(tile_w, win, d.C, blocks),
                  (hipStream_t)stream);
}

ImageDesc contiguous(const uint8_t *img, int H, int W, int C, uint8_t *out) {
    return ImageDesc{img, out, H, W, C, 0, 0};
}

}  // namespace

extern "C" {

int binarize(const uint8_t *img, int H, int W_img, int channels, int win, float k, float R, int rule,
             uint8_t *out) {
    return run(contiguous(img, H, W_img, channels, out), win, k, R, rule, 0, 0, nullptr, nullptr, nullptr,
               nullptr, nullptr, false, nullptr);
}

int binarize_async(const uint8_t *img, int H, int W_img, int channels, int win, float k, float R,
                   int rule, uint8_t *out, void *stream) {
    return run(contiguous(img, H, W_img, channels, out), win, k, R, rule, 0, 0, nullptr, nullptr, nullptr,
               nullptr, nullptr, false, stream);
}

int binarize_pitched(const uint8_t *img, int H, int W_img, int channels, int64_t pitch_in, int win, float k,
                     float R, int rule, uint8_t *out, int64_t pitch_out, void *stream) {
    if (pitch_in < 0 || pitch_out < 0) return BZ_ERR_SHAPE;
    return run(ImageDesc{img, out, H, W_img, channels, pitch_in, pitch_out}, win, k, R, rule, 0, 0, nullptr,
               nullptr, nullptr, nullptr, nullptr, false, stream);
}

int binarize_tuned(const uint8_t *img, int H, int W_img, int channels, int win, float k, float R,
                   int rule, uint8_t *out, int tile_w, int tile_h, void *stream) {
    if (tile_w <= 0 || tile_h <= 0) return BZ_ERR_TILE;
    return run(contiguous(img, H, W_img, channels, out), win, k, R, rule, tile_w, tile_h, nullptr, nullptr,
               nullptr, nullptr, nullptr, false, stream);
}

int binarize_stats(const uint8_t *img, int H, int W_img, int channels, int win, float k, float R,
                   int rule, uint8_t *out, uint8_t *gray, uint32_t *s1, uint32_t *s2, uint32_t *n,
                   float *t, void *stream) {
    return run(contiguous(img, H, W_img, channels, out), win, k, R, rule, 0, 0, gray, s1, s2, n, t, true,
               stream);
}

int binarize_tile_lds(int tile_w, int win, int channels) {
    if (check_window(win)) return BZ_ERR_WINDOW;
    if (channels != 1 && channels != 3) return BZ_ERR_CHANNELS;
    if (!tile_fits(tile_w, win, channels)) return BZ_ERR_TILE;
    return tile_lds_bytes(tile_w, win, channels);
}

int binarize_default_tile(int H, int W_img, int channels, int win, int *tile_w, int *tile_h) {
    if (!tile_w || !tile_h) return BZ_ERR_NULL;
    if (H < 1 || W_img < 1) return BZ_ERR_SHAPE;
    if (channels != 1 && channels != 3) return BZ_ERR_CHANNELS;
    if (check_window(win)) return BZ_ERR_WINDOW;
    pick_default_tile(H, W_img, channels, win, device_cus(), tile_w, tile_h);
    return BZ_OK;
}

const char *binarize_strerror(int code) {
    switch (code) {
        case BZ_OK: return "ok";
        case BZ_ERR_NULL: return "a required pointer is NULL";
        case BZ_ERR_SHAPE: return "image shape out of range (H, W_img >= 1, H*W_img*channels < 2^31, row pitches >= row bytes)";
        case BZ_ERR_CHANNELS: return "channels must be 1 or 3";
        case BZ_ERR_WINDOW: return "window side must be in [1, 255]";
        case BZ_ERR_PARAM: return "k must lie in [-1, 1], R must be finite and positive, and R >= 64 for Sauvola";
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
