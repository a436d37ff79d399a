// bz_staged.hip -- the unfused (staged) form of the exact Sauvola / Niblack
// path: the same statistics (Sec. 2, full W x W window) and decision (Eq. 3,
// Eq. 4, Niblack), in two passes through HBM instead of one.
//
//   bz_rowsum   one workgroup per (row, 256-column segment): stages the gray
//               levels of the segment and its halo (Eq. 1), prefix-sums f and
//               f^2 across the workgroup (DPP scans within 32-lane halves,
//               then across waves), and writes the row window sums
//               R1 = sum f and R2 = sum f^2 over columns [x - lo, x + hi] of
//               every pixel to two u32 planes of the caller's workspace.
//   bz_colsum   one lane per column slides the window down 64 rows of those
//               planes (S = S + R(y + hi) - R(y - lo - 1)), loading 8 rows'
//               entries at a time, and decides with the fused kernel's helpers.
//
// The decision form follows the fused kernel's rule exactly: pixels in a
// 256-column block of the page whose windows all span win columns, in an
// 8-row step (rows 8j .. 8j + 7) whose windows all span win rows, take the
// per-tile-constants Sauvola form; every other pixel the per-pixel n form.
// With exact integer sums this makes the output identical, byte for byte, to
// the fused kernel's.  The staged path moves about 8 B/px of planes out and
// twice that back in on top of the fused kernel's C + 1 B/px; it is the
// "fusion off" point the autotuner measures against the fused kernel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "binarize.h"
#include "bz_common.hpp"
#include "bz_host.hpp"
#include "bz_tile.hpp"

namespace {

using namespace bz;

constexpr int kSegW = 256;    // outputs per row-pass workgroup (one per lane)
constexpr int kColTH = 64;    // rows per column-pass workgroup
constexpr int kColGroup = 8;  // rows whose loads the column pass issues together
constexpr int kStagedThreads = 256;

struct StagedArgs {
    const uint8_t *img;
    uint8_t *out;
    uint32_t *r1, *r2;  // H x W row window sums of f and f^2
    int H, W, lo, hi, win;
    int segs;      // 256-column segments per row
    PageArgs dec;  // decision constants (k, c1, c2, c1n, c2n2) for the decision helpers
};

template <int C>
__device__ __forceinline__ uint32_t gray_at(const uint8_t *row, int x) {
    if (C == 1) return row[x];
    return gray_of(row[3 * x], row[3 * x + 1], row[3 * x + 2]);
}

// inclusive prefix sum across the 64 lanes of a wave
__device__ __forceinline__ uint32_t scan64(uint32_t v) {
    v = scan32(v);
    const uint32_t lower = (uint32_t)__shfl((int)v, 31);  // total of lanes 0..31
    return (threadIdx.x & 32) ? v + lower : v;
}

template <int C>
__global__ __launch_bounds__(kStagedThreads) void bz_rowsum(const StagedArgs s) {
    __shared__ uint32_t p1[2 * kStagedThreads], p2[2 * kStagedThreads];
    __shared__ uint32_t wt1[kStagedThreads / 64], wt2[kStagedThreads / 64];
    const int tid = threadIdx.x;
    const int seg = blockIdx.x % s.segs, y = blockIdx.x / s.segs;
    const int X0 = seg * kSegW;
    // entry i (0 <= i < L) is image column X0 - lo - 1 + i, 0 outside the image;
    // the window of output X0 + t is entries t + 1 .. t + win
    const int L = kSegW + s.win;
    const uint8_t *row = s.img + (size_t)y * s.W * C;
    uint32_t e[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = 2 * tid + u, x = X0 - s.lo - 1 + i;
        e[u] = (i < L && x >= 0 && x < s.W) ? gray_at<C>(row, x) : 0u;
    }
    const uint32_t a1 = e[0], a2 = e[0] * e[0];
    const uint32_t b1 = a1 + e[1], b2 = a2 + e[1] * e[1];  // this lane's two entries
    const uint32_t i1 = scan64(b1), i2 = scan64(b2);
    const int wave = tid >> 6;
    if ((tid & 63) == 63) {
        wt1[wave] = i1;
        wt2[wave] = i2;
    }
    __syncthreads();
    uint32_t o1 = i1 - b1, o2 = i2 - b2;  // sum of the entries before entry 2 tid
    for (int w = 0; w < wave; ++w) {
        o1 += wt1[w];
        o2 += wt2[w];
    }
    p1[2 * tid] = o1 + a1;
    p1[2 * tid + 1] = o1 + b1;
    p2[2 * tid] = o2 + a2;
    p2[2 * tid + 1] = o2 + b2;
    __syncthreads();
    const int x = X0 + tid;
    if (x < s.W) {
        const size_t o = (size_t)y * s.W + x;
        s.r1[o] = p1[tid + s.win] - p1[tid];
        s.r2[o] = p2[tid + s.win] - p2[tid];
    }
}

template <int C, int RULE>
__global__ __launch_bounds__(kStagedThreads) void bz_colsum(const StagedArgs s) {
    const int tid = threadIdx.x;
    const int seg = blockIdx.x % s.segs, ty = blockIdx.x / s.segs;
    const int x = seg * kSegW + tid, Y0 = ty * kColTH;
    if (x >= s.W) return;
    const int lo = s.lo, hi = s.hi, win = s.win, H = s.H, W = s.W;
    const uint32_t *c1 = s.r1 + x, *c2 = s.r2 + x;
    // window sums of row Y0: rows [Y0 - lo, Y0 + hi] inside the image
    uint32_t S1 = 0, S2 = 0;
    for (int r = max(Y0 - lo, 0); r <= min(Y0 + hi, H - 1); ++r) {
        S1 += c1[(size_t)r * W];
        S2 += c2[(size_t)r * W];
    }
    const int XB = x & ~255;
    const bool block_inside = XB - lo >= 0 && XB + 255 + hi <= W - 1;
    const int nx = min(x + hi, W - 1) - max(x - lo, 0) + 1;
    const uint32_t n_full = (uint32_t)__mul24(win, win);
    const WholeWindow q_full = whole_window(s.dec, n_full);
    const int Yend = min(Y0 + kColTH, H);
    // Rows go in groups of kColGroup: the entering and leaving plane entries
    // and the gray levels of a whole group are loaded before any is used, so
    // the loads are in flight together instead of one latency per row.
    // Entries outside the image (and the first row's, already in the initial
    // sum) read as zero.
    for (int yg = Y0; yg < Yend; yg += kColGroup) {
        uint32_t e1[kColGroup], e2[kColGroup], l1[kColGroup], l2[kColGroup], f[kColGroup];
#pragma unroll
        for (int i = 0; i < kColGroup; ++i) {
            const int y = yg + i;
            const bool row = y < Yend;
            const bool enter = row && y > Y0 && y + hi <= H - 1;
            const bool leave = row && y > Y0 && y - lo - 1 >= 0;
            e1[i] = enter ? c1[(size_t)(y + hi) * W] : 0u;
            e2[i] = enter ? c2[(size_t)(y + hi) * W] : 0u;
            l1[i] = leave ? c1[(size_t)(y - lo - 1) * W] : 0u;
            l2[i] = leave ? c2[(size_t)(y - lo - 1) * W] : 0u;
            f[i] = row ? gray_at<C>(s.img + (size_t)y * W * C, x) : 0u;
        }
#pragma unroll
        for (int i = 0; i < kColGroup; ++i) {
            const int y = yg + i;
            if (y >= Yend) break;
            S1 += e1[i] - l1[i];
            S2 += e2[i] - l2[i];
            const int ny = min(y + hi, H - 1) - max(y - lo, 0) + 1;
            const uint32_t n = (uint32_t)__mul24(nx, ny);
            const int y0 = y & ~(kRowsPerStep - 1);
            const bool full = block_inside && y0 - lo >= 0 && y0 + kRowsPerStep - 1 + hi <= H - 1;
            float sq;
            bool dark;
            if (RULE == BZ_SAUVOLA)
                dark = full ? dark_sauvola_full(q_full, f[i], S1, S2, sq)
                            : dark_sauvola(s.dec, f[i], S1, S2, n, sq);
            else
                dark = dark_niblack(s.dec, f[i], S1, S2, full ? n_full : n, sq);
            s.out[(size_t)y * W + x] = dark ? 0 : 255;
        }
    }
}

int fail(hipError_t e) {
    set_last_hip_error((int)e);
    return BZ_ERR_HIP;
}

template <int C, int RULE>
int staged_launch(const StagedArgs &s, hipStream_t st) {
    hipLaunchKernelGGL((bz_rowsum<C>), dim3((unsigned)(s.H * s.segs)), dim3(kStagedThreads), 0, st, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(e);
    const unsigned tiles = (unsigned)(((s.H + kColTH - 1) / kColTH) * s.segs);
    hipLaunchKernelGGL((bz_colsum<C, RULE>), dim3(tiles), dim3(kStagedThreads), 0, st, s);
    e = hipGetLastError();
    return e == hipSuccess ? BZ_OK : fail(e);
}

}  // namespace

extern "C" {

size_t binarize_staged_workspace_size(int H, int W_img) {
    if (H < 1 || W_img < 1) return 0;
    return (size_t)8 * (size_t)H * (size_t)W_img;
}

int binarize_staged(const uint8_t *img, int H, int W_img, int channels, int win, float k, float R, int rule,
                    uint8_t *out, uint32_t *ws, size_t ws_bytes, void *stream) {
    ImageDesc d{img, out, H, W_img, channels, 0, 0};
    int rc = check_page(d, win, k, R, rule);
    if (rc) return rc;
    const size_t npx = (size_t)H * (size_t)W_img;
    if (!ws || ws_bytes < 8 * npx || ((uintptr_t)ws & 3)) return BZ_ERR_WORKSPACE;
    const Region wr{(uintptr_t)ws, 1, (int64_t)(8 * npx), (int64_t)(8 * npx)};
    if (regions_overlap(wr, input_region(d)) || regions_overlap(wr, output_region(d))) return BZ_ERR_ALIAS;
    const Decision q = make_decision(rule, k, R, win);
    rule = q.rule;
    StagedArgs s;
    s.img = img;
    s.out = out;
    s.r1 = ws;
    s.r2 = ws + npx;
    s.H = H;
    s.W = W_img;
    s.win = win;
    s.lo = win / 2;
    s.hi = win - 1 - s.lo;
    s.segs = (W_img + kSegW - 1) / kSegW;
    s.dec = PageArgs{};
    s.dec.k = q.k;
    s.dec.c1 = q.c1;
    s.dec.c2 = q.c2;
    s.dec.c1n = q.c1n;
    s.dec.c2n2 = q.c2n2;
    hipStream_t st = (hipStream_t)stream;
    if (channels == 1)
        return rule == BZ_SAUVOLA ? staged_launch<1, BZ_SAUVOLA>(s, st) : staged_launch<1, BZ_NIBLACK>(s, st);
    return rule == BZ_SAUVOLA ? staged_launch<3, BZ_SAUVOLA>(s, st) : staged_launch<3, BZ_NIBLACK>(s, st);
}

}  // extern "C"
