// bz_tile.hpp -- gfx950 device code of the exact Sauvola / Niblack tile kernel.
//
// One workgroup (512 threads, 8 wave64s) produces a tile of TW output columns
// by tile_h output rows of one page.  The window statistics of the paper's
// Sec. 2 (mean and deviation over the full W x W window S) come from exact
// integer window sums of f and f^2, built separably inside the tile:
//
//   ring    LDS ring of gray rows (Sec. 1 Eq. 1 applied while staging), one
//           row per image row, win + 16 rows deep, tile plus halo wide.  Each
//           input byte is read from HBM once per tile.
//   V pass  one thread per LDS column slides the vertical window down the
//           tile: V(y) = V(y-1) + f(y+hi) - f(y-lo-1) for V1 = sum f and
//           V2 = sum f^2 (f_in^2 - f_out^2 formed as (f_in - f_out)(f_in + f_out)).
//   H pass  32 threads per output row turn V into the horizontal window sums
//           S(x) = S(x-1) + V(x+hi) - V(x-lo-1): per-thread prefix of the
//           differences, an exclusive scan across the 32 threads and the sum
//           of the first window as the row's starting value.
//   decide  exact D = n S2 - S1^2 in fp64, then the Eq. 4 / Niblack threshold
//           compared with f in fp32 after scaling both sides by n (Eq. 3).
//
// Border windows are clipped: rows and columns outside the image enter the
// sums as zeros and n counts only in-image pixels.  All sums are exact in
// 32-bit integers for win <= 255, so every tile shape gives bit-identical
// results.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bz_common.hpp"

namespace bz {

__device__ __forceinline__ uint32_t align_bytes(uint32_t hi, uint32_t lo, uint32_t sh) {
    return __builtin_amdgcn_alignbyte(hi, lo, sh);
}

// Sec. 1, Eq. 1 in integers: (299 r + 587 g + 114 b + 500) / 1000.  The
// numerator is below 2^18, and for every such value the quotient equals the
// high word of num * ceil(2^32 / 1000) (a 24-bit multiply-high).
__device__ __forceinline__ uint32_t gray_of(uint32_t r, uint32_t g, uint32_t b) {
    const uint32_t num = 299u * r + 587u * g + 114u * b + 500u;
    return (uint32_t)(((uint64_t)num * 4294968ull) >> 32);
}

template <int N>
__device__ __forceinline__ uint32_t byte_at(const uint32_t (&w)[N], int i) {
    return (w[i >> 2] >> (8 * (i & 3))) & 0xffu;
}

// 16 gray levels of image columns [xs, xs + 16) of one image row; columns
// outside [0, W) read as 0.  Only 4-byte words holding at least one byte of
// the row are touched, so no access leaves the caller's buffer's pages.
template <int C>
__device__ __forceinline__ uint4 load_gray16(const uint8_t *__restrict__ rowp, int xs, int W);

template <>
__device__ __forceinline__ uint4 load_gray16<1>(const uint8_t *__restrict__ rowp, int xs, int W) {
    if (xs >= 0 && xs + 16 <= W) {
        const uint8_t *p = rowp + xs;
        const uintptr_t ad = (uintptr_t)p;
        if ((ad & 15) == 0) return *(const uint4 *)p;
        const uint32_t sh = (uint32_t)(ad & 3);
        const uint32_t *q = (const uint32_t *)(ad - sh);
        const uint32_t w0 = q[0], w1 = q[1], w2 = q[2], w3 = q[3];
        const uint32_t w4 = sh ? q[4] : 0u;
        return make_uint4(align_bytes(w1, w0, sh), align_bytes(w2, w1, sh),
                          align_bytes(w3, w2, sh), align_bytes(w4, w3, sh));
    }
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int c = xs + i;
        if (c >= 0 && c < W) w[i >> 2] |= (uint32_t)rowp[c] << (8 * (i & 3));
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

template <>
__device__ __forceinline__ uint4 load_gray16<3>(const uint8_t *__restrict__ rowp, int xs, int W) {
    uint32_t o[4] = {0u, 0u, 0u, 0u};
    if (xs >= 0 && xs + 16 <= W) {
        const uint8_t *p = rowp + 3 * xs;
        const uintptr_t ad = (uintptr_t)p;
        const uint32_t sh = (uint32_t)(ad & 3);
        const uint32_t *q = (const uint32_t *)(ad - sh);
        uint32_t w[13];
#pragma unroll
        for (int i = 0; i < 12; ++i) w[i] = q[i];
        w[12] = sh ? q[12] : 0u;
        uint32_t b[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) b[i] = align_bytes(w[i + 1], w[i], sh);
#pragma unroll
        for (int px = 0; px < 16; ++px)
            o[px >> 2] |= gray_of(byte_at(b, 3 * px), byte_at(b, 3 * px + 1),
                                  byte_at(b, 3 * px + 2)) << (8 * (px & 3));
    } else {
#pragma unroll
        for (int px = 0; px < 16; ++px) {
            const int c = xs + px;
            if (c >= 0 && c < W) {
                const uint8_t *p = rowp + 3 * c;
                o[px >> 2] |= gray_of(p[0], p[1], p[2]) << (8 * (px & 3));
            }
        }
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
}

// Stage `cnt` consecutive image rows starting at row0 into ring slots
// slot0, slot0 + 1, ... (mod depth), LDS columns [0, rp) = image columns
// [xr0, xr0 + rp).  Rows outside the image are stored as zeros.
template <int C>
__device__ __forceinline__ void stage_rows(const PageArgs &a, uint8_t *ring, int row0, int cnt,
                                           int slot0, int xr0) {
    const int nq = a.rp >> 4;
    const int jobs = cnt * nq;
    for (int job = threadIdx.x; job < jobs; job += kThreads) {
        const int i = job / nq;
        const int q = job - i * nq;
        const int row = row0 + i;
        int sl = slot0 + i;
        if (sl >= a.depth) sl -= a.depth;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (row >= 0 && row < a.H)
            v = load_gray16<C>(a.img + (size_t)row * (size_t)a.W * C, xr0 + 16 * q, a.W);
        *(uint4 *)(ring + sl * a.rp + 16 * q) = v;
    }
}

// Sum over the 32 lanes of a row group (all lanes end with the total).
__device__ __forceinline__ uint32_t group_sum(uint32_t v) {
#pragma unroll
    for (int m = kThreadsPerRow / 2; m >= 1; m >>= 1) v += (uint32_t)__shfl_xor((int)v, m, kThreadsPerRow);
    return v;
}

// Exclusive prefix sum over the 32 lanes of a row group (lane s gets the sum
// of lanes 0..s-1).  Unsigned wrap-around is harmless: every final window sum
// is below 2^32.
__device__ __forceinline__ uint32_t group_excl_scan(uint32_t v, int s) {
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < kThreadsPerRow; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)incl, d, kThreadsPerRow);
        if (s >= d) incl += o;
    }
    return incl - v;
}

// Eq. 3 decision for one pixel from its exact window sums.
//   Sauvola (Eq. 4): f < m (1 + k (s/R - 1)) with m = S1/n, s = sqrt(D)/n
//     <=> n^2 f < S1 (n (1 - k) + (k/R) sqrt(D))       (n > 0)
//   Niblack: f < m + k s  <=>  n f - S1 < k sqrt(D)
// D = n S2 - S1^2 is formed exactly in fp64 (every term is an integer below
// 2^53).  n f is exact in fp32 (below 2^24), so a window of constant gray
// level (D = 0) decides ties exactly: Niblack gives f = t and therefore 255.
template <int RULE>
__device__ __forceinline__ uint32_t decide(const PageArgs &a, uint32_t f, uint32_t S1, uint32_t S2,
                                           uint32_t n, float *t_out) {
    const double s1d = (double)S1;
    const double D = __builtin_fma((double)n, (double)S2, -(s1d * s1d));
    const float sq = __builtin_amdgcn_sqrtf((float)D);
    const float nf = (float)n;
    uint32_t g;
    if (RULE == 0) {
        const float lhs = (float)(n * f) * nf;
        const float rhs = (float)S1 * __builtin_fmaf(a.c2, sq, a.c1 * nf);
        g = lhs < rhs ? 0u : 255u;
    } else {
        const int L = (int)(n * f) - (int)S1;
        g = (float)L < a.k * sq ? 0u : 255u;
    }
    if (t_out) {  // verification only: t itself, Eq. 4 / Niblack in fp32
        const float m = (float)S1 / nf;
        const float s = sq / nf;
        *t_out = (RULE == 0) ? m * __builtin_fmaf(a.c2, s, a.c1) : __builtin_fmaf(a.k, s, m);
    }
    return g;
}

// Store OPT output bytes (packed little-endian in w) at columns [xs, xs+OPT)
// of an output row, skipping columns >= W.
template <int OPT>
__device__ __forceinline__ void store_row(uint8_t *rowp, int xs, int W, const uint32_t (&w)[OPT / 4]) {
    if (xs + OPT <= W) {
        uint8_t *p = rowp + xs;
        const uintptr_t ad = (uintptr_t)p;
        if ((ad & (OPT - 1)) == 0) {
            if (OPT == 8)
                *(uint2 *)p = make_uint2(w[0], w[OPT / 4 - 1]);
            else
                *(uint32_t *)p = w[0];
            return;
        }
        if ((ad & 3) == 0) {
#pragma unroll
            for (int i = 0; i < OPT / 4; ++i) ((uint32_t *)p)[i] = w[i];
            return;
        }
    }
#pragma unroll
    for (int j = 0; j < OPT; ++j)
        if (xs + j < W) rowp[xs + j] = (uint8_t)(w[j >> 2] >> (8 * (j & 3)));
}

__device__ __forceinline__ int floor16(int x) { return x & ~15; }  // two's complement: rounds toward -inf

// Workgroups are dispatched round-robin over the 8 XCDs; give every XCD a
// contiguous run of tiles so neighbouring tiles (which share halo columns and
// rows) meet in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

template <int TW, int C, int RULE, bool STATS>
__device__ __forceinline__ void process_tile(const PageArgs &a, int tile, uint8_t *smem) {
    constexpr int RB = kRowsPerStep;
    constexpr int TPR = kThreadsPerRow;
    constexpr int OPT = TW / TPR;  // outputs per thread per row (4 or 8)
    static_assert(OPT == 4 || OPT == 8, "tile width must be 128 or 256");
    constexpr int LOG_OPT = OPT == 8 ? 3 : 2;

    const int tid = threadIdx.x;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int X0 = tx * TW, Y0 = ty * a.tile_h;
    const int Yend = min(Y0 + a.tile_h, a.H);
    const int lo = a.lo, hi = a.hi, win = a.win;
    const int xr0 = floor16(X0 - lo - 1);  // image column of LDS column 0
    const int off0 = X0 - lo - xr0;        // LDS column of the first window column, 1..16
    const int rp = a.rp, depth = a.depth, vp = a.vp;
    const int vrow = OPT * vp;
    uint8_t *ring = smem;
    uint16_t *V1 = (uint16_t *)(smem + a.off_v1);
    uint32_t *V2 = (uint32_t *)(smem + a.off_v2);
    const int base = Y0 - lo - 1;  // image row held by ring slot 0

    auto vpos = [&](int c) { return (c & (OPT - 1)) * vp + (c >> LOG_OPT); };

    // ---- start-up: rows [Y0-lo-1, Y0+hi-1] give V at row Y0-1
    stage_rows<C>(a, ring, base, win, 0, xr0);
    __syncthreads();
    const int c = tid;
    const bool vcol = c < rp;
    const int cpos = vpos(c);
    uint32_t v1 = 0, v2 = 0;
    if (vcol) {
        for (int i = 0; i < win; ++i) {
            const uint32_t f = ring[i * rp + c];
            v1 += f;
            v2 += f * f;
        }
    }

    const int hr = tid / TPR, hs = tid % TPR;

    for (int y0 = Y0; y0 < Yend; y0 += RB) {
        const int s_in = (y0 + hi - base) % depth;  // slot of the first entering row
        __syncthreads();
        stage_rows<C>(a, ring, y0 + hi, RB, s_in, xr0);
        __syncthreads();

        // ---- vertical pass: one LDS column per thread, RB rows
        if (vcol) {
            int se = s_in, sx = (y0 - Y0) % depth;  // entering / leaving row slots
#pragma unroll 4
            for (int r = 0; r < RB; ++r) {
                const int fn = ring[se * rp + c], fo = ring[sx * rp + c];
                const int d = fn - fo;
                v1 += (uint32_t)d;
                v2 += (uint32_t)(d * (fn + fo));
                V1[r * vrow + cpos] = (uint16_t)v1;
                V2[r * vrow + cpos] = v2;
                se = (se + 1 == depth) ? 0 : se + 1;
                sx = (sx + 1 == depth) ? 0 : sx + 1;
            }
        }
        __syncthreads();

        // ---- horizontal pass + threshold: 32 threads per output row
        const int y = y0 + hr;
        if (y < Yend) {  // uniform across each 32-lane row group
            const uint16_t *V1r = V1 + hr * vrow;
            const uint32_t *V2r = V2 + hr * vrow;
            // starting value: the window sum one column left of the tile
            uint32_t h1 = 0, h2 = 0;
            for (int cc = off0 - 1 + hs; cc < off0 - 1 + win; cc += TPR) {
                const int p = vpos(cc);
                h1 += V1r[p];
                h2 += V2r[p];
            }
            h1 = group_sum(h1);
            h2 = group_sum(h2);
            uint32_t E1[OPT], E2[OPT];
            uint32_t a1 = 0, a2 = 0;
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int xj = hs * OPT + j;
                const int pa = vpos(off0 + xj + win - 1), pb = vpos(off0 + xj - 1);
                a1 += (uint32_t)V1r[pa] - (uint32_t)V1r[pb];
                a2 += V2r[pa] - V2r[pb];
                E1[j] = a1;
                E2[j] = a2;
            }
            const uint32_t b1 = h1 + group_excl_scan(a1, hs);
            const uint32_t b2 = h2 + group_excl_scan(a2, hs);

            // gray levels of the output row (centre of the window)
            const int fo = ((y - base) % depth) * rp + off0 + lo + hs * OPT;
            const uint32_t fsh = (uint32_t)(fo & 3);
            const uint32_t *fq = (const uint32_t *)(smem + (fo & ~3));
            uint32_t fw[OPT / 4];
#pragma unroll
            for (int i = 0; i < OPT / 4; ++i) fw[i] = align_bytes(fq[i + 1], fq[i], fsh);

            const int ny = min(y + hi, a.H - 1) - max(y - lo, 0) + 1;
            uint32_t ow[OPT / 4];
#pragma unroll
            for (int i = 0; i < OPT / 4; ++i) ow[i] = 0u;
            const int xs = X0 + hs * OPT;
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int X = xs + j;
                const uint32_t S1 = b1 + E1[j], S2 = b2 + E2[j];
                const int nx = min(X + hi, a.W - 1) - max(X - lo, 0) + 1;
                const uint32_t n = (uint32_t)(nx * ny);
                const uint32_t f = byte_at(fw, j);
                float t;
                const uint32_t g = decide<RULE>(a, f, S1, S2, n, STATS ? &t : nullptr);
                ow[j >> 2] |= g << (8 * (j & 3));
                if (STATS && X < a.W) {
                    const size_t i = (size_t)y * a.W + X;
                    if (a.gray) a.gray[i] = (uint8_t)f;
                    if (a.s1) a.s1[i] = S1;
                    if (a.s2) a.s2[i] = S2;
                    if (a.n) a.n[i] = n;
                    if (a.t) a.t[i] = t;
                }
            }
            store_row<OPT>(a.out + (size_t)y * a.W, xs, a.W, ow);
        }
    }
}

template <int TW, int C, int RULE, bool STATS>
__global__ void __launch_bounds__(kThreads) bz_page_kernel(PageArgs a) {
    extern __shared__ uint4 bz_lds[];
    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    process_tile<TW, C, RULE, STATS>(a, tile, (uint8_t *)bz_lds);
}

}  // namespace bz
