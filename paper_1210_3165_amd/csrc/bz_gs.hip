// bz_gs.hip -- the paper's sampled-window Sauvola (Sec. 2, Eq. 5) and the
// F-measure counts of Sec. 3 (Eq. 6) on gfx950.
//
// Sampled window.  The threshold t' = m' [1 + k (s'/R' - 1)] takes its mean
// m' and deviation s' from a subset S' of the window: O(W) pixels on a
// geometric structure.  The paper's own structures (its Fig. 1) are not
// available; this library defines three for odd windows (r = win / 2),
// as offsets (dy, dx) from the centre:
//   BZ_GS_PLUS  dy == 0 or dx == 0        centre row and column, 2 win - 1
//   BZ_GS_X     |dy| == |dx|              both diagonals,        2 win - 1
//   BZ_GS_STAR  the union of the two,                            4 win - 3
// clipped to the image (n' = in-image members).
//
// One workgroup makes a tile of 128 x 32 outputs.  It stages the gray levels
// of the tile and its r-wide halo into LDS (Eq. 1 applied on the way; pixels
// outside the image stage as 0 and are left out of n').  The line sums are
// then sliding sums, O(1) per pixel and line instead of the 2r + 1 samples of
// a direct walk:
//   rows       128 walkers (32 rows x 4 segments of 32 outputs) slide along
//              the rows,
//   diagonals  159 walkers, one per diagonal crossing the tile, slide down
//              and right from the tile's top or left edge,
//   anti-diagonals  159 walkers slide down and left from the top or right
//              edge,
// each pass adding its line sums of f and f^2 into an LDS accumulator per
// output (a barrier between passes), and finally 256 walkers, two per column,
// slide down the columns, add the column line, remove the extra copies of the
// centre and decide.  Each walker pays 2r + 1 samples once to start.  S1' and
// S2' are exact 32-bit sums (S2' < 2^27); n' has a closed form per line.  The
// decision reuses the exact-sum helpers of the full-window kernel
// (D' = n' S2' - S1'^2 formed exactly, scaled fp32 comparison), so the same
// error bound holds.
//
// F-measure.  Counts TP (out == 0 where the ground truth marks text), FP
// (out == 0 on background) and FN (out != 0 on text) in 64-bit counters.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "binarize.h"
#include "bz_common.hpp"
#include "bz_host.hpp"
#include "bz_tile.hpp"

namespace {

using namespace bz;

constexpr int kGsThreads = 256;
constexpr int kGsTW = 128;  // output columns per tile (one lane each)
constexpr int kGsTH = 32;   // output rows per tile

struct GsArgs {
    const uint8_t *img;
    uint8_t *out;
    uint32_t *s1, *s2, *n;
    float *t;
    int H, W, r;
    int pitch;    // LDS row pitch (bytes)
    int tiles_x, n_tiles;
    PageArgs dec; // k, c1 = 1 - k, c2 = k / R' (fp64) for the decision helpers
};

// Staged row pitch: the tile plus halo plus up to 15 columns of chunk
// alignment and one chunk of slack, and an odd number of words, so that
// walkers on consecutive rows read different banks.
__host__ __device__ inline int gs_pitch(int r) { return round_up(kGsTW + 2 * r + 32, 8) + 4; }
// Accumulator row pitch in words (odd for the same reason).
constexpr int kGsAccPitch = kGsTW + 1;
__host__ __device__ inline int gs_stage_bytes(int r) { return round_up((kGsTH + 2 * r) * gs_pitch(r), 16); }
__host__ __device__ inline int gs_lds(int r) { return gs_stage_bytes(r) + 2 * 4 * kGsTH * kGsAccPitch; }

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

template <int C, int ST, int RULE, bool STATS>
__global__ __launch_bounds__(kGsThreads) void bz_gs_kernel(const GsArgs g) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int tid = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, g.n_tiles);
    const int ty = tile / g.tiles_x, tx = tile - ty * g.tiles_x;
    const int x0 = tx * kGsTW, y0 = ty * kGsTH;
    const int r = g.r, rows = kGsTH + 2 * r, cols = kGsTW + 2 * r;

    // stage the tile and its halo as gray levels (0 outside the image) in
    // 16-pixel chunks starting on multiples of 16 image columns: LDS column 0
    // holds image column xr0 = floor16(x0 - r), and staged column c (image
    // column x0 - r + c) sits at LDS column off + c.  A job is one chunk of
    // one row, fetched with word loads clamped to the row and reduced to gray
    // levels by the tile kernel's helpers; each lane runs two jobs at a time.
    const int xr0 = floor16(x0 - r), off = x0 - r - xr0;
    {
        const int nq = (off + cols + 15) >> 4;  // chunks per staged row
        const int jobs = rows * nq;
        for (int j0 = tid; j0 < jobs; j0 += 2 * kGsThreads) {
            RawChunk<C> k[2];
            bool ok[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int j = j0 + u * kGsThreads;
                ok[u] = false;
                if (j < jobs) {
                    const int ry = j / nq, q = j - ry * nq, yy = y0 - r + ry;
                    ok[u] = yy >= 0 && yy < g.H;
                    const int yc = imin(imax(yy, 0), g.H - 1);
                    fetch_chunk<C, false>(k[u], g.img + (size_t)yc * g.W * C, xr0 + 16 * q, g.W, true);
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int j = j0 + u * kGsThreads;
                if (j < jobs) {
                    const int ry = j / nq, q = j - ry * nq;
                    uint4 v = chunk_gray<C, false>(k[u], xr0 + 16 * q, g.W, true);
                    if (!ok[u]) v = make_uint4(0u, 0u, 0u, 0u);
                    uint32_t *d = reinterpret_cast<uint32_t *>(lds + ry * g.pitch + 16 * q);  // 4-byte aligned
                    d[0] = v.x;
                    d[1] = v.y;
                    d[2] = v.z;
                    d[3] = v.w;
                }
            }
        }
    }
    __syncthreads();
    const uint8_t *stg = lds + off;  // staged column 0

    const int P = g.pitch, w2 = 2 * r;
    uint32_t *acc1 = reinterpret_cast<uint32_t *>(lds + gs_stage_bytes(r));  // [kGsTH][kGsAccPitch]
    uint32_t *acc2 = acc1 + kGsTH * kGsAccPitch;
    constexpr bool HV = ST != BZ_GS_X;    // the row and the column through the centre
    constexpr bool DG = ST != BZ_GS_PLUS;  // the two diagonals
    // Staged coordinates: output (cx, cy) sits at row cy + r, column cx + r.

    // A walker starts with the line sum of its first cell (2r + 1 samples) and
    // slides: cell k adds the sample entering at staged offset in0 + k * din
    // and drops the one leaving at out0 + (k - 1) * dout, for L cells whose
    // accumulators sit at acc0 + k * dacc.  Reads are issued four cells at a
    // time, so each LDS round trip serves four cells.
    auto walk = [&](int first, int step_first, int in0, int din, int out0, int dout, int acc0, int dacc, int L,
                    bool add) {
        uint32_t a = 0, b = 0;
        for (int t = 0; t <= w2; ++t) {
            const uint32_t v = stg[first + t * step_first];
            a += v;
            b += __umul24(v, v);
        }
        for (int k0 = 0; k0 < L; k0 += 4) {
            uint32_t vi[4], vo[4], c1[4], c2[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = k0 + s;
                vi[s] = vo[s] = c1[s] = c2[s] = 0u;
                if (k < L) {
                    if (k > 0) {
                        vi[s] = stg[in0 + k * din];
                        vo[s] = stg[out0 + (k - 1) * dout];
                    }
                    if (add) {
                        c1[s] = acc1[acc0 + k * dacc];
                        c2[s] = acc2[acc0 + k * dacc];
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = k0 + s;
                if (k < L) {
                    a += vi[s] - vo[s];
                    b += __umul24(vi[s], vi[s]) - __umul24(vo[s], vo[s]);
                    acc1[acc0 + k * dacc] = c1[s] + a;
                    acc2[acc0 + k * dacc] = c2[s] + b;
                }
            }
        }
    };

    // rows: the line of output (cx, cy) is staged row cy + r, columns cx .. cx + 2r;
    // 128 walkers (32 rows x 4 segments of 32 outputs)
    if (HV) {
        if (tid < kGsTH * 4) {
            const int cy = tid & (kGsTH - 1), cx0 = (tid >> 5) * 32;
            const int row = (cy + r) * P + cx0;
            walk(row, 1, row + w2, 1, row, 1, cy * kGsAccPitch + cx0, 1, 32, false);
        }
        __syncthreads();
    }
    if (DG) {
        constexpr int ND = kGsTW + kGsTH - 1;  // diagonals crossing the tile
        // diagonals: the line of (cx, cy) is staged (cy + t, cx + t), t = 0 .. 2r;
        // walkers start on the top edge (tid < 128) or the left edge and move
        // down and right
        if (tid < ND) {
            const int cx = tid < kGsTW ? tid : 0, cy = tid < kGsTW ? 0 : tid - kGsTW + 1;
            const int L = imin(kGsTW - cx, kGsTH - cy);
            const int c = cy * P + cx;
            walk(c, P + 1, c + w2 * (P + 1), P + 1, c, P + 1, cy * kGsAccPitch + cx, kGsAccPitch + 1, L, HV);
        }
        __syncthreads();
        // anti-diagonals: the line of (cx, cy) is staged (cy + t, cx + 2r - t);
        // walkers start on the top edge (tid < 128) or the right edge and move
        // down and left
        if (tid < ND) {
            const int cx = tid < kGsTW ? tid : kGsTW - 1, cy = tid < kGsTW ? 0 : tid - kGsTW + 1;
            const int L = imin(cx + 1, kGsTH - cy);
            const int c = cy * P + cx;
            walk(c + w2, P - 1, c + w2 * P, P - 1, c + w2, P - 1, cy * kGsAccPitch + cx, kGsAccPitch - 1, L, true);
        }
        __syncthreads();
    }

    // columns and the decision: two walkers per column, 16 rows each; the
    // column line of (cx, cy) is staged rows cy .. cy + 2r, column cx + r
    const int cx = tid & (kGsTW - 1);
    const int x = x0 + cx;
    if (x >= g.W) return;
    constexpr int kHalf = kGsTH / (kGsThreads / kGsTW);
    const int cy0 = (tid / kGsTW) * kHalf;
    const uint8_t *col = stg + cx + r;
    uint32_t va = 0, vb = 0;
    if (HV)
        for (int t = 0; t <= w2; ++t) {
            const uint32_t v = col[(cy0 + t) * P];
            va += v;
            vb += __umul24(v, v);
        }
    for (int cy = cy0; cy < cy0 + kHalf; ++cy) {
        const int y = y0 + cy;
        if (y >= g.H) break;
        if (HV && cy > cy0) {
            const uint32_t in = col[(cy + w2) * P], out = col[(cy - 1) * P];
            va += in - out;
            vb += __umul24(in, in) - __umul24(out, out);
        }
        const uint32_t f = col[(cy + r) * P];
        const int i = cy * kGsAccPitch + cx;
        // every line passes through the centre: keep one copy of it
        const uint32_t extra = ST == BZ_GS_STAR ? 3u : 1u;
        const uint32_t S1 = acc1[i] + va - extra * f, S2 = acc2[i] + vb - extra * __umul24(f, f);
        // in-image members of each line
        int cnt = 0;
        if (HV) {
            const int nv = imin(y + r, g.H - 1) - imax(y - r, 0) + 1;
            const int nh = imin(x + r, g.W - 1) - imax(x - r, 0) + 1;
            cnt += nv + nh;
        }
        if (DG) {
            // (y + t, x + t) and (y + t, x - t) for |t| <= r
            const int nd = imin(imin(r, g.H - 1 - y), g.W - 1 - x) - imax(imax(-r, -y), -x) + 1;
            const int na = imin(imin(r, g.H - 1 - y), x) - imax(imax(-r, -y), x - (g.W - 1)) + 1;
            cnt += nd + na;
        }
        const uint32_t n = (uint32_t)cnt - extra;
        float sq;
        const bool dark = RULE == BZ_SAUVOLA ? dark_sauvola(g.dec, f, S1, S2, n, sq)
                                             : dark_niblack(g.dec, f, S1, S2, n, sq);
        const size_t o = (size_t)y * g.W + x;
        g.out[o] = dark ? 0 : 255;
        if (STATS) {
            if (g.s1) g.s1[o] = S1;
            if (g.s2) g.s2[o] = S2;
            if (g.n) g.n[o] = n;
            if (g.t) g.t[o] = threshold_value<RULE>(g.dec, S1, n, sq);
        }
    }
}

constexpr int kFmThreads = 256;

__global__ void bz_fm_zero(unsigned long long *counts) {
    if (threadIdx.x < 3) counts[threadIdx.x] = 0;
}

__device__ __forceinline__ void fm_count(uint32_t o, uint32_t g, uint32_t &tp, uint32_t &fp, uint32_t &fn) {
    const bool fg = o == 0, truth = g != 0;
    tp += fg && truth;
    fp += fg && !truth;
    fn += !fg && truth;
}

template <bool ALIGNED>
__global__ __launch_bounds__(kFmThreads) void bz_fm_kernel(const uint8_t *__restrict__ out,
                                                           const uint8_t *__restrict__ gt, long npx,
                                                           unsigned long long *counts) {
    __shared__ uint32_t red[3][kFmThreads / 64];
    const int tid = threadIdx.x;
    const long stride = (long)gridDim.x * kFmThreads;
    uint32_t tp = 0, fp = 0, fn = 0;
    if (ALIGNED) {
        const long nq = npx / 16;
        for (long j = (long)blockIdx.x * kFmThreads + tid; j < nq; j += stride) {
            const uint4 o = reinterpret_cast<const uint4 *>(out)[j];
            const uint4 q = reinterpret_cast<const uint4 *>(gt)[j];
            const uint32_t ow[4] = {o.x, o.y, o.z, o.w}, gw[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int p = 0; p < 16; ++p)
                fm_count((ow[p >> 2] >> (8 * (p & 3))) & 0xffu, (gw[p >> 2] >> (8 * (p & 3))) & 0xffu, tp, fp, fn);
        }
        if (blockIdx.x == 0)
            for (long i = nq * 16 + tid; i < npx; i += kFmThreads) fm_count(out[i], gt[i], tp, fp, fn);
    } else {
        for (long i = (long)blockIdx.x * kFmThreads + tid; i < npx; i += stride) fm_count(out[i], gt[i], tp, fp, fn);
    }
    // per-lane counts stay below 2^32 (each lane sees < 2^31 pixels)
    for (int off = 32; off > 0; off >>= 1) {
        tp += __shfl_down(tp, off);
        fp += __shfl_down(fp, off);
        fn += __shfl_down(fn, off);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = tp;
        red[1][tid >> 6] = fp;
        red[2][tid >> 6] = fn;
    }
    __syncthreads();
    if (tid < 3) {
        unsigned long long s = 0;
        for (int w = 0; w < kFmThreads / 64; ++w) s += red[tid][w];
        if (s) atomicAdd(&counts[tid], s);
    }
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

int fail(hipError_t e) {
    set_last_hip_error((int)e);
    return BZ_ERR_HIP;
}

int device_cus() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
        return 256;
    return v;
}

template <int C, int ST, int RULE, bool STATS>
int gs_launch(const GsArgs &g, hipStream_t st) {
    auto kern = bz_gs_kernel<C, ST, RULE, STATS>;
    static std::once_flag once[kMaxDevices];
    once_per_device(once, [&] {
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
        (void)hipGetLastError();
    });
    hipLaunchKernelGGL(kern, dim3((unsigned)g.n_tiles), dim3(kGsThreads), (unsigned)gs_lds(g.r), st, g);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BZ_OK : fail(e);
}

template <int C, int ST, int RULE>
int gs_s(const GsArgs &g, bool stats, hipStream_t st) {
    return stats ? gs_launch<C, ST, RULE, true>(g, st) : gs_launch<C, ST, RULE, false>(g, st);
}

template <int C, int ST>
int gs_r(const GsArgs &g, int rule, bool stats, hipStream_t st) {
    return rule == BZ_SAUVOLA ? gs_s<C, ST, BZ_SAUVOLA>(g, stats, st) : gs_s<C, ST, BZ_NIBLACK>(g, stats, st);
}

template <int C>
int gs_st(const GsArgs &g, int structure, int rule, bool stats, hipStream_t st) {
    switch (structure) {
        case BZ_GS_PLUS: return gs_r<C, BZ_GS_PLUS>(g, rule, stats, st);
        case BZ_GS_X: return gs_r<C, BZ_GS_X>(g, rule, stats, st);
        default: return gs_r<C, BZ_GS_STAR>(g, rule, stats, st);
    }
}

}  // namespace

extern "C" {

int binarize_gs(const uint8_t *img, int H, int W_img, int channels, int win, float k, float Rp,
                int structure, uint8_t *out, uint32_t *s1, uint32_t *s2, uint32_t *n, float *t,
                void *stream) {
    if (!img || !out) return BZ_ERR_NULL;
    if (H < 1 || W_img < 1) return BZ_ERR_SHAPE;
    if (channels != 1 && channels != 3) return BZ_ERR_CHANNELS;
    const int64_t npx = (int64_t)H * W_img;
    if (npx * channels >= ((int64_t)1 << 31)) return BZ_ERR_SHAPE;
    if (win < 1 || win > 255 || win % 2 == 0) return BZ_ERR_WINDOW;
    if (structure != BZ_GS_PLUS && structure != BZ_GS_X && structure != BZ_GS_STAR) return BZ_ERR_PARAM;
    if (check_params(BZ_SAUVOLA, k, Rp)) return BZ_ERR_PARAM;  // |k| <= 1, R' >= 64: the 1e-4 bound
    const void *planes[5] = {out, s1, s2, n, t};
    const size_t sizes[5] = {(size_t)npx, 4 * (size_t)npx, 4 * (size_t)npx, 4 * (size_t)npx, 4 * (size_t)npx};
    for (int i = 0; i < 5; ++i) {
        if (!planes[i]) continue;
        if (overlaps(planes[i], sizes[i], img, (size_t)(npx * channels))) return BZ_ERR_ALIAS;
        for (int j = 0; j < i; ++j)
            if (planes[j] && overlaps(planes[i], sizes[i], planes[j], sizes[j])) return BZ_ERR_ALIAS;
    }
    GsArgs g{};
    g.img = img;
    g.out = out;
    g.s1 = s1;
    g.s2 = s2;
    g.n = n;
    g.t = t;
    g.H = H;
    g.W = W_img;
    g.r = win / 2;
    g.pitch = gs_pitch(g.r);
    g.tiles_x = (W_img + kGsTW - 1) / kGsTW;
    g.n_tiles = g.tiles_x * ((H + kGsTH - 1) / kGsTH);
    // k = 0 makes t' = m', the Niblack form with k = 0 (exact ties)
    const Decision q = make_decision(BZ_SAUVOLA, k, Rp, win);
    g.dec.k = q.k;
    g.dec.c1 = q.c1;
    g.dec.c2 = q.c2;
    const int rule = q.rule;
    const bool stats = s1 || s2 || n || t;
    hipStream_t st = (hipStream_t)stream;
    return channels == 1 ? gs_st<1>(g, structure, rule, stats, st) : gs_st<3>(g, structure, rule, stats, st);
}

int binarize_fmeasure_counts(const uint8_t *out, const uint8_t *gt, int64_t npx, unsigned long long *counts,
                             void *stream) {
    if (!out || !gt || !counts) return BZ_ERR_NULL;
    if (npx < 1 || npx >= ((int64_t)1 << 31)) return BZ_ERR_SHAPE;
    if (((uintptr_t)counts & 7) != 0) return BZ_ERR_WORKSPACE;
    if (overlaps(counts, 24, out, (size_t)npx) || overlaps(counts, 24, gt, (size_t)npx)) return BZ_ERR_ALIAS;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(bz_fm_zero, dim3(1), dim3(64), 0, st, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(e);
    const bool aligned = (((uintptr_t)out | (uintptr_t)gt) & 15) == 0;
    const long units = aligned ? npx / 16 : npx;
    long grid = (units + kFmThreads - 1) / kFmThreads;
    const long cap = 4L * device_cus();
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    if (aligned)
        hipLaunchKernelGGL(bz_fm_kernel<true>, dim3((unsigned)grid), dim3(kFmThreads), 0, st, out, gt, (long)npx,
                           counts);
    else
        hipLaunchKernelGGL(bz_fm_kernel<false>, dim3((unsigned)grid), dim3(kFmThreads), 0, st, out, gt, (long)npx,
                           counts);
    e = hipGetLastError();
    return e == hipSuccess ? BZ_OK : fail(e);
}

}  // extern "C"
