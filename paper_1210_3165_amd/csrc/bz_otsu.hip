// bz_otsu.hip -- Otsu's global threshold on gfx950: the paper's global
// baseline (Sec. 1, Eq. 2) with its threshold T from Otsu's method.
//
//   otsu_hist    one workgroup per CU streams its share of the image once (16
//                pixels per lane per load, 16-byte loads, up to 4 loads in
//                flight per lane), reduces every pixel
//                to its Eq. 1 gray level and counts it in LDS with one
//                sub-histogram per lane position, laid out [level][lane]: the
//                64 lanes of a wave always hit 64 different banks, whatever
//                levels they carry.  The sub-histograms are summed and stored
//                as the workgroup's row of 256 counts in the workspace (plain
//                stores: no device atomics, no fences).
//   otsu_select  one workgroup sums the rows into the histogram and selects
//                k*: prefix counts and level sums by wave scans over four
//                waves of 64 levels joined by one barrier, the between-class
//                variance w0 w1 (mu0 - mu1)^2 of every split in fp64, and the
//                first split of largest variance (wave reductions, then over
//                the four waves).  It stores the
//                histogram, k* and T = k* + 1 in the workspace.
//   otsu_apply   out = 0 where f < T, 255 elsewhere (Eq. 2), 16 pixels per
//                lane per step, again from 16-byte loads and stores (the
//                stores non-temporal: the output is not read back).
//
// The kernel boundaries order the three steps; every call rewrites every
// workspace word it reads, so the workspace needs no initialisation.  The
// histogram and the decision are bound by HBM: the first reads C bytes per
// pixel, the second reads C and writes 1.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "binarize.h"
#include "bz_common.hpp"
#include "bz_tile.hpp"

namespace {

using namespace bz;

constexpr int kHistThreads = 1024;
constexpr int kSelectThreads = 1024;
constexpr int kApplyThreads = 256;
constexpr int kLanes = 64;       // sub-histograms, one per lane position
constexpr int kPx = 16;          // pixels per lane per step

// Workspace words (the public offsets are in binarize.h).
constexpr int kWsHist = BZ_OTSU_WS_HIST;
constexpr int kWsT = BZ_OTSU_WS_T;
constexpr int kWsK = BZ_OTSU_WS_KSTAR;
constexpr int kWsRows = 1024;     // per-workgroup rows of 256 counts
constexpr int kMaxRows = (BZ_OTSU_WS_BYTES / 4 - kWsRows) / 256;
static_assert(kMaxRows >= 256, "workspace holds a row per CU");

// 16 gray levels of the pixels of one chunk (16 * C bytes, 16-byte aligned).
template <int C>
__device__ __forceinline__ void load_chunk(const uint8_t *p, uint32_t (&w)[4 * C]) {
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const uint4 v = q[i];
        w[4 * i + 0] = v.x;
        w[4 * i + 1] = v.y;
        w[4 * i + 2] = v.z;
        w[4 * i + 3] = v.w;
    }
}

template <int C>
__device__ __forceinline__ uint32_t level(const uint32_t (&w)[4 * C], int px) {
    if (C == 1) return byte_at(w, px);
    return gray_of(byte_at(w, 3 * px), byte_at(w, 3 * px + 1), byte_at(w, 3 * px + 2));
}

template <int C>
__device__ __forceinline__ uint32_t level_at(const uint8_t *img, long i) {
    if (C == 1) return img[i];
    return gray_of(img[3 * i], img[3 * i + 1], img[3 * i + 2]);
}

// Between-class variance of the split {f <= k} / {f > k}: n0, s0 are the
// count and level sum of the lower class, n, s those of the image.
__device__ __forceinline__ double between_var(uint64_t n0, uint64_t s0, uint64_t n, uint64_t s) {
    const uint64_t n1 = n - n0, s1 = s - s0;
    if (n0 == 0 || n1 == 0) return 0.0;
    const double w0 = (double)n0 / (double)n;
    const double w1 = (double)n1 / (double)n;
    const double mu0 = (double)s0 / (double)n0;
    const double mu1 = (double)s1 / (double)n1;
    const double d = mu0 - mu1;
    return w0 * w1 * (d * d);
}

// Sum the rows of the histogram workgroups, then select k* and T.  `copy`
// (optional) receives the histogram, T and k* as well, at the workspace's
// offsets.
__global__ __launch_bounds__(kSelectThreads) void otsu_select(uint32_t *__restrict__ ws, int rows,
                                                              uint32_t *__restrict__ copy) {
    constexpr int kParts = kSelectThreads / 64;  // rows summed in parallel
    __shared__ uint4 part[kParts][64];
    __shared__ uint32_t wn[4];              // per wave of levels: total count
    __shared__ unsigned long long ws64[4];  // and total level sum
    __shared__ double sv[4];
    __shared__ int si[4];
    uint32_t n_lvl = 0;                     // this thread's level: prefix count
    unsigned long long s_lvl = 0;           // and prefix level sum
    const int tid = threadIdx.x;
    {
        // thread: levels 4q..4q+3 (q = tid % 64) of rows tid / 64 + 16 i,
        // as 16-byte loads, 16 of them in flight
        constexpr int kUnroll = 16;
        const uint4 *col = reinterpret_cast<const uint4 *>(ws + kWsRows) + (tid & 63);
        uint4 acc = make_uint4(0, 0, 0, 0);
        int r = tid >> 6;
        for (; r + (kUnroll - 1) * kParts < rows; r += kUnroll * kParts) {
            uint4 v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) v[u] = col[(r + u * kParts) * 64];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                acc.x += v[u].x;
                acc.y += v[u].y;
                acc.z += v[u].z;
                acc.w += v[u].w;
            }
        }
        for (; r < rows; r += kParts) {
            const uint4 v = col[r * 64];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
        part[tid >> 6][tid & 63] = acc;
    }
    __syncthreads();
    // Levels 0..255 on the first four waves, level = tid: inclusive prefix
    // sums of the counts and level sums inside each wave (shuffles), then
    // the totals of the waves before it (one barrier); the first split of
    // largest variance per wave, then over the four waves (one barrier).
    uint32_t h = 0;
    if (tid < 256) {
        const uint32_t *pw = reinterpret_cast<const uint32_t *>(&part[0][0]);
#pragma unroll
        for (int p = 0; p < kParts; ++p) h += pw[p * 256 + tid];
        const int lane = tid & 63;
        uint32_t n0 = h;
        unsigned long long s0 = (unsigned long long)tid * h;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t a = __shfl_up(n0, off, 64);
            const unsigned long long b = __shfl_up(s0, off, 64);
            if (lane >= off) {
                n0 += a;
                s0 += b;
            }
        }
        if (lane == 63) {
            wn[tid >> 6] = n0;
            ws64[tid >> 6] = s0;
        }
        n_lvl = n0;
        s_lvl = s0;
    }
    __syncthreads();
    if (tid < 256) {
        const int w = tid >> 6, lane = tid & 63;
        uint32_t n = 0;
        unsigned long long s = 0;
        for (int i = 0; i < 4; ++i) {
            if (i < w) {
                n_lvl += wn[i];
                s_lvl += ws64[i];
            }
            n += wn[i];
            s += ws64[i];
        }
        double v = between_var(n_lvl, s_lvl, n, s);
        int k = tid;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double vo = __shfl_xor(v, off, 64);
            const int ko = __shfl_xor(k, off, 64);
            if (vo > v || (vo == v && ko < k)) {
                v = vo;
                k = ko;
            }
        }
        if (lane == 0) {
            sv[w] = v;
            si[w] = k;
        }
    }
    __syncthreads();
    if (tid == 0) {  // waves in level order: a later wave wins only with a larger variance
        for (int w = 1; w < 4; ++w)
            if (sv[w] > sv[0]) {
                sv[0] = sv[w];
                si[0] = si[w];
            }
    }
    __syncthreads();
    if (tid < 256) ws[kWsHist + tid] = h;
    if (tid == 0) {
        ws[kWsK] = (uint32_t)si[0];
        ws[kWsT] = (uint32_t)si[0] + 1u;
    }
    if (copy) {
        if (tid < 256) copy[kWsHist + tid] = h;
        if (tid == 0) {
            copy[kWsK] = (uint32_t)si[0];
            copy[kWsT] = (uint32_t)si[0] + 1u;
        }
    }
}

template <int C, bool ALIGNED>
__global__ __launch_bounds__(kHistThreads) void otsu_hist(const uint8_t *__restrict__ img, long npx,
                                                          uint32_t *__restrict__ ws) {
    __shared__ uint32_t hist[256 * kLanes];  // [level][lane]
    const int tid = threadIdx.x;
    for (int i = tid; i < 256 * kLanes; i += kHistThreads) hist[i] = 0;
    __syncthreads();
    uint32_t *mine = hist + (tid & (kLanes - 1));
#define BZ_COUNT(f) atomicAdd(&mine[(f) * kLanes], 1u)

    const long stride = (long)gridDim.x * kHistThreads;
    if (ALIGNED) {
        // rounds of U chunks per thread, all U loads issued before any is
        // counted: a page of a few Mpx is one or two rounds, so the wait is
        // one memory latency per round instead of one per chunk
        constexpr int U = C == 1 ? 4 : 2;
        const long nchunks = npx / kPx;
        for (long j0 = (long)blockIdx.x * kHistThreads + tid; j0 < nchunks; j0 += U * stride) {
            uint32_t w[U][4 * C];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (j0 + u * stride < nchunks) load_chunk<C>(img + (j0 + u * stride) * (kPx * C), w[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (j0 + u * stride < nchunks) {
#pragma unroll
                    for (int p = 0; p < kPx; ++p) BZ_COUNT(level<C>(w[u], p));
                }
        }
        // the last npx % 16 pixels
        if (blockIdx.x == 0)
            for (long i = nchunks * kPx + tid; i < npx; i += kHistThreads)
                BZ_COUNT(level_at<C>(img, i));
    } else {
        for (long i = (long)blockIdx.x * kHistThreads + tid; i < npx; i += stride)
            BZ_COUNT(level_at<C>(img, i));
    }
#undef BZ_COUNT
    __syncthreads();

    if (tid < 256) {
        // level tid: sum its 64 lane counts, starting at lane tid % 64 so
        // that the 64 lanes of a wave read 64 different banks
        const uint32_t *row = hist + tid * kLanes;
        uint32_t v = 0;
#pragma unroll 16
        for (int c = 0; c < kLanes; ++c) v += row[(c + tid) & (kLanes - 1)];
        ws[kWsRows + blockIdx.x * 256 + tid] = v;
    }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int C, bool ALIGNED>
__global__ __launch_bounds__(kApplyThreads) void otsu_apply(const uint8_t *__restrict__ img,
                                                            uint8_t *__restrict__ out, long npx,
                                                            const uint32_t *__restrict__ ws) {
    const uint32_t T = ws[kWsT];
    const int tid = threadIdx.x;
    const long stride = (long)gridDim.x * kApplyThreads;
    if (ALIGNED) {
        const long nchunks = npx / kPx;
        for (long j = (long)blockIdx.x * kApplyThreads + tid; j < nchunks; j += stride) {
            uint32_t w[4 * C];
            load_chunk<C>(img + j * (kPx * C), w);
            uint32_t o[4] = {0, 0, 0, 0};
#pragma unroll
            for (int p = 0; p < kPx; ++p)
                if (level<C>(w, p) >= T) o[p >> 2] |= 0xffu << (8 * (p & 3));
            // written once, never read back here: non-temporal (streaming) store
            const u32x4 v = {o[0], o[1], o[2], o[3]};
            __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(out + j * kPx));
        }
        if (blockIdx.x == 0)
            for (long i = nchunks * kPx + tid; i < npx; i += kApplyThreads)
                out[i] = level_at<C>(img, i) < T ? 0 : 255;
    } else {
        for (long i = (long)blockIdx.x * kApplyThreads + tid; i < npx; i += stride)
            out[i] = level_at<C>(img, i) < T ? 0 : 255;
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

unsigned grid_for(long units, int threads, long cap) {
    long g = (units + threads - 1) / threads;
    if (g > cap) g = cap;
    return (unsigned)(g < 1 ? 1 : g);
}

// Histogram + selection, then (if out is given) the decision.  A = img is
// 16-byte aligned; the vector form of the decision also needs out aligned.
template <int C, bool A>
int launch_pair(const uint8_t *img, uint8_t *out, long npx, uint32_t *ws, uint32_t *copy, int cus,
                bool aligned_out, hipStream_t st) {
    const long hist_units = A ? npx / kPx : npx;
    const unsigned rows = grid_for(hist_units, kHistThreads, cus < kMaxRows ? cus : kMaxRows);
    hipLaunchKernelGGL((otsu_hist<C, A>), dim3(rows), dim3(kHistThreads), 0, st, img, npx, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(e);
    hipLaunchKernelGGL(otsu_select, dim3(1), dim3(kSelectThreads), 0, st, ws, (int)rows, copy);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(e);
    if (!out) return BZ_OK;
    if (A && aligned_out)
        hipLaunchKernelGGL((otsu_apply<C, true>), dim3(grid_for(npx / kPx, kApplyThreads, 8L * cus)),
                           dim3(kApplyThreads), 0, st, img, out, npx, (const uint32_t *)ws);
    else
        hipLaunchKernelGGL((otsu_apply<C, false>), dim3(grid_for(npx, kApplyThreads, 8L * cus)),
                           dim3(kApplyThreads), 0, st, img, out, npx, (const uint32_t *)ws);
    e = hipGetLastError();
    return e == hipSuccess ? BZ_OK : fail(e);
}

// Validation and dispatch shared by both entry points: ws is the caller's
// workspace or this library's scratch array, copy an optional second home
// for the histogram, T and k*.
int run_otsu(const uint8_t *img, int H, int W_img, int channels, uint8_t *out, uint32_t *ws,
             uint32_t *copy, hipStream_t st) {
    const int64_t npx = (int64_t)H * W_img;
    const bool a_in = ((uintptr_t)img & 15) == 0;
    const bool a_out = out && ((uintptr_t)out & 15) == 0;
    const int cus = device_cus();
    if (channels == 1)
        return a_in ? launch_pair<1, true>(img, out, npx, ws, copy, cus, a_out, st)
                    : launch_pair<1, false>(img, out, npx, ws, copy, cus, a_out, st);
    return a_in ? launch_pair<3, true>(img, out, npx, ws, copy, cus, a_out, st)
                : launch_pair<3, false>(img, out, npx, ws, copy, cus, a_out, st);
}

int check_image(const uint8_t *img, int H, int W_img, int channels, const uint8_t *out) {
    if (!img) return BZ_ERR_NULL;
    if (H < 1 || W_img < 1) return BZ_ERR_SHAPE;
    if (channels != 1 && channels != 3) return BZ_ERR_CHANNELS;
    const int64_t npx = (int64_t)H * W_img;
    if (npx * channels >= ((int64_t)1 << 31)) return BZ_ERR_SHAPE;
    if (out && overlaps(img, (size_t)(npx * channels), out, (size_t)npx)) return BZ_ERR_ALIAS;
    return BZ_OK;
}

}  // namespace

// Scratch of the allocation-free entry point: the words of one Otsu
// workspace (per-workgroup histogram rows, histogram, T, k*).  Every device
// the library runs on holds its own copy until the process ends.  In host
// code this name is only a stand-in for the symbol: kernels receive the
// device address looked up once per device below, never the name.
static __device__ __align__(256) uint32_t scratch[BZ_OTSU_WS_BYTES / 4];

namespace {

std::once_flag g_scratch_once[kMaxDevices];
uint32_t *g_scratch[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// Device address of this device's scratch (looked up on the first call
// made while that device is current).
int scratch_address(uint32_t **p) {
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(e);
    if (dev < 0 || dev >= kMaxDevices) return fail(hipErrorInvalidDevice);
    std::call_once(g_scratch_once[dev], [dev] {
        void *ptr = nullptr;
        const hipError_t r = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_err[dev] = r;
        g_scratch[dev] = r == hipSuccess ? static_cast<uint32_t *>(ptr) : nullptr;
    });
    if (g_scratch_err[dev] != hipSuccess) return fail(g_scratch_err[dev]);
    if (!g_scratch[dev]) return fail(hipErrorInvalidSymbol);
    *p = g_scratch[dev];
    return BZ_OK;
}

}  // namespace

extern "C" {

size_t binarize_otsu_workspace_size(void) { return BZ_OTSU_WS_BYTES; }

int binarize_otsu(const uint8_t *img, int H, int W_img, int channels, uint8_t *out, uint32_t *ws,
                  size_t ws_bytes, void *stream) {
    if (!img) return BZ_ERR_NULL;
    if (!ws || ws_bytes < BZ_OTSU_WS_BYTES || ((uintptr_t)ws & 15)) return BZ_ERR_WORKSPACE;
    int rc = check_image(img, H, W_img, channels, out);
    if (rc) return rc;
    const int64_t npx = (int64_t)H * W_img;
    if (overlaps(ws, BZ_OTSU_WS_BYTES, img, (size_t)(npx * channels))) return BZ_ERR_ALIAS;
    if (out && overlaps(ws, BZ_OTSU_WS_BYTES, out, (size_t)npx)) return BZ_ERR_ALIAS;
    return run_otsu(img, H, W_img, channels, out, ws, nullptr, (hipStream_t)stream);
}

int binarize_otsu_noalloc(const uint8_t *img, int H, int W_img, int channels, uint8_t *out,
                          uint32_t *result, void *stream) {
    int rc = check_image(img, H, W_img, channels, out);
    if (rc) return rc;
    if (result && ((uintptr_t)result & 3)) return BZ_ERR_WORKSPACE;
    const int64_t npx = (int64_t)H * W_img;
    const size_t rbytes = 4 * (BZ_OTSU_WS_KSTAR + 1);
    if (result && overlaps(result, rbytes, img, (size_t)(npx * channels))) return BZ_ERR_ALIAS;
    if (result && out && overlaps(result, rbytes, out, (size_t)npx)) return BZ_ERR_ALIAS;
    uint32_t *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    return run_otsu(img, H, W_img, channels, out, ws, result, (hipStream_t)stream);
}

}  // extern "C"
