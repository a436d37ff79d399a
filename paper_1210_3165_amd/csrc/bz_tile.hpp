// bz_tile.hpp -- gfx950 device code of the exact Sauvola / Niblack tile kernel.
//
// One workgroup (256 threads, 4 wave64s) produces a tile of TW output columns
// by tile_h output rows of one page.  The window statistics of the paper's
// Sec. 2 (mean and deviation over the full W x W window S) come from exact
// integer window sums of f and f^2, built separably inside the tile:
//
//   ring    LDS ring of gray rows (Sec. 1 Eq. 1 applied while staging), one
//           row per image row, at least win + 8 rows deep, tile plus halo
//           wide.  Each
//           input byte is read from HBM once per tile; the rows of the next
//           step are loaded into registers while the current step computes.
//   V pass  one thread per two LDS columns slides the vertical window down the
//           tile: V(y) = V(y-1) + f(y+hi) - f(y-lo-1) for V1 = sum f and
//           V2 = sum f^2 (f_in^2 - f_out^2 formed as (f_in - f_out)(f_in + f_out)).
//           Each V row is stored twice, shifted so that output column x finds
//           the column entering its window (Va[x]) and the one leaving it
//           (Vb[x]) at the same index.
//   H pass  32 threads per output row, 8 (or 4) consecutive outputs each:
//           S(x) = S(x-1) + Va[x] - Vb[x], i.e. a per-thread prefix of the
//           differences, a DPP scan across the 32 threads, and the window sum
//           left of the tile as the starting value.
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

// Difference and sum of byte B of two words, each one VALU instruction with
// byte-select operands (plain arithmetic instructions, no memory access).
#define BZ_SDWA_BYTE_OP(NAME, OP)                                                                          \
    template <int B>                                                                                       \
    __device__ __forceinline__ int NAME(uint32_t x, uint32_t y) {                                          \
        static_assert(B >= 0 && B <= 3, "byte index");                                                     \
        int d;                                                                                             \
        if (B == 0)                                                                                        \
            asm(OP " %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_0 src1_sel:BYTE_0"       \
                : "=v"(d) : "v"(x), "v"(y));                                                               \
        else if (B == 1)                                                                                   \
            asm(OP " %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_1 src1_sel:BYTE_1"       \
                : "=v"(d) : "v"(x), "v"(y));                                                               \
        else if (B == 2)                                                                                   \
            asm(OP " %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_2 src1_sel:BYTE_2"       \
                : "=v"(d) : "v"(x), "v"(y));                                                               \
        else                                                                                               \
            asm(OP " %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_3 src1_sel:BYTE_3"       \
                : "=v"(d) : "v"(x), "v"(y));                                                               \
        return d;                                                                                          \
    }
BZ_SDWA_BYTE_OP(byte_sub, "v_sub_u32_sdwa")
BZ_SDWA_BYTE_OP(byte_add, "v_add_u32_sdwa")
#undef BZ_SDWA_BYTE_OP


// Output byte b of w (b a constant after unrolling) becomes 0x00 on lanes
// where `dark` holds and 0xff elsewhere; the other bytes of w are kept.  One
// VALU instruction: a byte-select conditional move on the lane mask.
#define BZ_PUT_BYTE(BSEL)                                                                               \
    asm("s_mov_b64 vcc, %3\n\tv_cndmask_b32_sdwa %0, %1, %2, vcc dst_sel:" BSEL                            \
        " dst_unused:UNUSED_PRESERVE src0_sel:DWORD src1_sel:DWORD"                                        \
        : "+v"(w)                                                                                          \
        : "v"(ff), "v"(zero), "s"(m)                                                                       \
        : "vcc")
__device__ __forceinline__ void put_out_byte(uint32_t &w, int b, bool dark, uint32_t ff, uint32_t zero) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(dark);
    if (b == 0) BZ_PUT_BYTE("BYTE_0");
    else if (b == 1) BZ_PUT_BYTE("BYTE_1");
    else if (b == 2) BZ_PUT_BYTE("BYTE_2");
    else BZ_PUT_BYTE("BYTE_3");
}
#undef BZ_PUT_BYTE

// LDS-typed views, so that offsets into the tile's LDS stay 32-bit (plain
// vector types: the HIP vector classes have no address-space-qualified
// assignment).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(3))) u32x2 lds_v2;
typedef __attribute__((address_space(3))) u32x4 lds_v4;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(1))) uint8_t glb_u8;

// A pointer whose value is the same on every lane, kept in scalar registers:
// reading it through readfirstlane stops the compiler from folding
// per-thread offsets into it (which would turn a scalar base plus a 32-bit
// offset back into a 64-bit per-thread address).
__device__ __forceinline__ glb_u8 *uniform_global(uint8_t *p) {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (glb_u8 *)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

// Unaligned views (alignment 1) for the wide accesses of the tiles
// of pages whose rows are not 16-byte aligned: gfx950 loads and stores them
// whole (global memory runs in unaligned access mode under ROCm).
typedef unsigned int u32x4_a1 __attribute__((ext_vector_type(4), aligned(1)));
typedef unsigned int u32x2_a1 __attribute__((ext_vector_type(2), aligned(1)));
typedef __attribute__((address_space(1))) u32x2_a1 glb_u32x2_a1;

// How a tile stages its input rows and stores its outputs:
//   kAligned  rows 16-byte aligned, a multiple of 16 pixels wide, pitches
//             below 2^28 (every tile of such a page): 16-byte loads and
//             8-byte stores from a uniform row address plus 32-bit offsets;
//   kWide     other pages at least 16 pixels wide with pitches below 2^28
//             (every tile): unaligned 16-byte loads and 8-byte stores from a
//             uniform row address plus 32-bit offsets.  Chunks start on
//             multiples of 16 columns, so only the chunk that holds a row's
//             last column can reach past it: that chunk loads the row's last
//             16 pixels and moves them down in registers (shift_out), and
//             outputs past the row end take byte stores;
//   kEdge     pages narrower than 16 pixels or with larger pitches: word
//             loads clamped into the row, byte masks, byte stores at the
//             ragged end of a row.
// All three give identical bytes.
enum { kEdge = 0, kWide = 1, kAligned = 2 };

// ---------------------------------------------------------------- staging
//
// A staging job is 16 consecutive pixels of one image row.  Its raw bytes are
// fetched into registers (RawChunk) one step ahead of use and reduced to 16
// gray levels when written into the ring.

template <int C>
struct RawChunk {
    static constexpr int NW = C == 1 ? 5 : 13;  // aligned words covering 16*C bytes + 1
    uint32_t w[NW];
    uint32_t sh;  // byte offset of the chunk's first byte in w[0]
};

// Issue the loads for the raw bytes of image columns [xs, xs + 16) of one row.
// Nothing reads the loaded registers until chunk_gray, one step later, so the
// loads stay in flight while the tile computes.  Word i nominally sits at
// (first byte & ~3) + 4 i; on tiles that reach past the image's left or right
// edge (clamp == true) every word address is clamped into the words that hold
// at least one byte of this row, so no access leaves the caller's buffer.
// Bytes that belong to columns outside [0, W) are discarded by chunk_gray.
template <int C, bool AL>
__device__ __forceinline__ void fetch_chunk(RawChunk<C> &k, const uint8_t *__restrict__ rowp, int xs, int W,
                                            bool clamp) {
    if (AL) {  // 16-byte aligned chunk, wholly inside the row: C vector loads
        const uint4 *q = reinterpret_cast<const uint4 *>(rowp + C * xs);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const uint4 v = q[i];
            k.w[4 * i] = v.x;
            k.w[4 * i + 1] = v.y;
            k.w[4 * i + 2] = v.z;
            k.w[4 * i + 3] = v.w;
        }
        k.sh = 0;
        return;
    }
    // word offsets relative to the row pointer (the row's bytes are
    // [0, C W)), so every address derives from the image pointer and the
    // loads stay global
    const int r = (int)((uintptr_t)rowp & 3);  // the row's first byte within its word
    const int o = C * xs;                      // the chunk's first byte
    k.sh = (uint32_t)((r + o) & 3);
    const int q = o - (int)k.sh;               // word-aligned (relative to the row's words)
    if (clamp) {
        const int first = -r;                            // word holding byte 0
        const int last = ((r + C * W - 1) & ~3) - r;     // word holding byte C W - 1
#pragma unroll
        for (int i = 0; i < RawChunk<C>::NW; ++i) {
            const int qi = min(max(q + 4 * i, first), last);
            k.w[i] = *(const uint32_t *)(rowp + qi);
        }
    } else {
#pragma unroll
        for (int i = 0; i < RawChunk<C>::NW; ++i) k.w[i] = *(const uint32_t *)(rowp + q + 4 * i);
    }
}

// 16 gray levels from a fetched chunk; columns outside [0, W) become 0.
template <int C, bool AL>
__device__ __forceinline__ uint4 chunk_gray(const RawChunk<C> &k, int xs, int W, bool clamp) {
    constexpr int NB = C == 1 ? 4 : 12;
    uint32_t b[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) b[i] = AL ? k.w[i] : align_bytes(k.w[i + 1], k.w[i], k.sh);
    uint32_t o[4];
    if (C == 1) {
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = b[i];
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = 0u;
#pragma unroll
        for (int px = 0; px < 16; ++px)
            o[px >> 2] |= gray_of(byte_at(b, 3 * px), byte_at(b, 3 * px + 1), byte_at(b, 3 * px + 2))
                          << (8 * (px & 3));
    }
    if (!AL && clamp) {
#pragma unroll
        for (int px = 0; px < 16; ++px) {
            const int c = xs + px;
            if (c < 0 || c >= W) o[px >> 2] &= ~(0xffu << (8 * (px & 3)));
        }
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
}

// Gray levels g of columns [W - 16, W) moved down so that byte j holds column
// xs + j, for the chunk [xs, xs + 16) that holds column W - 1 (cut = xs + 16 - W
// in 1..15): byte j takes byte j + cut, and the bytes past the row become 0.
__device__ __forceinline__ u32x4 shift_out(u32x4 g, int cut) {
    const uint64_t lo = (uint64_t)g.x | ((uint64_t)g.y << 32), hi = (uint64_t)g.z | ((uint64_t)g.w << 32);
    const uint32_t sb = 8u * (uint32_t)cut;  // 8..120 bits
    const uint64_t nlo = sb < 64 ? (lo >> sb) | (hi << (64 - sb)) : hi >> (sb - 64);
    const uint64_t nhi = sb < 64 ? hi >> sb : 0;
    return u32x4{(uint32_t)nlo, (uint32_t)(nlo >> 32), (uint32_t)nhi, (uint32_t)(nhi >> 32)};
}

// The job of this thread for a block of up to RB rows: row i = job / nq of
// the block, chunk q = job % nq (nq = rp / 16 chunks per row).  RB * rp / 16
// <= 256 gives at most one job per thread.  Rows outside the image load a clamped
// row (always a valid address) and store zeros.  INT: a page whose rows are
// 16-byte aligned and a multiple of 16 pixels wide, so every chunk lies wholly
// inside or wholly outside the image: chunks are loaded whole with one 16-byte
// load, and chunks outside load a clamped chunk and store zeros.
template <int C, int BODY>
struct Stager {
    static constexpr bool INT = BODY == kAligned;
    static constexpr bool WIDE = BODY == kWide;
    RawChunk<C> k;
    int job_row, job_q;  // job_row >= kRowsPerStep: this thread has no job
    bool in_image;
    // INT and WIDE bodies: the job's byte offsets from the first row of its
    // block and from its row (32-bit offsets: pitches are below 2^28 there),
    // and whether its chunk starts inside the image's columns; cols_in: every
    // chunk of the tile lies wholly inside; cut (WIDE): columns of the chunk
    // past the row's end when it holds the row's last column, else 0 (the
    // chunk then loads the row's last 16 pixels instead).
    uint32_t voff, xoff;
    bool col_in, cols_in;
    int cut;
    bool zero_free;  // the last fetch staged rows and chunks all inside the image

    __device__ __forceinline__ void init(const PageArgs &a, int xr0) {
        const int nq = a.rp >> 4;
        job_row = (int)threadIdx.x / nq;
        job_q = (int)threadIdx.x - job_row * nq;
        in_image = true;
        zero_free = false;
        if (INT || WIDE) {
            const int xs = xr0 + 16 * job_q;
            col_in = xs >= 0 && xs < a.W;
            cols_in = xr0 >= 0 && xr0 + a.rp <= a.W;
            cut = WIDE && col_in && xs + 16 > a.W ? xs + 16 - a.W : 0;
            xoff = (uint32_t)(C * min(max(xs, 0), a.W - 16));
            voff = (uint32_t)job_row * (uint32_t)a.pitch_in + xoff;
        }
    }

    __device__ __forceinline__ void fetch(const PageArgs &a, int row0, int nrows, int xr0, bool clamp) {
        if (INT || WIDE) {
            // Every job loads from one uniform row address, that of the
            // block's first row clamped into the image, plus a 32-bit offset:
            // fixed when every row of the block lies inside the image (the
            // usual case), else from the job's own clamped row.  Chunks
            // outside the columns load a clamped chunk (stored as zeros).
            const bool inside = row0 >= 0 && row0 + nrows <= a.H;  // uniform
            const int rb = min(max(row0, 0), a.H - 1);
            uint32_t off = voff;
            in_image = col_in;
            if (!inside) {
                const int row = row0 + job_row;
                const int rc = min(max(row, 0), a.H - 1);
                off = (uint32_t)(rc - rb) * (uint32_t)a.pitch_in + xoff;
                in_image = col_in && row >= 0 && row < a.H;
            }
            zero_free = inside && cols_in;
            if (job_row < nrows) {
                const uint8_t *blk = a.img + (size_t)rb * (size_t)a.pitch_in;  // uniform
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const u32x4 v = WIDE ? (u32x4)reinterpret_cast<const u32x4_a1 *>(blk + off)[i]
                                         : reinterpret_cast<const u32x4 *>(blk + off)[i];
                    k.w[4 * i] = v.x;
                    k.w[4 * i + 1] = v.y;
                    k.w[4 * i + 2] = v.z;
                    k.w[4 * i + 3] = v.w;
                }
                k.sh = 0;
            }
            return;
        }
        zero_free = false;
        if (job_row < nrows) {
            const int row = row0 + job_row;
            int xs = xr0 + 16 * job_q;
            in_image = row >= 0 && row < a.H;
            if (INT) {
                in_image = in_image && xs >= 0 && xs < a.W;
                xs = min(max(xs, 0), a.W - 16);
            }
            const int rc = min(max(row, 0), a.H - 1);
            fetch_chunk<C, INT>(k, a.img + (size_t)rc * (size_t)a.pitch_in, xs, a.W, clamp);
        }
    }

    // Store into rows `rows`, `rows` + rp, ... (no ring wrap).
    // Store the fetched chunk as 16 gray levels at `p`, zero outside the
    // image.  Chunks outside are rare (edge tiles, rows beyond the image):
    // they are overwritten with zeros (or, the chunk that holds a row's last
    // column, with its shifted levels) behind the uniform zero_free test,
    // which the empty volatile asm keeps a branch (as selects, the masking
    // would run on every step).
    template <class P>
    __device__ __forceinline__ void put(const PageArgs &a, P *p, int xr0, bool clamp) const {
        const uint4 v = chunk_gray<C, BODY != kEdge>(k, xr0 + 16 * job_q, a.W, clamp);
        const u32x4 g = u32x4{v.x, v.y, v.z, v.w};
        *p = g;
        if (!zero_free) {
            asm volatile("");
            if (!in_image)
                *p = u32x4{0u, 0u, 0u, 0u};
            else if (WIDE && cut)
                *p = shift_out(g, cut);
        }
    }

    __device__ __forceinline__ void store_rows(const PageArgs &a, uint8_t *rows, int nrows, int xr0,
                                               bool clamp) const {
        if (job_row >= nrows) return;
        put(a, (u32x4 *)(rows + job_row * a.rp + 16 * job_q), xr0, clamp);
    }

    __device__ __forceinline__ void store(const PageArgs &a, uint8_t *ring, int slot0, int nrows, int xr0,
                                          bool clamp) const {
        if (job_row >= nrows) return;
        int sl = slot0 + job_row;
        if (sl >= a.depth) sl -= a.depth;
        put(a, (u32x4 *)(ring + sl * a.rp + 16 * job_q), xr0, clamp);
    }

    // Store at byte `off` of the tile's LDS (the job's own slot and chunk).
    __device__ __forceinline__ void store_at(const PageArgs &a, lds_u8 *lds, uint32_t off, int nrows, int xr0,
                                             bool clamp) const {
        if (job_row >= nrows) return;
        put(a, (lds_v4 *)(lds + off), xr0, clamp);
    }
};

// ---------------------------------------------------------------- scans

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp_src(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, true);
}

// Inclusive prefix sum within each 32-lane half of the wave: row_shr 1, 2,
// 4, 8 inside each 16-lane DPP row, then row_bcast:15 carries the total of
// rows 0 and 2 into rows 1 and 3.  Unsigned wrap-around is harmless: every
// final window sum is below 2^32.
__device__ __forceinline__ uint32_t scan32(uint32_t v) {
    v += dpp_src<0x111>(v);
    v += dpp_src<0x112>(v);
    v += dpp_src<0x114>(v);
    v += dpp_src<0x118>(v);
    v += dpp_src<0x142, 0xa>(v);
    return v;
}

// Total of the 32-lane half this lane belongs to, given its inclusive scan:
// every lane reads the last lane of its half (ds_swizzle in bit mode with
// or-mask 31, which works within 32-lane groups; no LDS memory is touched).
__device__ __forceinline__ uint32_t half_total(uint32_t incl) {
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)incl, 0x1f << 5);
}

// ---------------------------------------------------------------- decision
//
// Eq. 3 decides f < t.  With the exact integer window sums S1, S2 and count n,
// m = S1 / n and s = sqrt(D) / n where D = n S2 - S1^2 is formed exactly in
// fp64 (every term is an integer below 2^53); sqrt(D) is taken in fp32.
//
//   Sauvola (Eq. 4), t = m (c1 + c2 s) with c1 = 1 - k, c2 = k / R, both
//   sides scaled by n (fp64 after the square root):
//     steps whose windows are all whole (n = win^2, constants per page):
//       f < t  <=>  f < S1 (c1/n + (c2/n^2) sqrt(D))
//     clipped windows (n per pixel, no division):
//       f < t  <=>  (n f) n < S1 (n c1 + c2 sqrt(D))
//   Niblack, t = m + k s (fp32; n f - S1 is an exact integer below 2^24):
//       f < t  <=>  n f - S1 < k sqrt(D)
//
// The only sizeable rounding is that of sqrt(D) in fp32 (relative 1.35e-7
// at most), which moves the Sauvola threshold by at most
// m |k| s / R * 1.35e-7 and the Niblack threshold by |k| s * 1.9e-7 with the
// fp32 product: below 4.5e-5 and 2.5e-5 in the accepted range |k| <= 1,
// R >= 64 (Sauvola).  Niblack decides ties exactly: a window of constant
// gray level (D = 0) gives f = t and the output 255.  A Sauvola call with
// k = 0 is the same rule (t = m) and is routed to the Niblack form by the
// host.

// Whole-window Sauvola constants of a page: n = win^2, c1 / n, c2 / n^2.
struct WholeWindow {
    double nd, c1n, c2n2;
};

__device__ __forceinline__ WholeWindow whole_window(const PageArgs &a, uint32_t n) {
    WholeWindow q;
    q.nd = (double)n;
    q.c1n = a.c1n;
    q.c2n2 = a.c2n2;
    return q;
}

// sqrt(D) in fp32 with D = n S2 - S1^2 exact in fp64; s1d receives S1.
__device__ __forceinline__ float exact_sqrt_d(double nd, uint32_t S1, uint32_t S2, double &s1d) {
    s1d = (double)S1;
    const double D = __builtin_fma(nd, (double)S2, -(s1d * s1d));
    return __builtin_amdgcn_sqrtf((float)D);
}

// t itself, fp64 rounded to fp32 (verification planes only).
template <int RULE>
__device__ __forceinline__ float threshold_value(const PageArgs &a, uint32_t S1, uint32_t n, float sq) {
    const double nd = (double)n;
    const double m = (double)S1 / nd;
    const double s = (double)sq / nd;
    return (float)(RULE == 0 ? m * __builtin_fma(a.c2, s, a.c1) : __builtin_fma((double)a.k, s, m));
}

// sqrt(D) in fp32 for a whole window (n = win^2), with S2 = b2 + e2 given
// as nb2 = n b2 (an exact fp64 product, shared by a thread's outputs) and
// e2 = S2 - b2 (|e2| < 2^27): D = n e2 + (n b2 - S1^2), each step exact (all
// terms are integers below 2^49), so D equals n S2 - S1^2 bit for bit.
__device__ __forceinline__ float exact_sqrt_d_whole(double nd, double nb2, uint32_t S1, int32_t e2, double &s1d) {
    s1d = (double)S1;
    const double D = __builtin_fma(nd, (double)e2, __builtin_fma(-s1d, s1d, nb2));
    return __builtin_amdgcn_sqrtf((float)D);
}

// Whole-window Sauvola (per-page constants): true if f < t (output 0).
__device__ __forceinline__ bool dark_sauvola_full(const WholeWindow &q, uint32_t f, uint32_t S1, uint32_t S2,
                                                  float &sq) {
    double s1d;
    sq = exact_sqrt_d(q.nd, S1, S2, s1d);
    return (double)f < s1d * __builtin_fma(q.c2n2, (double)sq, q.c1n);
}

// The same with S2 given as for exact_sqrt_d_whole (identical D and result).
__device__ __forceinline__ bool dark_sauvola_full(const WholeWindow &q, uint32_t f, uint32_t S1, double nb2,
                                                  int32_t e2, float &sq) {
    double s1d;
    sq = exact_sqrt_d_whole(q.nd, nb2, S1, e2, s1d);
    return (double)f < s1d * __builtin_fma(q.c2n2, (double)sq, q.c1n);
}

// Sauvola, any n.
__device__ __forceinline__ bool dark_sauvola(const PageArgs &a, uint32_t f, uint32_t S1, uint32_t S2,
                                             uint32_t n, float &sq) {
    const double nd = (double)n;
    double s1d;
    sq = exact_sqrt_d(nd, S1, S2, s1d);
    return (double)__umul24(n, f) * nd < s1d * __builtin_fma(a.c2, (double)sq, a.c1 * nd);
}

// Niblack, any n.
__device__ __forceinline__ bool dark_niblack(const PageArgs &a, uint32_t f, uint32_t S1, uint32_t S2,
                                            uint32_t n, float &sq) {
    double s1d;
    sq = exact_sqrt_d((double)n, S1, S2, s1d);
    return (float)((int)__umul24(n, f) - (int)S1) < a.k * sq;
}

// Whole-window Niblack (n = win^2), S2 given as for exact_sqrt_d_whole.
__device__ __forceinline__ bool dark_niblack_full(const PageArgs &a, const WholeWindow &q, uint32_t n, uint32_t f,
                                                 uint32_t S1, double nb2, int32_t e2, float &sq) {
    double s1d;
    sq = exact_sqrt_d_whole(q.nd, nb2, S1, e2, s1d);
    return (float)((int)__umul24(n, f) - (int)S1) < a.k * sq;
}

// ---------------------------------------------------------------- output

// Output bytes are written once and never read back by the kernel: their
// stores carry the non-temporal hint, so the caches treat them as streaming
// data rather than keeping them resident next to the input rows that
// neighbouring tiles read again.
__device__ __forceinline__ void store_nt8(uint8_t *p, uint32_t lo, uint32_t hi) {
    const u32x2 v = {lo, hi};
    __builtin_nontemporal_store(v, (u32x2 *)p);
}

__device__ __forceinline__ void store_nt4(uint8_t *p, uint32_t w) {
    __builtin_nontemporal_store(w, (uint32_t *)p);
}

__device__ __forceinline__ void store_nt8(glb_u8 *p, uint32_t lo, uint32_t hi) {
    const u32x2 v = {lo, hi};
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) u32x2 *)p);
}

__device__ __forceinline__ void store_nt4(glb_u8 *p, uint32_t w) {
    __builtin_nontemporal_store(w, (__attribute__((address_space(1))) uint32_t *)p);
}

// The same at any byte address (the wide body of unaligned pages).
typedef uint32_t u32_a1 __attribute__((aligned(1)));
__device__ __forceinline__ void store_nt8_a1(glb_u8 *p, uint32_t lo, uint32_t hi) {
    const u32x2_a1 v = {lo, hi};
    __builtin_nontemporal_store(v, (glb_u32x2_a1 *)p);
}

__device__ __forceinline__ void store_nt4_a1(glb_u8 *p, uint32_t w) {
    __builtin_nontemporal_store(w, (__attribute__((address_space(1))) u32_a1 *)p);
}

// Store OPT output bytes (packed little-endian in w) at columns [xs, xs+OPT)
// of an output row, skipping columns >= W.
template <int OPT>
__device__ __forceinline__ void store_row(uint8_t *rowp, int xs, int W, const uint32_t (&w)[OPT / 4]) {
    if (xs + OPT <= W) {  // one store at any byte address
        glb_u8 *p = (glb_u8 *)(rowp + xs);
        if (OPT == 8)
            store_nt8_a1(p, w[0], w[OPT / 4 - 1]);
        else
            store_nt4_a1(p, w[0]);
        return;
    }
#pragma unroll
    for (int j = 0; j < OPT; ++j)  // the ragged end of the row
        if (xs + j < W) rowp[xs + j] = (uint8_t)(w[j >> 2] >> (8 * (j & 3)));
}

__device__ __forceinline__ int floor16(int x) { return x & ~15; }  // two's complement: rounds toward -inf

// Workgroups are dispatched round-robin over the 8 XCDs; give every XCD a
// contiguous run of tiles so neighbouring tiles (which share halo columns and
// rows) meet in the same L2.  Inside a run of L tiles, workgroup i takes tile
// (i % G) * R + i / G (G groups of R = ceil(L / G) tiles, the last groups one
// tile shorter): a bijection of the run.  Workgroups placed on the same CU
// (i a multiple of the XCD's CU count apart) then take tiles G apart within a
// group instead of tiles a CU count apart, which on power-of-two page widths
// stacks them in one tile column; the slower edge-column tiles are thereby
// spread over the CUs instead of loading a few of them four times.
template <int G = 8>
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    const int L = q + (x < r ? 1 : 0);
    const int R = (L + G - 1) / G, full = L - (R - 1) * G;  // groups with R tiles
    const int g = i % G, k = i / G;
    const int j = g < full ? g * R + k : full * R + (g - full) * (R - 1) + k;
    return x * q + (x < r ? x : r) + j;
}

template <int OPT>
__device__ __forceinline__ void load_u16(const uint16_t *p, uint32_t (&v)[OPT]) {
    if (OPT == 8) {
        const uint4 q = *(const uint4 *)p;
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[2 * i] = w[i] & 0xffffu;
            v[2 * i + 1] = w[i] >> 16;
        }
    } else {
        const uint2 q = *(const uint2 *)p;
        v[0] = q.x & 0xffffu;
        v[1] = q.x >> 16;
        v[2] = q.y & 0xffffu;
        v[3] = q.y >> 16;
    }
}

// Entries OPT*h .. OPT*h+OPT-1 of a V2 row laid out by v2_pos<OPT == 8>
// (with OPT == 8 the second quad holds its entries pairwise swapped).
template <int OPT>
__device__ __forceinline__ void load_v2(const uint32_t *row, int width, int h, uint32_t (&v)[OPT]) {
#pragma unroll
    for (int i = 0; i < OPT / 4; ++i) {
        const int x = OPT * h + 4 * i;
        const uint4 q = *(const uint4 *)(row + v2_quad(x, width));
        const bool sw = OPT == 8 && i == 1;
        v[4 * i] = sw ? q.y : q.x;
        v[4 * i + 1] = sw ? q.x : q.y;
        v[4 * i + 2] = sw ? q.w : q.z;
        v[4 * i + 3] = sw ? q.z : q.w;
    }
}

template <int TW, int C, int RULE, bool STATS, int BODY, bool BLK>
__device__ __forceinline__ void process_tile(const PageArgs &a, int tile, uint8_t *smem) {
    constexpr int RB = kRowsPerStep;
    constexpr int TPR = kThreadsPerRow;
    constexpr int OPT = TW / TPR;  // outputs per thread per row (4 or 8)
    static_assert(OPT == 4 || OPT == 8, "tile width must be 128 or 256");

    const int tid = threadIdx.x;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int X0 = tx * TW, Y0 = ty * a.tile_h;
    const int Yend = min(Y0 + a.tile_h, a.H);
    const int lo = a.lo, hi = a.hi, win = a.win;
    const int xr0 = floor16(X0 - lo - 1);  // image column of LDS column 0
    const int off0 = X0 - lo - xr0;        // LDS column of the first window column, 1..16
    const int rp = a.rp, depth = a.depth;
    const int vbw = vb_width(TW, win);
    constexpr int VAP = TW + kTrash;                        // va_pitch
    const int VBP = TW == 256 ? 256 + kTrash : vbw + kTrash;  // vb_pitch (constant for 256 columns)
    uint8_t *ring = smem;
    uint16_t *Va1 = (uint16_t *)(smem + rows_bytes(depth, TW, win));
    // blocks layout (gray pages with wide windows): the step's entering,
    // leaving and centre rows; otherwise the ring of depth rows
    constexpr bool blocks = C == 1 && BLK;
    uint8_t *const blkE = smem, *const blkL = smem + RB * rp, *const blkC = smem + 2 * RB * rp;
    uint16_t *Vb1 = Va1 + RB * VAP;
    uint32_t *Va2 = (uint32_t *)(Vb1 + RB * VBP);
    uint32_t *Vb2 = Va2 + RB * VAP;
    const int base = Y0 - lo - 1;  // image row held by ring slot 0

    // Clamp loads and mask bytes in the kEdge body: some of columns [xr0,
    // xr0 + rp), or the one extra word a chunk may read past its last byte,
    // may lie outside the row.
    constexpr bool INT = BODY == kAligned;
    constexpr bool clamp = BODY == kEdge;

    // Wave priorities.  The waves of a CU come from several workgroups, each
    // of which alternates a short phase that every other wave of it waits
    // for at a barrier (start-up, vertical pass, the reads that open the
    // horizontal pass, the staging and stores that close a step) with a long
    // arithmetic phase (the decisions).  Issuing the waited-on phases first
    // (s_setprio 3 for the start-up and vertical pass, 2 for the reads that
    // open the horizontal pass, 1 for the step's end) and the arithmetic at
    // priority 0 lets the arithmetic of some workgroups fill the VALU while
    // others cross their barriers, instead of all of them queueing behind
    // one another's decisions.
    __builtin_amdgcn_s_setprio(3);

    // ---- vertical-pass ownership: LDS columns c0 = 2 tid and c0 + 1
    const int c0 = 2 * tid;
    const bool vcol = c0 < rp;
    uint32_t v1[2] = {0u, 0u}, v2[2] = {0u, 0u};
    // Column sums of nr rows, rp apart.  Four rows at a time: the bytes of
    // each column are gathered into one word, whose byte sum (v_sad_u8
    // against zero) and dot product with itself (v_dot4_u32_u8) add four
    // rows' f and f^2 in one instruction each.
    auto add_rows = [&](const uint8_t *rows, int nr) {
        if (vcol) {
            int i = 0;
#pragma unroll 2
            for (; i + 4 <= nr; i += 4) {
                const uint32_t w0 = *(const uint16_t *)(rows + i * rp + c0);
                const uint32_t w1 = *(const uint16_t *)(rows + (i + 1) * rp + c0);
                const uint32_t w2 = *(const uint16_t *)(rows + (i + 2) * rp + c0);
                const uint32_t w3 = *(const uint16_t *)(rows + (i + 3) * rp + c0);
                const uint32_t t01 = w0 | (w1 << 16), t23 = w2 | (w3 << 16);
                const uint32_t col0 = __builtin_amdgcn_perm(t23, t01, 0x06040200u);  // bytes 0 of w0..w3
                const uint32_t col1 = __builtin_amdgcn_perm(t23, t01, 0x07050301u);  // bytes 1 of w0..w3
                v1[0] = __builtin_amdgcn_sad_u8(col0, 0u, v1[0]);
                v2[0] = __builtin_amdgcn_udot4(col0, col0, v2[0], false);
                v1[1] = __builtin_amdgcn_sad_u8(col1, 0u, v1[1]);
                v2[1] = __builtin_amdgcn_udot4(col1, col1, v2[1], false);
            }
            for (; i < nr; ++i) {
                const uint32_t w = *(const uint16_t *)(rows + i * rp + c0);
                const uint32_t f0 = w & 0xffu, f1 = w >> 8;
                v1[0] += f0;
                v2[0] += f0 * f0;
                v1[1] += f1;
                v2[1] += f1 * f1;
            }
        }
    };

    // Rows of the next step, in flight while this one computes: the
    // entering rows (and in the blocks layout the leaving and centre rows
    // too).
    Stager<C, BODY> pre, pre_l, pre_c;
    pre.init(a, xr0);
    if (blocks) {
        pre_l.init(a, xr0);
        pre_c.init(a, xr0);
        // Rounds of kStartRows rows staged and summed, in the two halves of
        // a 2 kStartRows-row area at the start of the tile's LDS in turn: a
        // round stores into the half that was summed two rounds before,
        // which every wave has finished with once it has passed the previous
        // round's barrier, so one barrier per round suffices.  The next
        // round's loads are issued as soon as this round's rows are stored,
        // so they are in flight across the barrier and the summing.
        constexpr int NS = kStartRows / RB;
        Stager<C, BODY> st[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) st[u].init(a, xr0);
        // loads of the rounds starting at r (with the first step's blocks
        // alongside the last round's)
        auto fetch_round = [&](int r) {
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                const int rr = r + u * RB;
                if (rr < win) st[u].fetch(a, base + rr, min(RB, win - rr), xr0, clamp);
            }
            if (r + kStartRows >= win) {
                pre.fetch(a, Y0 + hi, RB, xr0, clamp);
                pre_l.fetch(a, base, RB, xr0, clamp);
                pre_c.fetch(a, Y0, RB, xr0, clamp);
            }
        };
        fetch_round(0);
        for (int r0 = 0, half = 0; r0 < win; r0 += kStartRows, half ^= 1) {
            uint8_t *const rows = smem + half * kStartRows * rp;
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                const int rr = r0 + u * RB;
                if (rr < win) st[u].store_rows(a, rows + u * RB * rp, min(RB, win - rr), xr0, clamp);
            }
            if (r0 + kStartRows < win) fetch_round(r0 + kStartRows);
            __syncthreads();
            add_rows(rows, min(kStartRows, win - r0));
        }
        __syncthreads();  // start-up rows summed: the blocks may be written
        pre.store_rows(a, blkE, RB, xr0, clamp);
        pre_l.store_rows(a, blkL, RB, xr0, clamp);
        if (Y0 + RB < Yend) {
            pre.fetch(a, Y0 + RB + hi, RB, xr0, clamp);
            pre_l.fetch(a, Y0 + RB - lo - 1, RB, xr0, clamp);
        }
        // pre_c holds the first step's centre rows: stored during its vertical pass
    } else {
        // ---- start-up: rows [Y0-lo-1, Y0+hi-1] give V at row Y0-1.  Several
        // blocks of RB rows are fetched before any of them is stored, so their
        // loads are in flight together instead of one latency per block.
        // The rows of the first step are requested together with the last
        // blocks, and go in behind the start-up rows (slots the start-up
        // reads do not touch).
        constexpr int NS = C == 1 ? 4 : 2;  // blocks in flight (registers per block: 5 or 13 words)
        Stager<C, BODY> st[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) st[u].init(a, xr0);
        for (int r0 = 0; r0 < win; r0 += NS * RB) {
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                const int rr = r0 + u * RB;
                if (rr < win) st[u].fetch(a, base + rr, min(RB, win - rr), xr0, clamp);
            }
            if (r0 + NS * RB >= win) pre.fetch(a, Y0 + hi, RB, xr0, clamp);
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                const int rr = r0 + u * RB;
                if (rr < win) st[u].store(a, ring, rr, min(RB, win - rr), xr0, clamp);
            }
        }
        __syncthreads();
        add_rows(ring, win);
        pre.store(a, ring, win, RB, xr0, clamp);
        if (Y0 + RB < Yend) pre.fetch(a, Y0 + RB + hi, RB, xr0, clamp);
    }

    // Va index of column c: c - off0 - win + 1; Vb index: c - off0 + 1.
    // Columns whose V is not needed in Va / Vb write to a trash entry of the
    // same row instead, which keeps the vertical pass free of branches and
    // every store at a fixed offset from its row.
    int pa1[2], pa2[2], pb1[2], pb2[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = c0 + h;
        const int ia = c - off0 - win + 1, ib = c - off0 + 1;
        const bool wa = ia >= 0 && ia < TW;
        const bool wb = ib >= 0 && ib < vbw;
        const int tr = c & (kTrash - 1);
        pa1[h] = wa ? ia : TW + tr;
        pa2[h] = wa ? v2_pos<OPT == 8>(ia, TW) : TW + tr;
        pb1[h] = wb ? ib : vbw + tr;
        pb2[h] = wb ? v2_pos<OPT == 8>(ib, vbw) : vbw + tr;
    }

    const int hr = tid / TPR, hs = tid % TPR;
    // INT and WIDE bodies: this thread's output bytes relative to the step's
    // first output row (pitches are below 2^28 there)
    const uint32_t out_off = (uint32_t)hr * (uint32_t)a.pitch_out + (uint32_t)(X0 + hs * OPT);
    // Steps whose windows all span win rows, in a 256-column block of the
    // page (counted from column 0) whose windows all span win columns, are
    // decided with the per-tile Sauvola constants; every other pixel takes
    // the per-pixel n form.  The two forms round differently, so the choice
    // is made per 256-column block rather than per tile: a 128-column tile
    // lies inside one block, and steps start on multiples of 8 image rows
    // for every tile height, so the output bytes never depend on the tile
    // shape.
    const int XB = X0 & ~255;
    const bool x_inside = XB - lo >= 0 && XB + 255 + hi <= a.W - 1;
    // steps whose windows are all whole: n = win^2, Sauvola constants per tile
    const uint32_t n_full = (uint32_t)__mul24(win, win);
    const WholeWindow q_full = whole_window(a, n_full);

    // Ring layout: slots of the step's first entering row (image row
    // y0 + hi), first leaving row (y0 - lo - 1) and first output row (y0),
    // advanced by RB per step; slot 0 holds image row base = Y0 - lo - 1 and
    // depth > win.
    int s_in = win, s_out = 0;
    const int ring_len = depth * rp;  // bytes of the ring
    lds_u8 *const lds = (lds_u8 *)smem;
    // Per-thread LDS byte offsets, advanced by RB rows per step with one
    // wrap test (a row plus a column below rp: at or past ring_len means
    // the row wrapped): this thread's staging chunk in the slots of the next
    // step's entering rows, and its window centres (in the blocks layout, a
    // fixed row of the centre block).
    auto wrap_row = [&](int r) { return r >= depth ? r - depth : r; };
    uint32_t st_off = (uint32_t)(wrap_row(win + RB + pre.job_row) * rp + 16 * pre.job_q);
    uint32_t ctr_off = (uint32_t)((blocks ? 2 * RB + hr : wrap_row(lo + 1 + hr)) * rp + off0 + lo + hs * OPT);
    auto advance = [&](uint32_t &off) {
        off += (uint32_t)(RB * rp);
        if (off >= (uint32_t)ring_len) off -= (uint32_t)ring_len;
    };
    __syncthreads();

    for (int y0 = Y0; y0 < Yend; y0 += RB) {
        // ---- vertical pass: two LDS columns per thread, RB rows, no branches
        __builtin_amdgcn_s_setprio(3);
        if (blocks) {
            // this step's centre rows go into the centre block, which the
            // previous step's horizontal pass has finished reading
            pre_c.store_rows(a, blkC, RB, xr0, clamp);
            if (y0 + RB < Yend) pre_c.fetch(a, y0 + RB, RB, xr0, clamp);
        }
        if (vcol) {
            uint32_t fn[RB], fo[RB];
            if (blocks) {
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    fn[r] = *(const uint16_t *)(blkE + r * rp + c0);
                    fo[r] = *(const uint16_t *)(blkL + r * rp + c0);
                }
            } else {
                int pe = s_in * rp, px = s_out * rp;  // byte offsets of the entering / leaving rows
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    fn[r] = *(const uint16_t *)(ring + pe + c0);
                    fo[r] = *(const uint16_t *)(ring + px + c0);
                    pe += rp;
                    px += rp;
                    pe = pe == ring_len ? 0 : pe;
                    px = px == ring_len ? 0 : px;
                }
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    // d = f_in - f_out, V2 += d (f_in + f_out)
                    const int d = h == 0 ? byte_sub<0>(fn[r], fo[r]) : byte_sub<1>(fn[r], fo[r]);
                    const int e = h == 0 ? byte_add<0>(fn[r], fo[r]) : byte_add<1>(fn[r], fo[r]);
                    v1[h] += (uint32_t)d;
                    v2[h] += (uint32_t)__mul24(d, e);
                    Va1[r * VAP + pa1[h]] = (uint16_t)v1[h];
                    Va2[r * VAP + pa2[h]] = v2[h];
                    Vb1[r * VBP + pb1[h]] = (uint16_t)v1[h];
                    Vb2[r * VBP + pb2[h]] = v2[h];
                }
            }
        }
        __builtin_amdgcn_s_setprio(2);
        __syncthreads();

        // ---- horizontal pass + threshold: 32 threads per output row.
        // Every group runs (rows past the tile compute on stale LDS data and
        // store nothing) so the cross-lane scans see full 32-lane halves.
        const int y = y0 + hr;
        uint32_t A1[OPT], B1[OPT], A2[OPT], B2[OPT];
        load_u16<OPT>(Va1 + hr * VAP + hs * OPT, A1);
        load_u16<OPT>(Vb1 + hr * VBP + hs * OPT, B1);
        load_v2<OPT>(Va2 + hr * VAP, TW, hs, A2);
        load_v2<OPT>(Vb2 + hr * VBP, vbw, hs, B2);
        // starting value: window sum one column left of the tile (entries
        // 0 .. win-1 of the Vb row).  A uniform, not unrolled loop over
        // 32-entry blocks: reads stay below 32 * ceil(win / 32) <= vbw, and
        // entries at i >= win are masked after the read.
        uint32_t h1, h2;
        const int nblk = (win + TPR - 1) / TPR;
        {
            const int i = hs;  // block 0, always present
            const uint32_t z1 = Vb1[hr * VBP + i], z2 = Vb2[hr * VBP + v2_pos<OPT == 8>(i, vbw)];
            h1 = i < win ? z1 : 0u;
            h2 = i < win ? z2 : 0u;
        }
#pragma unroll 1
        for (int it = 1; it < nblk; ++it) {
            const int i = hs + it * TPR;
            const uint32_t z1 = Vb1[hr * VBP + i], z2 = Vb2[hr * VBP + v2_pos<OPT == 8>(i, vbw)];
            h1 += i < win ? z1 : 0u;
            h2 += i < win ? z2 : 0u;
        }
        // running sums of the entering-minus-leaving columns
        uint32_t E1[OPT], E2[OPT];
        uint32_t a1 = 0, a2 = 0;
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            a1 += A1[j] - B1[j];
            a2 += A2[j] - B2[j];
            E1[j] = a1;
            E2[j] = a2;
        }
        const uint32_t s1i = scan32(a1), s2i = scan32(a2);
        const uint32_t h1i = scan32(h1), h2i = scan32(h2);
        const uint32_t b1 = half_total(h1i) + s1i - a1;
        const uint32_t b2 = half_total(h2i) + s2i - a2;

        __builtin_amdgcn_s_setprio(0);  // the decisions: fill-in work
        // gray levels of the output row (centre of the window), at ctr_off.
        // (X0 is a multiple of 16 and xr0 = X0 - ceil16(lo + 1), so the
        // window centre of column X0 sits at LDS column off0 + lo =
        // ceil16(lo + 1) and each thread's OPT bytes are OPT-aligned.)
        uint32_t fw[OPT / 4];
        if (OPT == 8) {
            const u32x2 q = *(const lds_v2 *)(lds + ctr_off);
            fw[0] = q.x;
            fw[OPT / 4 - 1] = q.y;
        } else {
            fw[0] = *(const lds_u32 *)(lds + ctr_off);
        }

        // every window of the step's rows has win rows (uniform per step)
        const bool full_rows = y0 - lo >= 0 && y0 + RB - 1 + hi <= a.H - 1;
        const int ny = min(y + hi, a.H - 1) - max(y - lo, 0) + 1;
        const int xs = X0 + hs * OPT;
        uint32_t ow[OPT / 4];
#pragma unroll
        for (int i = 0; i < OPT / 4; ++i) ow[i] = 0u;
        const uint32_t kFF = __builtin_amdgcn_readfirstlane(0xffu), kZero = 0u;
        float sqv[OPT];
        if (x_inside && full_rows) {  // uniform: every window of the step and block is win x win
            const double nb2 = q_full.nd * (double)b2;  // exact: below 2^48
            if (RULE == 0) {
#pragma unroll
                for (int j = 0; j < OPT; ++j) {
                    const bool dark = dark_sauvola_full(q_full, byte_at(fw, j), b1 + E1[j], nb2, (int32_t)E2[j],
                                                        sqv[j]);
                    put_out_byte(ow[j >> 2], j & 3, dark, kFF, kZero);
                }
            } else {
#pragma unroll
                for (int j = 0; j < OPT; ++j) {
                    const bool dark = dark_niblack_full(a, q_full, n_full, byte_at(fw, j), b1 + E1[j], nb2,
                                                        (int32_t)E2[j], sqv[j]);
                    put_out_byte(ow[j >> 2], j & 3, dark, kFF, kZero);
                }
            }
        } else {  // clipped windows: n per pixel, no division
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int X = xs + j;
                const int nx = x_inside ? win : min(X + hi, a.W - 1) - max(X - lo, 0) + 1;
                const uint32_t n = (uint32_t)__mul24(nx, ny);
                const bool dark = RULE == 0 ? dark_sauvola(a, byte_at(fw, j), b1 + E1[j], b2 + E2[j], n, sqv[j])
                                            : dark_niblack(a, byte_at(fw, j), b1 + E1[j], b2 + E2[j], n, sqv[j]);
                put_out_byte(ow[j >> 2], j & 3, dark, kFF, kZero);
            }
        }
        // The rows of the next step go where no thread reads during the
        // horizontal pass: in the blocks layout the entering and leaving
        // blocks (read by the vertical pass only), in the ring the slots of
        // this step's leaving rows (see ring_depth).  Storing them here,
        // before this step's output stores, means the wait for their loads
        // (issued a step ago) does not also wait for output stores just
        // issued: vector-memory waits count loads and stores together, in
        // order.
        __builtin_amdgcn_s_setprio(1);
        if (blocks) {
            if (y0 + RB < Yend) {
                pre.store_rows(a, blkE, RB, xr0, clamp);
                pre_l.store_rows(a, blkL, RB, xr0, clamp);
                if (y0 + 2 * RB < Yend) {
                    pre.fetch(a, y0 + 2 * RB + hi, RB, xr0, clamp);
                    pre_l.fetch(a, y0 + 2 * RB - lo - 1, RB, xr0, clamp);
                }
            }
        } else {
            s_in = s_in + RB >= depth ? s_in + RB - depth : s_in + RB;
            advance(ctr_off);
            s_out = s_out + RB >= depth ? s_out + RB - depth : s_out + RB;
            if (y0 + RB < Yend) {
                pre.store_at(a, lds, st_off, RB, xr0, clamp);
                advance(st_off);
                if (y0 + 2 * RB < Yend) pre.fetch(a, y0 + 2 * RB + hi, RB, xr0, clamp);
            }
        }
        if (y < Yend) {
            if (INT) {  // W is a multiple of 16: the thread's outputs lie wholly inside or outside
                if (xs < a.W) {
                    // the step's first output row (uniform) plus a fixed 32-bit offset
                    glb_u8 *p = uniform_global(a.out + (size_t)y0 * (size_t)a.pitch_out) + out_off;
                    if (OPT == 8)
                        store_nt8(p, ow[0], ow[OPT / 4 - 1]);
                    else
                        store_nt4(p, ow[0]);
                }
            } else if (BODY == kWide && xs + OPT <= a.W) {  // every output inside the row
                glb_u8 *p = uniform_global(a.out + (size_t)y0 * (size_t)a.pitch_out) + out_off;
                if (OPT == 8)
                    store_nt8_a1(p, ow[0], ow[OPT / 4 - 1]);
                else
                    store_nt4_a1(p, ow[0]);
            } else {
                store_row<OPT>(a.out + (size_t)y * (size_t)a.pitch_out, xs, a.W, ow);
            }
            if (STATS) {
#pragma unroll
                for (int j = 0; j < OPT; ++j) {
                    const int X = xs + j;
                    if (X >= a.W) continue;
                    const size_t i = (size_t)y * a.W + X;
                    const uint32_t n = (uint32_t)__mul24(min(X + hi, a.W - 1) - max(X - lo, 0) + 1, ny);
                    if (a.gray) a.gray[i] = (uint8_t)byte_at(fw, j);
                    if (a.s1) a.s1[i] = b1 + E1[j];
                    if (a.s2) a.s2[i] = b2 + E2[j];
                    if (a.n) a.n[i] = n;
                    if (a.t) a.t[i] = threshold_value<RULE>(a, b1 + E1[j], n, sqv[j]);
                }
            }
        }
        __syncthreads();  // next step: ring rows stored, V rows free again
    }
}

// Pages with aligned rows take a specialised body (a uniform choice per
// launch): input rows 16-byte aligned and a multiple of 16 pixels wide, so
// every 16-pixel chunk lies wholly inside or outside the image and staging
// loads whole chunks with no per-byte masking; output rows 8-byte aligned, so
// every thread stores its outputs with one store.  Other pages take the wide
// body when they are at least 16 pixels wide and both pitches are below 2^28
// (unaligned 16-byte loads and 8-byte stores), else the edge body.  All
// bodies produce identical bytes.  In each, tiles whose windows all span win
// columns decide steps whose windows also span win rows with the per-tile
// constants, and every other step with per-pixel n.  BLK selects the blocks
// layout of the input rows (gray pages; see gray_blocks), a separate kernel
// so that each layout gets its own register allocation.
template <int TW, int C, int RULE, bool STATS, bool BLK = false>
__device__ __forceinline__ void run_tile(const PageArgs &a, int tile, uint8_t *smem) {
    if (a.row_aligned) {
        process_tile<TW, C, RULE, STATS, kAligned, BLK>(a, tile, smem);
        return;
    }
    if (!a.small_pitch || a.W < 16)
        process_tile<TW, C, RULE, STATS, kEdge, BLK>(a, tile, smem);
    else
        process_tile<TW, C, RULE, STATS, kWide, BLK>(a, tile, smem);
}

template <int TW, int C, int RULE, bool STATS, bool BLK>
__global__ void __launch_bounds__(kThreads, 4) bz_page_kernel(PageArgs a) {
    extern __shared__ uint4 bz_lds[];
    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    run_tile<TW, C, RULE, STATS, BLK>(a, tile, (uint8_t *)bz_lds);
}

}  // namespace bz
