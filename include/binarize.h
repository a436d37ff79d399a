/*
 * binarize.h -- C ABI of libbinarize.so: exact locally adaptive (Sauvola /
 * Niblack) binarization of 8-bit document images on AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Mollah, Basu, Nasipuri, "Computationally Efficient Implementation
 * of Convolution-based Locally Adaptive Binarization Techniques",
 * arXiv:1210.3165.  For every pixel the library computes the mean m and the
 * standard deviation s of the gray levels in the W x W window around it
 * (Sec. 2), the Sauvola threshold t = m [1 + k (s / R - 1)] (Sec. 1, Eq. 4) or
 * the Niblack threshold t = m + k s, and the binary output g = 0 if f < t,
 * 255 otherwise (Sec. 1, Eq. 3).  Colour input is first reduced to gray with
 * the weights 0.299 / 0.587 / 0.114 (Sec. 1, Eq. 1).  The window statistics are
 * exact (full window, not the paper's sampled subset S').
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Image layout  img: H rows x W_img columns x `channels` bytes, row-major,
 *               rows contiguous (row pitch = W_img * channels), channels
 *               interleaved r, g, b.  out: H x W_img bytes, row pitch W_img.
 * Gray level    channels == 1: f = img.  channels == 3:
 *               f = (299 r + 587 g + 114 b + 500) / 1000 in integers, i.e. the
 *               Eq. 1 weighted sum rounded to nearest with halves up.
 * Window        rows [y - lo, y + hi] and columns [x - lo, x + hi] with
 *               lo = win / 2 and hi = win - 1 - lo (an even window reaches one
 *               further up/left), intersected with the image; n is the number
 *               of in-image window pixels.  Window sums S1 = sum f and
 *               S2 = sum f^2 are exact 32-bit integers for win <= 255.
 * Statistics    m = S1 / n, s = sqrt(n S2 - S1^2) / n (population deviation;
 *               n S2 - S1^2 is formed exactly).
 * Threshold     rule BZ_SAUVOLA: t = m (1 + k (s / R - 1))   (Eq. 4)
 *               rule BZ_NIBLACK: t = m + k s                 (R unused)
 *               from the exact integer sums: sqrt(n S2 - S1^2) in fp32, the
 *               rest of the Sauvola threshold and its comparison in fp64,
 *               the Niblack comparison in fp32.  For the accepted k and R
 *               (see Limits) the threshold the decision uses, and the fp32
 *               t plane of binarize_stats, stay within 1e-4 gray levels of
 *               the exact t: at most about 4.5e-5 (Sauvola) and 2.5e-5
 *               (Niblack) from the square root, plus 3.1e-5 of fp32
 *               rounding in the t plane.
 * Output        out = 0 where f < t, 255 elsewhere (ties give 255, Eq. 3).
 * Pointers      img, out and every plane are DEVICE pointers owned by the
 *               caller (e.g. torch CUDA tensors).  The library never
 *               allocates, frees or keeps them; the single-image entry points
 *               allocate no device memory at all.  out must not overlap img.
 * Streams       `stream` is a hipStream_t passed as void*; NULL selects the
 *               default (null) stream.  Every call only enqueues work and
 *               returns; results are ready when the stream is synchronised.
 * Graphs        binarize*, binarize_otsu, binarize_gs and
 *               binarize_fmeasure_counts enqueue kernel launches only (no
 *               memset, allocation or host synchronisation), so a caller
 *               may capture them in a HIP graph and replay it.  The batch
 *               object has its own graph mode and is not capturable: a run
 *               waits on the host for its previous run.
 * Errors        0 on success, a negative BZ_ERR_* code otherwise.  Arguments
 *               are validated before anything is enqueued; on BZ_ERR_HIP the
 *               HIP error code is kept per thread (binarize_last_hip_error).
 *               Faults inside a kernel surface at the caller's next
 *               synchronisation, as with any asynchronous HIP launch.
 * Limits        1 <= win <= 255; channels in {1, 3}; H, W_img >= 1;
 *               H * W_img * channels < 2^31; -1 <= k <= 1; R finite and
 *               > 0, and R >= 64 for BZ_SAUVOLA (outside this range the
 *               1e-4 bound above would not hold: BZ_ERR_PARAM).
 * Threads       All entry points are re-entrant; calls that share a stream
 *               are ordered by that stream.
 */
#ifndef BINARIZE_H
#define BINARIZE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BINARIZE_VERSION 1

/* Threshold rules. */
#define BZ_SAUVOLA 0 /* Sec. 1, Eq. 4 */
#define BZ_NIBLACK 1 /* t = m + k s  */

/* Status codes. */
#define BZ_OK 0
#define BZ_ERR_NULL (-1)        /* a required pointer is NULL               */
#define BZ_ERR_SHAPE (-2)       /* H or W_img < 1, image too big, bad pitch */
#define BZ_ERR_CHANNELS (-3)    /* channels not 1 or 3                      */
#define BZ_ERR_WINDOW (-4)      /* win outside [1, 255]                     */
#define BZ_ERR_PARAM (-5)       /* |k| > 1, R <= 0, or Sauvola R < 64       */
#define BZ_ERR_RULE (-6)        /* rule not BZ_SAUVOLA / BZ_NIBLACK         */
#define BZ_ERR_ALIAS (-7)       /* out overlaps img (or a stats plane)      */
#define BZ_ERR_HIP (-8)         /* the HIP runtime refused a call           */
#define BZ_ERR_TILE (-9)        /* unsupported tile configuration           */
#define BZ_ERR_WORKSPACE (-10)  /* workspace missing or too small           */

/*
 * binarize -- binarize one image on the null stream (Sec. 1, Eq. 1, 3, 4;
 * Sec. 2).  img: device, H x W_img x channels; out: device, H x W_img.
 * Returns after enqueueing the work.
 */
int binarize(const uint8_t *img, int H, int W_img, int channels, int win,
             float k, float R, int rule, uint8_t *out);

/* binarize_async -- as binarize, enqueued on `stream` (a hipStream_t). */
int binarize_async(const uint8_t *img, int H, int W_img, int channels, int win,
                   float k, float R, int rule, uint8_t *out, void *stream);

/*
 * binarize_pitched -- as binarize_async for an image and an output whose rows
 * are not contiguous: a crop or a padded-row layout inside a larger buffer
 * (the M x N matrix of Sec. 1 as a window into that buffer).  pitch_in is
 * the number of bytes from one input row to the next (>= W_img * channels),
 * pitch_out the same for the output (>= W_img); 0 selects the contiguous
 * pitch.  Only the H rows of W_img * channels (W_img) bytes are read
 * (written): bytes between rows are never touched.  The output rows must
 * not share a byte with the input rows (the test is exact, so interleaved
 * rows of one buffer are accepted).  BZ_ERR_SHAPE for a pitch below the row
 * size or negative; the other errors as binarize.
 */
int binarize_pitched(const uint8_t *img, int H, int W_img, int channels,
                     int64_t pitch_in, int win, float k, float R, int rule,
                     uint8_t *out, int64_t pitch_out, void *stream);

/*
 * binarize_tuned -- as binarize_async with an explicit tile shape: tile_w
 * output columns (128 or 256; 256 needs win <= 241) by tile_h output rows
 * (a multiple of 8, 8..4096) per workgroup.  The result is bit-identical
 * for every tile shape; only the speed changes.  BZ_ERR_TILE otherwise.
 */
int binarize_tuned(const uint8_t *img, int H, int W_img, int channels, int win,
                   float k, float R, int rule, uint8_t *out, int tile_w,
                   int tile_h, void *stream);

/*
 * binarize_staged -- as binarize_async, computed in two passes through HBM
 * (the unfused form): a row pass writes the row window sums of f and f^2
 * (Sec. 2) of every pixel to two u32 planes in the caller's workspace, and a
 * column pass sums them down the window and decides (Eq. 3, Eq. 4 / Niblack).
 * The output is identical, byte for byte, to binarize's.  It moves about
 * 24 B/px more than binarize and exists so that the autotuner can measure
 * pass fusion.
 *   ws: device workspace of at least binarize_staged_workspace_size(H, W_img)
 *       bytes (8 H W_img), 4-byte aligned, not overlapping img or out; its
 *       contents are overwritten.  BZ_ERR_WORKSPACE if missing, too small or
 *       misaligned; BZ_ERR_ALIAS on overlap; the other errors as binarize.
 */
int binarize_staged(const uint8_t *img, int H, int W_img, int channels,
                    int win, float k, float R, int rule, uint8_t *out,
                    uint32_t *ws, size_t ws_bytes, void *stream);

/* Workspace bytes binarize_staged needs for an H x W_img page (0 if the
 * shape is invalid). */
size_t binarize_staged_workspace_size(int H, int W_img);

/*
 * binarize_stats -- as binarize_async, and also writes the intermediate
 * quantities of every pixel, each an H x W_img device plane (row pitch
 * W_img): gray (u8, Eq. 1), s1 and s2 (u32 window sums of f and f^2), n
 * (u32 in-image window count) and t (f32 threshold, Eq. 4 or Niblack).  Any
 * plane may be NULL.  Meant for verification; slower than binarize.
 */
int binarize_stats(const uint8_t *img, int H, int W_img, int channels,
                   int win, float k, float R, int rule, uint8_t *out,
                   uint8_t *gray, uint32_t *s1, uint32_t *s2, uint32_t *n,
                   float *t, void *stream);

/*
 * Batched form: many pages of uneven size, channels, window, k, R and rule in
 * a few persistent launches on one stream.  Every tile of every page is a
 * work item that workgroups take from a device counter, so uneven pages
 * leave no idle tail per page; each page's output is bit-identical to
 * binarizing it alone.  Pages are grouped by tile width, input-row layout
 * and LDS need: each group is one launch whose workgroups reserve the LDS
 * share of the highest occupancy that holds its tiles (4, 3, 2 or 1
 * workgroups per CU), so narrow windows keep four workgroups per CU when
 * wide ones share the batch.  Gray pages whose ring of rows would exceed a
 * quarter of the CU's LDS take the blocks layout (three 8-row blocks, at
 * most 38 KiB for any window), as in the single-page kernel.
 *
 * binarize_batch_create -- allocate a batch object for up to max_pages pages:
 *   two sets of a device page table, a pinned host staging copy of it, work
 *   counters and an event; a capture stream; host scratch for checking the
 *   pages.
 *   lds_cap_bytes bounds the LDS of one workgroup (0: 81856, the share of
 *   two workgroups per CU; at most 163776); a page's tile takes 256 columns
 *   when that fits the cap, else 128, and pages that fit neither fail with
 *   BZ_ERR_TILE.  The only entry points that allocate.
 * binarize_batch_run -- plan the pages (host, into the pinned table), then
 *   enqueue on `stream`: table copy, counter reset, one persistent kernel per
 *   group of pages (each starts when the previous one ends).  With
 *   use_graph != 0 these are captured into a HIP graph on the first call
 *   and replayed afterwards (the table contents change, the graph does not;
 *   it is captured again when n_pages rounded up to a power of two, at
 *   least 64, or the set of groups changes).  Within a group, items run
 *   longest tile first.
 *   An object holds two sets of run buffers (pinned and device table, work
 *   counters, graph) and uses them in turn: a run waits on the host only
 *   for the run before the previous one, so planning overlaps the GPU's
 *   work on the previous run.  Every img/out pointer must stay valid until the stream reaches
 *   the end of the run.  Errors as for binarize (per page), BZ_ERR_SHAPE for
 *   n_pages outside [1, max_pages], BZ_ERR_ALIAS when a page's output
 *   overlaps another page's output or any page's input (the pages run
 *   concurrently; inputs may be shared).
 * binarize_batch_info -- persistent grid of 256-column ring pages at four
 *   workgroups per CU, LDS cap, items of the last run.
 * binarize_batch_destroy -- wait for the last run, free everything.
 */
typedef struct bz_page {
    const uint8_t *img; /* device, H rows of W_img x channels bytes          */
    uint8_t *out;       /* device, H rows of W_img bytes                     */
    int H, W_img, channels, win;
    float k, R;
    int rule;           /* BZ_SAUVOLA or BZ_NIBLACK                          */
    int tile_w, tile_h; /* 0: chosen by the library (tile_h default 128)    */
    int64_t pitch_in;   /* bytes between input rows, 0: W_img * channels     */
    int64_t pitch_out;  /* bytes between output rows, 0: W_img               */
} bz_page;

typedef struct bz_batch bz_batch; /* opaque batch object */

/*
 * binarize_batch -- the batched form in one call (Sec. 1, Eq. 1, 3, 4;
 * Sec. 2 on every page): validates and plans `pages` and enqueues their
 * persistent launch on `stream`, as binarize_batch_run without a graph.
 * The library keeps one batch object per device for these calls (created
 * on first use, grown to the largest n_pages seen, kept until the process
 * ends); a call waits on the host for the run before the previous one.  Errors as binarize_batch_run; BZ_ERR_NULL for a NULL
 * pages array.
 */
int binarize_batch(const bz_page *pages, int n_pages, void *stream);

int binarize_batch_create(int max_pages, int lds_cap_bytes, bz_batch **out);
int binarize_batch_run(bz_batch *b, const bz_page *pages, int n_pages,
                       int use_graph, void *stream);
int binarize_batch_info(const bz_batch *b, int *grid, int *lds_cap,
                        int *last_items);
void binarize_batch_destroy(bz_batch *b);

/*
 * Otsu global threshold -- the paper's global baseline (Sec. 1, Eq. 2),
 * whose single threshold T comes from Otsu's method.  From the 256-bin
 * histogram of the Eq. 1 gray levels f, every split level k defines the
 * classes {f <= k} and {f > k}; k* is the first level with the largest
 * between-class variance w0 w1 (mu0 - mu1)^2 (w = class share of the pixels,
 * mu = class mean; 0 when a class is empty, so k* = 0 if nothing can be
 * separated), evaluated in fp64.  T = k* + 1 and out = 0 where f < T, 255
 * elsewhere.
 *
 * binarize_otsu -- img: device, H x W_img x channels (layout as above).
 *   out: device, H x W_img, or NULL to compute only the histogram and T.
 *   ws: device workspace of at least BZ_OTSU_WS_BYTES bytes, 16-byte aligned,
 *   owned by the caller; it needs no initialisation (every call rewrites
 *   what it reads).  After the call (in stream order) ws holds, as u32
 *   words, the histogram at BZ_OTSU_WS_HIST (256 words), T at BZ_OTSU_WS_T
 *   and k* at BZ_OTSU_WS_KSTAR; the rest is scratch.  Calls that share a
 *   workspace must be ordered (same stream, or synchronised).  Three
 *   launches (histogram, selection, decision; two if out is NULL); no
 *   allocation.  Errors: BZ_ERR_NULL (img), BZ_ERR_WORKSPACE (ws NULL, too
 *   small or misaligned), BZ_ERR_SHAPE, BZ_ERR_CHANNELS, BZ_ERR_ALIAS (out,
 *   img and ws must not overlap), BZ_ERR_HIP.
 * binarize_otsu_workspace_size -- BZ_OTSU_WS_BYTES.
 */
#define BZ_OTSU_WS_BYTES (4096 + 512 * 1024)
#define BZ_OTSU_WS_HIST 0
#define BZ_OTSU_WS_T 256
#define BZ_OTSU_WS_KSTAR 257

int binarize_otsu(const uint8_t *img, int H, int W_img, int channels, uint8_t *out,
                  uint32_t *ws, size_t ws_bytes, void *stream);
size_t binarize_otsu_workspace_size(void);

/*
 * binarize_otsu_noalloc -- binarize_otsu for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same three launches and the same
 * results, with the caller's workspace replaced by a scratch array inside
 * the library: BZ_OTSU_WS_BYTES (528 KiB) per device, held until the process
 * ends.  The call allocates nothing and calls no allocating routine; the
 * scratch needs no clearing (every word a call reads, it first writes).
 *   img, out: as binarize_otsu (out may be NULL: threshold only).
 *   result: device, optional (NULL to skip), at least 258 u32 words, 4-byte
 *     aligned; receives the histogram (words 0..255), T (word 256) and k*
 *     (word 257), the words binarize_otsu leaves in its workspace.
 * Sizes: as binarize_otsu (H * W_img * channels < 2^31, else BZ_ERR_SHAPE);
 * the scratch is sized for the largest grid the call launches, so no image
 * size depends on it.
 * Concurrency: every call on one device shares that device's scratch.
 * Calls that may overlap on one device (different streams without
 * ordering, or several host threads) race and can return wrong results;
 * order them.
 * Errors: as binarize_otsu; BZ_ERR_WORKSPACE if result is misaligned,
 * BZ_ERR_ALIAS if result overlaps img or out, BZ_ERR_HIP if the scratch's
 * device address cannot be obtained.
 */
int binarize_otsu_noalloc(const uint8_t *img, int H, int W_img, int channels,
                          uint8_t *out, uint32_t *result, void *stream);

/*
 * Sampled-window Sauvola -- the paper's variant (Sec. 2, Eq. 5): mean m' and
 * deviation s' over a subset S' of O(W) window pixels on a geometric
 * structure, t' = m' [1 + k (s'/R' - 1)] with R' the dynamic range of s',
 * out = 0 where f < t', 255 elsewhere (Eq. 3).  The paper's own structures
 * (its Fig. 1) are not available; these three are this library's, as
 * offsets (dy, dx) from the centre of an ODD win x win window:
 *   BZ_GS_PLUS  dy == 0 or dx == 0 (centre row and column, 2 win - 1 px)
 *   BZ_GS_X     |dy| == |dx|       (both diagonals,        2 win - 1 px)
 *   BZ_GS_STAR  both               (                       4 win - 3 px)
 * clipped to the image; n' counts the in-image members.  Sums are exact,
 * s' = sqrt(n' S2' - S1'^2) / n', t' is evaluated as for binarize (same
 * precision and bound, |t' - t'_exact| < 1e-4, for -1 <= k <= 1 and
 * R' >= 64).
 *
 * binarize_gs -- img, out as for binarize; Rp is R'.  s1, s2, n (u32) and
 *   t (f32) are optional H x W_img verification planes (NULL to skip).
 *   Errors: BZ_ERR_WINDOW for an even win or one outside [1, 255],
 *   BZ_ERR_PARAM for an unknown structure, |k| > 1 or not finite, or Rp
 *   not finite or below 64, otherwise as for binarize_stats.  No
 *   allocation, one launch.
 */
#define BZ_GS_PLUS 0
#define BZ_GS_X 1
#define BZ_GS_STAR 2

int binarize_gs(const uint8_t *img, int H, int W_img, int channels, int win,
                float k, float Rp, int structure, uint8_t *out, uint32_t *s1,
                uint32_t *s2, uint32_t *n, float *t, void *stream);

/*
 * binarize_fmeasure_counts -- the counts behind the F-measure of Sec. 3
 * (Eq. 6: FM = 2 R P / (R + P), R = TP / (TP + FN), P = TP / (TP + FP)).
 * out: device, npx binarized bytes (0 = text, Eq. 3); gt: device, npx
 * ground-truth bytes (nonzero = text).  counts: device, 3 x u64, 8-byte
 * aligned, overwritten with TP (out == 0, gt != 0), FP (out == 0, gt == 0)
 * and FN (out != 0, gt != 0).  Two launches (clear, count); no allocation.
 * Errors: BZ_ERR_NULL, BZ_ERR_SHAPE (npx outside [1, 2^31)),
 * BZ_ERR_WORKSPACE (counts misaligned), BZ_ERR_ALIAS, BZ_ERR_HIP.
 */
int binarize_fmeasure_counts(const uint8_t *out, const uint8_t *gt, int64_t npx,
                             unsigned long long *counts, void *stream);

/* LDS bytes one workgroup of the given tile width needs for a window and a
 * channel count (1 or 3: gray pages keep three 8-row blocks of input rows in
 * LDS, colour pages a ring of win + 8 or more rows), or BZ_ERR_TILE if that
 * tile cannot hold the window (BZ_ERR_WINDOW, BZ_ERR_CHANNELS for arguments
 * out of range). */
int binarize_tile_lds(int tile_w, int win, int channels);

/* Default tile shape binarize/binarize_async pick for a problem. */
int binarize_default_tile(int H, int W_img, int channels, int win,
                          int *tile_w, int *tile_h);

/* Diagnostics. */
const char *binarize_strerror(int code); /* static string, never NULL      */
int binarize_version(void);              /* BINARIZE_VERSION               */
int binarize_last_hip_error(void);       /* hipError_t of the last BZ_ERR_HIP
                                            on this thread (0 if none)      */

#ifdef __cplusplus
}
#endif

#endif /* BINARIZE_H */
