// bz_batch.hip -- many pages of uneven size, channels, window and rule in
// one persistent launch (the batched form of the tile kernel), optionally
// replayed from a captured HIP graph.
//
// Every tile of every page is one work item.  Items are numbered page by page
// (page p owns items [item0[p], item0[p] + tiles[p])); a workgroup takes the
// next item from a device counter, finds its page by binary search over
// item0, and runs the tile code of that page's variant (tile width,
// channels, rule) -- the same code as the single-page kernel.  Results are
// bit-identical to binarizing each page alone: the arithmetic of a pixel does
// not depend on which tile, launch or neighbour page it is computed with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>

#include "binarize.h"
#include "bz_common.hpp"
#include "bz_host.hpp"
#include "bz_tile.hpp"

using namespace bz;

namespace {

// Tile variant of a page, 0..7: (tile_w == 256) * 4 + (channels == 3) * 2 + rule.
inline int kind_of(int tile_w, int channels, int rule) { return (tile_w == 256) * 4 + (channels == 3) * 2 + rule; }

struct BatchHeader {
    uint32_t n_pages;
    uint32_t n_items;
    uint32_t pad[14];
};

struct BatchPage {
    PageArgs a;
    int item0;  // first work item of this page
    int kind;   // tile variant, kind_of()
    int pad[2];
};

// Persistent workgroups pull items until the counter passes n_items; every
// workgroup reaches that exit because the counter only grows.  One kernel
// holds all eight tile variants and branches on the page's kind (uniform per
// workgroup), so pages of every kind share one launch and one queue of
// items.  MINW is the occupancy the register budget is sized for (waves per
// SIMD): 2 for LDS caps above a quarter of the CU's LDS, 4 below.
template <int MINW>
__global__ void __launch_bounds__(kThreads, MINW)
    bz_batch_kernel(const BatchHeader *__restrict__ hdr, const BatchPage *__restrict__ pages,
                    uint32_t *__restrict__ counter) {
    extern __shared__ uint4 bz_lds[];
    __shared__ int s_item;
    uint8_t *smem = (uint8_t *)bz_lds;
    const int n_items = (int)hdr->n_items;
    const int n_pages = (int)hdr->n_pages;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        // uniform across the workgroup: keep it (and the page search and page
        // fields that follow) in scalar registers
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();  // every thread has read s_item before it is rewritten
        if (item >= n_items) break;
        int lo = 0, hi = n_pages - 1;
        while (lo < hi) {  // last page whose first item is <= item
            const int mid = (lo + hi + 1) >> 1;
            if (pages[mid].item0 <= item) lo = mid;
            else hi = mid - 1;
        }
        const BatchPage &pg = pages[lo];
        const int tile = item - pg.item0;
        switch (__builtin_amdgcn_readfirstlane(pg.kind)) {
            case 0: run_tile<128, 1, BZ_SAUVOLA, false>(pg.a, tile, smem); break;
            case 1: run_tile<128, 1, BZ_NIBLACK, false>(pg.a, tile, smem); break;
            case 2: run_tile<128, 3, BZ_SAUVOLA, false>(pg.a, tile, smem); break;
            case 3: run_tile<128, 3, BZ_NIBLACK, false>(pg.a, tile, smem); break;
            case 4: run_tile<256, 1, BZ_SAUVOLA, false>(pg.a, tile, smem); break;
            case 5: run_tile<256, 1, BZ_NIBLACK, false>(pg.a, tile, smem); break;
            case 6: run_tile<256, 3, BZ_SAUVOLA, false>(pg.a, tile, smem); break;
            default: run_tile<256, 3, BZ_NIBLACK, false>(pg.a, tile, smem); break;
        }
        __syncthreads();  // the next item restages LDS
    }
}

using BatchKernel = void (*)(const BatchHeader *, const BatchPage *, uint32_t *);
const BatchKernel kBatchKernels[2] = {bz_batch_kernel<2>, bz_batch_kernel<4>};

// LDS the batch kernels declare statically (the item slot), rounded up.
constexpr int kStaticLds = 64;

__global__ void bz_counter_reset(uint32_t *counter) {
    if (threadIdx.x == 0) *counter = 0u;
}

int fail(hipError_t e) {
    bz::set_last_hip_error((int)e);
    return BZ_ERR_HIP;
}

}  // namespace

// Bytes a page's output rows span, for the batch alias check.
struct Span {
    uintptr_t begin, end;
    int page;
};

// Tile choice and work estimate of one page, for ordering the item list.
struct PagePlan {
    double cost;  // estimated time of one of its tiles (arbitrary unit)
    int tw, th, kind, page;
};

// Opaque batch object (bz_batch in the C ABI).
struct bz_batch {
    int max_pages;
    int lds_cap;
    int grid;
    size_t table_bytes;
    void *host_table;    // pinned staging copy of header + pages
    void *dev_table;     // device copy read by the kernel
    uint32_t *counter;   // device work counter
    hipStream_t cap_stream;
    hipGraph_t graph;       // captured for tables of up to graph_pages pages
    hipGraphExec_t exec;
    int graph_pages;
    int variant;            // 0: register budget for 2 workgroups per CU, 1: for 4
    hipEvent_t done;     // completion of the last run (guards the pinned table)
    bool pending;
    int last_items;
    Span *spans;            // host scratch for the alias check: max_pages output spans
    uintptr_t *span_max;    // and the running maximum of their ends
    ImageDesc *descs;       // the checked pages (pitches filled in)
    PagePlan *plans;        // tile choice and order of the pages
};

namespace {

ImageDesc page_desc(const bz_page &p) {
    return ImageDesc{p.img, p.out, p.H, p.W_img, p.channels, p.pitch_in, p.pitch_out};
}

// The pages of a batch run concurrently, so no output may overlap another
// page's output or any page's input (inputs may overlap each other: they
// are only read).  Output spans sorted by their first byte, with the running
// maximum of their ends, bound the candidates of each comparison; only
// candidates whose spans intersect get the exact strided test, so disjoint
// pages cost O(n log n).  `descs` holds the checked pages (pitches filled).
int check_cross_alias(const ImageDesc *descs, int n, Span *spans, uintptr_t *span_max) {
    for (int i = 0; i < n; ++i) {
        const Region r = output_region(descs[i]);
        spans[i] = Span{r.base, region_end(r), i};
    }
    std::sort(spans, spans + n, [](const Span &a, const Span &b) { return a.begin < b.begin; });
    for (int i = 0; i < n; ++i) span_max[i] = i ? std::max(span_max[i - 1], spans[i].end) : spans[i].end;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n && spans[j].begin < spans[i].end; ++j)
            if (regions_overlap(output_region(descs[spans[i].page]), output_region(descs[spans[j].page])))
                return BZ_ERR_ALIAS;
    for (int i = 0; i < n; ++i) {
        const Region in = input_region(descs[i]);
        const uintptr_t a = in.base, b = region_end(in);
        // outputs starting before the input ends, latest first, while some
        // earlier output may still end after the input starts
        int j = (int)(std::lower_bound(spans, spans + n, b, [](const Span &s, uintptr_t v) { return s.begin < v; }) -
                      spans) - 1;
        for (; j >= 0 && span_max[j] > a; --j)
            if (spans[j].end > a && regions_overlap(in, output_region(descs[spans[j].page]))) return BZ_ERR_ALIAS;
    }
    return BZ_OK;
}

// Tile for one page within the batch's LDS cap: the caller's choice if it
// fits, else 256 columns when the window allows, else 128; tile_h 128 unless
// given.
int page_tile(const bz_page &p, int lds_cap, int *tw, int *th) {
    int w = p.tile_w, h = p.tile_h;
    if (w == 0) {
        w = (tile_fits(256, p.win, p.channels, false) && tile_lds_bytes(256, p.win, p.channels, false) <= lds_cap)
                ? 256
                : 128;
    }
    if (h == 0) h = 128;
    if (w != 128 && w != 256) return BZ_ERR_TILE;
    if (h < kRowsPerStep || h > 4096 || h % kRowsPerStep) return BZ_ERR_TILE;
    if (!tile_fits(w, p.win, p.channels, false) || tile_lds_bytes(w, p.win, p.channels, false) > lds_cap)
        return BZ_ERR_TILE;
    *tw = w;
    *th = h;
    return BZ_OK;
}

// Table bytes for n pages.
size_t table_size(int n) { return sizeof(BatchHeader) + (size_t)n * sizeof(BatchPage); }

// Fill header + pages of the table at `mem` and return the item count in
// *items.  Pages are ordered by the estimated time of one of their tiles,
// longest first (ties: kind, then the caller's order), so the queue ends
// with the shortest items and the last workgroups to finish finish close
// together; pages of one kind stay mostly adjacent.
int plan(const bz_page *pages, int n, int lds_cap, void *mem, ImageDesc *descs, Span *spans, uintptr_t *span_max,
         PagePlan *plans, int *items) {
    BatchHeader *hdr = (BatchHeader *)mem;
    BatchPage *bp = (BatchPage *)(hdr + 1);
    std::memset(hdr, 0, sizeof(*hdr));
    for (int i = 0; i < n; ++i) {
        const bz_page &p = pages[i];
        descs[i] = page_desc(p);
        int rc = check_page(descs[i], p.win, p.k, p.R, p.rule);
        if (rc) return rc;
        PagePlan &q = plans[i];
        if ((rc = page_tile(p, lds_cap, &q.tw, &q.th))) return rc;
        q.kind = kind_of(q.tw, p.channels, make_decision(p.rule, p.k, p.R, p.win).rule);
        q.page = i;
        // rows streamed (with the window's start-up rows) times columns
        // summed (with the halo); colour pages also convert on staging
        q.cost = (double)(q.th + p.win - 1) * (double)(q.tw + p.win - 1) * (p.channels == 3 ? 1.5 : 1.0);
    }
    if (int rc = check_cross_alias(descs, n, spans, span_max)) return rc;
    std::sort(plans, plans + n, [](const PagePlan &x, const PagePlan &y) {
        if (x.cost != y.cost) return x.cost > y.cost;
        if (x.kind != y.kind) return x.kind < y.kind;
        return x.page < y.page;
    });
    long total = 0;
    for (int j = 0; j < n; ++j) {
        const PagePlan &q = plans[j];
        const bz_page &p = pages[q.page];
        BatchPage &e = bp[j];
        std::memset(&e, 0, sizeof(e));
        e.a = page_args(descs[q.page], p.win, p.k, p.R, p.rule, q.tw, q.th, false);
        e.item0 = (int)total;
        e.kind = q.kind;
        total += e.a.n_tiles;
        if (total >= (1L << 31)) return BZ_ERR_SHAPE;
    }
    hdr->n_pages = (uint32_t)n;
    hdr->n_items = (uint32_t)total;
    *items = (int)total;
    return BZ_OK;
}

// Enqueue the copy of the first `bytes` of the table, the counter reset and
// the persistent kernel.
int record(bz_batch *b, size_t bytes, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(b->dev_table, b->host_table, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(e);
    hipLaunchKernelGGL(bz_counter_reset, dim3(1), dim3(64), 0, st, b->counter);
    const BatchHeader *hdr = (const BatchHeader *)b->dev_table;
    const BatchPage *pg = (const BatchPage *)(hdr + 1);
    hipLaunchKernelGGL(kBatchKernels[b->variant], dim3((unsigned)b->grid), dim3(kThreads), (unsigned)b->lds_cap,
                       st, hdr, pg, b->counter);
    e = hipGetLastError();
    return e == hipSuccess ? BZ_OK : fail(e);
}

}  // namespace

extern "C" {

int binarize_batch_create(int max_pages, int lds_cap_bytes, bz_batch **out) {
    if (!out) return BZ_ERR_NULL;
    *out = nullptr;
    if (max_pages < 1 || max_pages > (1 << 20)) return BZ_ERR_SHAPE;
    // default: two workgroups per CU with their static LDS
    if (lds_cap_bytes <= 0) lds_cap_bytes = kMaxLds / 2 - kStaticLds;
    if (lds_cap_bytes < tile_lds_bytes(128, 1, 1, false) || lds_cap_bytes > kMaxLds - kStaticLds) return BZ_ERR_TILE;
    bz_batch *b = new (std::nothrow) bz_batch();
    if (!b) return BZ_ERR_HIP;
    b->max_pages = max_pages;
    b->lds_cap = lds_cap_bytes;
    b->variant = (lds_cap_bytes + kStaticLds) * 4 <= kMaxLds ? 1 : 0;
    b->table_bytes = table_size(max_pages);
    hipError_t e = hipSuccess;
    for (int v = 0; v < 2; ++v)
        (void)hipFuncSetAttribute((const void *)kBatchKernels[v], hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kMaxLds - kStaticLds);
    (void)hipGetLastError();
    int per_cu = 1 << 30, dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) {
        delete b;
        return fail(e);
    }
    {  // the grid that fills the GPU
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kBatchKernels[b->variant], kThreads,
                                                              lds_cap_bytes)) != hipSuccess) {
            delete b;
            return fail(e);
        }
    }
    if (per_cu < 1) {
        delete b;
        return BZ_ERR_TILE;
    }
    b->grid = cus * per_cu;
    if ((e = hipHostMalloc(&b->host_table, b->table_bytes, hipHostMallocDefault)) != hipSuccess) {
        delete b;
        return fail(e);
    }
    if ((e = hipMalloc(&b->dev_table, b->table_bytes)) != hipSuccess ||
        (e = hipMalloc((void **)&b->counter, sizeof(uint32_t))) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming)) != hipSuccess) {
        binarize_batch_destroy(b);
        return fail(e);
    }
    std::memset(b->host_table, 0, b->table_bytes);
    b->spans = new (std::nothrow) Span[(size_t)max_pages];
    b->span_max = new (std::nothrow) uintptr_t[(size_t)max_pages];
    b->descs = new (std::nothrow) ImageDesc[(size_t)max_pages];
    b->plans = new (std::nothrow) PagePlan[(size_t)max_pages];
    if (!b->spans || !b->span_max || !b->descs || !b->plans) {
        binarize_batch_destroy(b);
        return BZ_ERR_HIP;
    }
    *out = b;
    return BZ_OK;
}

int binarize_batch_run(bz_batch *b, const bz_page *pages, int n_pages, int use_graph, void *stream) {
    if (!b || !pages) return BZ_ERR_NULL;
    if (n_pages < 1 || n_pages > b->max_pages) return BZ_ERR_SHAPE;
    hipStream_t st = (hipStream_t)stream;
    // the pinned table may still be read by the previous run's copy
    if (b->pending) {
        hipError_t e = hipEventSynchronize(b->done);
        if (e != hipSuccess) return fail(e);
        b->pending = false;
    }
    int items = 0;
    int rc = plan(pages, n_pages, b->lds_cap, b->host_table, b->descs, b->spans, b->span_max, b->plans, &items);
    if (rc) return rc;
    b->last_items = items;
    if (use_graph) {
        // the graph copies a table of graph_pages pages (a power of two, at
        // least 64, at most max_pages); capture again when the batch needs
        // another size
        int gp = 64;
        while (gp < n_pages) gp *= 2;
        if (gp > b->max_pages) gp = b->max_pages;
        if (b->exec && b->graph_pages != gp) {
            (void)hipGraphExecDestroy(b->exec);
            (void)hipGraphDestroy(b->graph);
            b->exec = nullptr;
            b->graph = nullptr;
        }
        if (!b->exec) {
            hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return fail(e);
            rc = record(b, table_size(gp), b->cap_stream);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(b->cap_stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(e);
            b->graph = g;
            if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess) return fail(e);
            b->graph_pages = gp;
        }
        hipError_t e = hipGraphLaunch(b->exec, st);
        if (e != hipSuccess) return fail(e);
    } else {
        rc = record(b, table_size(n_pages), st);
        if (rc) return rc;
    }
    hipError_t e = hipEventRecord(b->done, st);
    if (e != hipSuccess) return fail(e);
    b->pending = true;
    return BZ_OK;
}

int binarize_batch_info(const bz_batch *b, int *grid, int *lds_cap, int *last_items) {
    if (!b) return BZ_ERR_NULL;
    if (grid) *grid = b->grid;
    if (lds_cap) *lds_cap = b->lds_cap;
    if (last_items) *last_items = b->last_items;
    return BZ_OK;
}

}  // extern "C"

namespace {

// Batch objects behind the one-call binarize_batch: two per device, used in
// turn, so a call waits on the host only for the run before the previous
// one (whose pinned table it rewrites).  They grow to the largest call seen
// and live until the process ends.
struct OneCallPool {
    std::mutex mu;
    bz_batch *obj[2] = {nullptr, nullptr};
    int next = 0;
};
OneCallPool g_pools[kMaxDevices];

}  // namespace

extern "C" {

int binarize_batch(const bz_page *pages, int n_pages, void *stream) {
    if (!pages) return BZ_ERR_NULL;
    if (n_pages < 1 || n_pages > (1 << 20)) return BZ_ERR_SHAPE;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(e);
    if (dev < 0 || dev >= kMaxDevices) return fail(hipErrorInvalidDevice);
    OneCallPool &pool = g_pools[dev];
    std::lock_guard<std::mutex> lock(pool.mu);
    bz_batch *&b = pool.obj[pool.next];
    if (!b || b->max_pages < n_pages) {
        if (b) binarize_batch_destroy(b);  // waits for its last run
        b = nullptr;
        int cap = 64;
        while (cap < n_pages) cap *= 2;
        const int rc = binarize_batch_create(cap, 0, &b);
        if (rc) {
            b = nullptr;
            return rc;
        }
    }
    pool.next ^= 1;
    return binarize_batch_run(b, pages, n_pages, 0, stream);
}

void binarize_batch_destroy(bz_batch *b) {
    if (!b) return;
    if (b->pending) (void)hipEventSynchronize(b->done);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->counter) (void)hipFree(b->counter);
    if (b->dev_table) (void)hipFree(b->dev_table);
    if (b->host_table) (void)hipHostFree(b->host_table);
    delete[] b->spans;
    delete[] b->span_max;
    delete[] b->descs;
    delete[] b->plans;
    delete b;
}


}  // extern "C"
