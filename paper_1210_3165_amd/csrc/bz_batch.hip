// bz_batch.hip -- many pages of uneven size, channels, window and rule in
// one batched launch (persistent kernels of the tile code), optionally
// replayed from a captured HIP graph.
//
// Every tile of every page is one work item.  Pages are split into kernel
// groups by tile width and input-row layout, each group a persistent kernel
// launched after the previous one on the same stream.  Items are numbered
// page by page (page p owns items [item0[p], item0[p] + tiles[p])); a
// workgroup takes the next item of its group from the group's device
// counter, finds its page by binary search over item0, and runs the tile
// code of that page's variant (channels, rule) -- the same code as the
// single-page kernel.  Results are bit-identical to binarizing each page
// alone: the arithmetic of a pixel does not depend on which tile, launch,
// layout or neighbour page it is computed with.
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

// Launch L owns pages [page_begin[L], page_begin[L + 1]) and work items
// [item_begin[L], item_begin[L + 1]).
struct BatchHeader {
    uint32_t n_pages;
    uint32_t n_items;
    uint32_t page_begin[kLaunches + 1];
    uint32_t item_begin[kLaunches + 1];
    uint32_t pad[12];
};
static_assert(sizeof(BatchHeader) == 256, "header size");

struct BatchPage {
    PageArgs a;
    int item0;  // first work item of this page
    int kind;   // tile variant within a ring group, kind_of (blocks groups: one variant each)
    int pad[2];
};

// Persistent workgroups pull items of their launch until its counter passes
// its end; every workgroup reaches that exit because the counter only grows.
// A ring group's kernel holds the four ring tile variants of its tile width
// and branches on the page's kind (uniform per workgroup), so gray and
// colour pages of either rule share one launch and one queue of items.  A
// blocks group's kernel holds one variant.  Kernels with more variants
// spilled registers at four workgroups per CU (all eight ring variants: 10
// VGPRs; all four blocks variants: 52), as the register allocation of a
// kernel is that of its costliest variant and the page fields of every
// variant compete for scalar registers.  Blocks pages read their table
// entry through the constant address space, whose loads the compiler may
// repeat instead of keeping every page field in a register (fewer spills).
// MINW is the occupancy the register budget is sized for (waves per SIMD):
// 4 for class 0, 2 (which still fits three waves) for the others.
template <int MINW, int G>
__global__ void __launch_bounds__(kThreads, MINW)
    bz_batch_kernel(const BatchHeader *__restrict__ hdr, const BatchPage *__restrict__ pages,
                    uint32_t *__restrict__ counters, int launch) {
    extern __shared__ uint4 bz_lds[];
    __shared__ int s_item;
    uint8_t *smem = (uint8_t *)bz_lds;
    const int page0 = (int)hdr->page_begin[launch], page1 = (int)hdr->page_begin[launch + 1];
    const int item0 = (int)hdr->item_begin[launch], item1 = (int)hdr->item_begin[launch + 1];
    for (;;) {
        if (threadIdx.x == 0) s_item = item0 + (int)atomicAdd(counters + launch, 1u);
        __syncthreads();
        // uniform across the workgroup: keep it (and the page search and page
        // fields that follow) in scalar registers
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();  // every thread has read s_item before it is rewritten
        if (item >= item1) break;
        int lo = page0, hi = page1 - 1;
        while (lo < hi) {  // last page whose first item is <= item
            const int mid = (lo + hi + 1) >> 1;
            if (pages[mid].item0 <= item) lo = mid;
            else hi = mid - 1;
        }
        if (G < 2) {
            constexpr int TW = G == 0 ? 256 : 128;
            const BatchPage &pg = pages[lo];
            const int tile = item - pg.item0;
            switch (__builtin_amdgcn_readfirstlane(pg.kind)) {
                case 0: run_tile<TW, 1, BZ_SAUVOLA, false>(pg.a, tile, smem); break;
                case 1: run_tile<TW, 1, BZ_NIBLACK, false>(pg.a, tile, smem); break;
                case 2: run_tile<TW, 3, BZ_SAUVOLA, false>(pg.a, tile, smem); break;
                default: run_tile<TW, 3, BZ_NIBLACK, false>(pg.a, tile, smem); break;
            }
        } else {
            constexpr int TW = G >= 4 ? 256 : 128;
            constexpr int RULE = G & 1;
            typedef const __attribute__((address_space(4))) BatchPage ConstPage;
            const BatchPage &pg = *(const BatchPage *)((ConstPage *)pages + lo);
            const int tile = item - pg.item0;
            run_tile<TW, 1, RULE, false, true>(pg.a, tile, smem);
        }
        __syncthreads();  // the next item restages LDS
    }
}

using BatchKernel = void (*)(const BatchHeader *, const BatchPage *, uint32_t *, int);
// [group][register budget: 0 for 2 waves per SIMD, 1 for 4]
const BatchKernel kBatchKernels[kGroups][2] = {
    {bz_batch_kernel<2, 0>, bz_batch_kernel<4, 0>}, {bz_batch_kernel<2, 1>, bz_batch_kernel<4, 1>},
    {bz_batch_kernel<2, 2>, bz_batch_kernel<4, 2>}, {bz_batch_kernel<2, 3>, bz_batch_kernel<4, 3>},
    {bz_batch_kernel<2, 4>, bz_batch_kernel<4, 4>}, {bz_batch_kernel<2, 5>, bz_batch_kernel<4, 5>}};
inline int budget_of(int c) { return c == 0 ? 1 : 0; }

__global__ void bz_counter_reset(uint32_t *counters) {
    if (threadIdx.x < kLaunches) counters[threadIdx.x] = 0u;
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
    int launch;   // launch key: group_of * kClasses + class_of
};

// What one run reads or writes after it is enqueued.  A batch object holds
// two and uses them in turn, so the host plans a run while the GPU still
// executes the one before (it waits only for the run before that, which
// used the same buffers; runs may go to different streams).
struct RunBuffers {
    void *host_table;    // pinned staging copy of header + pages
    void *dev_table;     // device copy read by the kernels
    uint32_t *counter;   // device work counters, one per launch key
    hipGraph_t graph;    // captured for tables of up to graph_pages pages
    hipGraphExec_t exec;
    int graph_pages;
    uint32_t graph_launches;  // launch keys the graph launches (bit L: key L)
    hipEvent_t done;     // completion of the last run on these buffers
    bool pending;
};

// Opaque batch object (bz_batch in the C ABI).
struct bz_batch {
    int max_pages;
    int lds_cap;
    int grid[kLaunches];    // persistent grid of each launch key
    size_t table_bytes;
    RunBuffers buf[2];
    int cur;                // buffers of the next run
    hipStream_t cap_stream;
    int last_items;
    uint32_t last_launches;   // launch keys the last plan used
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

// Table bytes for n pages.
size_t table_size(int n) { return sizeof(BatchHeader) + (size_t)n * sizeof(BatchPage); }

// Fill header + pages of the table at `mem` and return the item count in
// *items and the launch keys used in *launches (bit L: key L).  Pages are
// ordered by launch key, and within a launch by the estimated time of one of
// their tiles, longest first (ties: kind, then the caller's order), so each
// launch's queue ends with its shortest items and its last workgroups finish
// close together; pages of one kind stay mostly adjacent.
int plan(const bz_page *pages, int n, int lds_cap, void *mem, ImageDesc *descs, Span *spans, uintptr_t *span_max,
         PagePlan *plans, int *items, uint32_t *launches) {
    BatchHeader *hdr = (BatchHeader *)mem;
    BatchPage *bp = (BatchPage *)(hdr + 1);
    std::memset(hdr, 0, sizeof(*hdr));
    for (int i = 0; i < n; ++i) {
        const bz_page &p = pages[i];
        descs[i] = page_desc(p);
        int rc = check_page(descs[i], p.win, p.k, p.R, p.rule);
        if (rc) return rc;
        PagePlan &q = plans[i];
        bool blk = false;
        int lds = 0;
        if ((rc = page_tile(p, lds_cap, &q.tw, &q.th, &blk, &lds))) return rc;
        const int rule = make_decision(p.rule, p.k, p.R, p.win).rule;
        q.kind = kind_of(p.channels, rule);
        q.launch = group_of(q.tw, rule, blk) * kClasses + class_of(lds);
        q.page = i;
        // rows streamed (with the window's start-up rows) times columns
        // summed (with the halo); colour pages also convert on staging
        q.cost = (double)(q.th + p.win - 1) * (double)(q.tw + p.win - 1) * (p.channels == 3 ? 1.5 : 1.0);
    }
    if (int rc = check_cross_alias(descs, n, spans, span_max)) return rc;
    std::sort(plans, plans + n, [](const PagePlan &x, const PagePlan &y) {
        if (x.launch != y.launch) return x.launch < y.launch;
        if (x.cost != y.cost) return x.cost > y.cost;
        if (x.kind != y.kind) return x.kind < y.kind;
        return x.page < y.page;
    });
    long total = 0;
    int l = 0;  // launch boundaries filled so far: page_begin[0..l]
    *launches = 0;
    for (int j = 0; j < n; ++j) {
        const PagePlan &q = plans[j];
        const bz_page &p = pages[q.page];
        for (; l < q.launch; ++l) {
            hdr->page_begin[l + 1] = (uint32_t)j;
            hdr->item_begin[l + 1] = (uint32_t)total;
        }
        *launches |= 1u << q.launch;
        BatchPage &e = bp[j];
        std::memset(&e, 0, sizeof(e));
        e.a = page_args(descs[q.page], p.win, p.k, p.R, p.rule, q.tw, q.th, blk_group(q.launch / kClasses));
        e.item0 = (int)total;
        e.kind = q.kind;
        total += e.a.n_tiles;
        if (total >= (1L << 31)) return BZ_ERR_SHAPE;
    }
    for (; l < kLaunches; ++l) {
        hdr->page_begin[l + 1] = (uint32_t)n;
        hdr->item_begin[l + 1] = (uint32_t)total;
    }
    hdr->n_pages = (uint32_t)n;
    hdr->n_items = (uint32_t)total;
    *items = (int)total;
    return BZ_OK;
}

// Enqueue the copy of the first `bytes` of the table, the counter reset and
// the persistent kernel of each launch key in `launches`, in key order (each
// starts when the one before has finished), with its class's LDS share per
// workgroup.
int record(const bz_batch *b, const RunBuffers &r, size_t bytes, uint32_t launches, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(r.dev_table, r.host_table, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(e);
    hipLaunchKernelGGL(bz_counter_reset, dim3(1), dim3(64), 0, st, r.counter);
    const BatchHeader *hdr = (const BatchHeader *)r.dev_table;
    const BatchPage *pg = (const BatchPage *)(hdr + 1);
    for (int l = 0; l < kLaunches; ++l) {
        if (!(launches & (1u << l))) continue;
        const int g = l / kClasses, c = l % kClasses;
        hipLaunchKernelGGL(kBatchKernels[g][budget_of(c)], dim3((unsigned)b->grid[l]), dim3(kThreads),
                           (unsigned)class_lds(c), st, hdr, pg, r.counter, l);
    }
    e = hipGetLastError();
    return e == hipSuccess ? BZ_OK : fail(e);
}

}  // namespace

extern "C" {

int binarize_batch_create(int max_pages, int lds_cap_bytes, bz_batch **out) {
    if (!out) return BZ_ERR_NULL;
    *out = nullptr;
    if (max_pages < 1 || max_pages > (1 << 20)) return BZ_ERR_SHAPE;
    // default: the share of two workgroups per CU
    if (lds_cap_bytes <= 0) lds_cap_bytes = class_lds(2);
    if (lds_cap_bytes < tile_lds_bytes(128, 1, 1, false) || lds_cap_bytes > class_lds(kClasses - 1))
        return BZ_ERR_TILE;
    bz_batch *b = new (std::nothrow) bz_batch();
    if (!b) return BZ_ERR_HIP;
    b->max_pages = max_pages;
    b->lds_cap = lds_cap_bytes;
    b->table_bytes = table_size(max_pages);
    hipError_t e = hipSuccess;
    for (int g = 0; g < kGroups; ++g)
        for (int v = 0; v < 2; ++v)
            (void)hipFuncSetAttribute((const void *)kBatchKernels[g][v], hipFuncAttributeMaxDynamicSharedMemorySize,
                                      kMaxLds - kStaticLds);
    (void)hipGetLastError();
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) {
        delete b;
        return fail(e);
    }
    for (int l = 0; l < kLaunches; ++l) {  // the grid that fills the GPU, per launch key
        const int g = l / kClasses, c = l % kClasses;
        int per_cu = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kBatchKernels[g][budget_of(c)], kThreads,
                                                              class_lds(c))) != hipSuccess) {
            delete b;
            return fail(e);
        }
        if (per_cu < 1) {
            delete b;
            return BZ_ERR_TILE;
        }
        b->grid[l] = cus * per_cu;
    }
    if ((e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
        binarize_batch_destroy(b);
        return fail(e);
    }
    for (RunBuffers &r : b->buf) {
        if ((e = hipHostMalloc(&r.host_table, b->table_bytes, hipHostMallocDefault)) != hipSuccess ||
            (e = hipMalloc(&r.dev_table, b->table_bytes)) != hipSuccess ||
            (e = hipMalloc((void **)&r.counter, kLaunches * sizeof(uint32_t))) != hipSuccess ||
            (e = hipEventCreateWithFlags(&r.done, hipEventDisableTiming)) != hipSuccess) {
            binarize_batch_destroy(b);
            return fail(e);
        }
        std::memset(r.host_table, 0, b->table_bytes);
    }
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
    RunBuffers &r = b->buf[b->cur];
    // these buffers may still be in use by the run before the previous one
    if (r.pending) {
        hipError_t e = hipEventSynchronize(r.done);
        if (e != hipSuccess) return fail(e);
        r.pending = false;
    }
    int items = 0;
    uint32_t launches = 0;
    int rc = plan(pages, n_pages, b->lds_cap, r.host_table, b->descs, b->spans, b->span_max, b->plans, &items,
                  &launches);
    if (rc) return rc;
    b->last_items = items;
    b->last_launches = launches;
    if (use_graph) {
        // the graph copies a table of graph_pages pages (a power of two, at
        // least 64, at most max_pages) and makes the launches the plan uses;
        // capture again when the batch needs another size or other launches
        int gp = 64;
        while (gp < n_pages) gp *= 2;
        if (gp > b->max_pages) gp = b->max_pages;
        if (r.exec && (r.graph_pages != gp || r.graph_launches != launches)) {
            (void)hipGraphExecDestroy(r.exec);
            (void)hipGraphDestroy(r.graph);
            r.exec = nullptr;
            r.graph = nullptr;
        }
        if (!r.exec) {
            hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return fail(e);
            rc = record(b, r, table_size(gp), launches, b->cap_stream);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(b->cap_stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(e);
            r.graph = g;
            if ((e = hipGraphInstantiate(&r.exec, g, nullptr, nullptr, 0)) != hipSuccess) return fail(e);
            r.graph_pages = gp;
            r.graph_launches = launches;
        }
        hipError_t e = hipGraphLaunch(r.exec, st);
        if (e != hipSuccess) return fail(e);
    } else {
        rc = record(b, r, table_size(n_pages), launches, st);
        if (rc) return rc;
    }
    hipError_t e = hipEventRecord(r.done, st);
    if (e != hipSuccess) return fail(e);
    r.pending = true;
    b->cur ^= 1;
    return BZ_OK;
}

int binarize_batch_info(const bz_batch *b, int *grid, int *lds_cap, int *last_items) {
    if (!b) return BZ_ERR_NULL;
    if (grid) *grid = b->grid[0];  // 256-column ring pages at four workgroups per CU
    if (lds_cap) *lds_cap = b->lds_cap;
    if (last_items) *last_items = b->last_items;
    return BZ_OK;
}

}  // extern "C"

namespace {

// The batch object behind the one-call binarize_batch, one per device: its
// two sets of run buffers let a call wait on the host only for the run
// before the previous one.  It grows to the largest call seen and lives
// until the process ends.
struct OneCallPool {
    std::mutex mu;
    bz_batch *obj = nullptr;
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
    bz_batch *&b = pool.obj;
    if (!b || b->max_pages < n_pages) {
        if (b) binarize_batch_destroy(b);  // waits for its last runs
        b = nullptr;
        int cap = 64;
        while (cap < n_pages) cap *= 2;
        const int rc = binarize_batch_create(cap, 0, &b);
        if (rc) {
            b = nullptr;
            return rc;
        }
    }
    return binarize_batch_run(b, pages, n_pages, 0, stream);
}

void binarize_batch_destroy(bz_batch *b) {
    if (!b) return;
    for (RunBuffers &r : b->buf) {
        if (r.pending) (void)hipEventSynchronize(r.done);
        if (r.exec) (void)hipGraphExecDestroy(r.exec);
        if (r.graph) (void)hipGraphDestroy(r.graph);
        if (r.done) (void)hipEventDestroy(r.done);
        if (r.counter) (void)hipFree(r.counter);
        if (r.dev_table) (void)hipFree(r.dev_table);
        if (r.host_table) (void)hipHostFree(r.host_table);
    }
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete[] b->spans;
    delete[] b->span_max;
    delete[] b->descs;
    delete[] b->plans;
    delete b;
}


}  // extern "C"
