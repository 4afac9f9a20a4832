// C ABI of the mknn library: contexts, device memory, argument checks and
// the enqueueing of the index build and the query kernels.  Declarations
// and the contract of every entry point are in include/mknn.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mknn.h"
#include "mknn_internal.hpp"
#include "query.hpp"

using namespace mknn;

struct mknn_ctx {
    mknn_config cfg{};
    int th = 0, L = 16, k_max = 1;
    int sweep = MKNN_SWEEP_AUTO;  // sweep flavour (mknn_schedule)
    bool group_k = false;         // variable k answered per k class
    int tile_queries = 0;         // lane flavour queries per wavefront (0: automatic)
    int compute_units = 256;      // of the context's device (automatic query tiles)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool dead = false;         // sticky device error
    std::string err;

    bool loaded = false, ticked = false, queried = false;
    bool inv_ready = false;    // ix.inv matches the current index
    int64_t n = 0, nq = 0, entries = 0;
    int32_t k_uniform = 0;
    bool var_k = false;
    int64_t ticks = 0;

    bool built = false;        // a full build exists (refit ticks may follow)
    int64_t built_n = 0;       // object count of that build
    int64_t refits = 0;        // refit ticks since it
    float *x = nullptr, *y = nullptr;           // copies of host-supplied positions
    const float *src_x = nullptr, *src_y = nullptr;  // positions the next build reads
    uint32_t build_epoch = 0, query_epoch = 0;  // tags of the device flags
    IndexBuffers ix{};
    SortBuffers qs{};          // query-order sort (subset queries)
    Workspace qws{};           // its workspace (and the offsets scan's)
    ScanSpace qscan{};
    // Subset queries ordered through a table of issuer positions (when they
    // are many; see order_by_marks): the table clears itself as it is read.
    uint32_t *qowner = nullptr;   // query owning each sorted position, or kNoOwner
    uint32_t *qpopc = nullptr, *qbase = nullptr;  // per 64 positions
    uint32_t *qorder = nullptr;   // [0] repeats counted, [1] repeats, [2] positions
    int32_t *issuers = nullptr, *ks = nullptr;  // staging of host query arrays
    float *qcx = nullptr, *qcy = nullptr;       // staging of host free centres
    QPoint *qpts = nullptr;                     // free centres in processing order
    uint32_t *class_bounds = nullptr;           // per-k-class query ranges [8]
    uint32_t *kcount = nullptr, *kscan = nullptr, *ktotal = nullptr;
    int64_t *offsets = nullptr;
    int32_t *out_ids = nullptr;
    float *out_d2 = nullptr;
    int32_t *out_cnt = nullptr;
    unsigned long long *counters = nullptr;  // query-kernel work counters [5]

    // Timing (MKNN_FLAG_TIMING): one ring slot of events per build and per
    // query, [0] build start, [1] build end, [2] query start, [3] start of
    // the leaf-sweep kernel, [4] query end.  [3] is not recorded when no
    // preparation work precedes the kernel (then [2] stands for it).
    static constexpr int kRing = 256;
    static constexpr int kMarks = 5;
    hipEvent_t ring[kRing][kMarks]{};
    bool main_is_start[kRing]{};
    bool have_ring = false;
    int64_t builds_timed = 0, queries_timed = 0;  // since the last reset
    int64_t build_slot = 0, query_slot = 0;       // calls ever recorded
    std::vector<void *> allocs;
};

namespace {

int fail(mknn_ctx *c, int code, const char *fmt, const char *detail = "")
{
    if (c) {
        char buf[512];
        snprintf(buf, sizeof buf, fmt, detail);
        c->err = buf;
        if (code == MKNN_E_DEVICE) c->dead = true;
    }
    return code;
}

int hip_fail(mknn_ctx *c, hipError_t e, const char *where)
{
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    return fail(c, MKNN_E_DEVICE, "%s", buf);
}

#define HIP_OR_FAIL(ctx, call)                                   \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
    } while (0)

// Makes a context's device current for one call and gives the caller its
// own current device back when the call returns, on every path.
class DeviceScope {
  public:
    explicit DeviceScope(int dev)
    {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) cur = -1;
        if (cur == dev) return;  // already current: nothing to restore
        err = hipSetDevice(dev);
        if (err == hipSuccess) prev_ = cur;
    }
    ~DeviceScope()
    {
        if (prev_ >= 0) (void)hipSetDevice(prev_);
    }
    DeviceScope(const DeviceScope &) = delete;
    DeviceScope &operator=(const DeviceScope &) = delete;
    hipError_t err = hipSuccess;

  private:
    int prev_ = -1;
};

template <typename T>
int dalloc(mknn_ctx *c, T **p, int64_t count)
{
    if (count < 1) count = 1;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, (size_t)count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, MKNN_E_NOMEM, "device allocation of %s failed",
                    std::to_string((size_t)count * sizeof(T)).c_str());
    }
    c->allocs.push_back(q);
    *p = (T *)q;
    return MKNN_OK;
}

int check_launch(mknn_ctx *c, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, what);
    return MKNN_OK;
}

// Selection-list class of a k: lists of 8 << class keys.
int class_slot(int k)
{
    return k <= 8 ? 0 : k <= 16 ? 1 : k <= 32 ? 2 : k <= 64 ? 3 : 4;
}

// Bits that hold a sorted position below n.
int pos_bits(int64_t n)
{
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < n) ++b;
    return b;
}

int bits_for(int64_t n)
{
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) < n) ++b;
    return ((b + kRadixBits - 1) / kRadixBits) * kRadixBits;
}

__global__ void k_reset_counters(IndexCounters *ctr) { *ctr = IndexCounters{}; }

// Epochs run 1 .. 2^24-1 (the deepest-level word keeps 8 bits for the level).
uint32_t next_epoch(uint32_t e) { return e >= (1u << 24) - 1 ? 1u : e + 1u; }

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

constexpr uint32_t kNoOwner = 0xffffffffu;

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t n, uint32_t v)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = v;
}

// Subset queries in ascending order of their issuers' sorted positions
// without a radix sort, for when the queries are many: each query writes
// its index at its issuer's position of an owner table (one of several
// queries of a repeated issuer keeps the position; a second pass lists the
// others), the marked positions of every run of 64 are counted and the
// counts scanned, and a wavefront over 64 positions ranks its marked ones
// by a ballot.  Plain stores, then plain loads: swapping the index in with
// an atomic exchange that returns the displaced query took 77 us for 2M
// queries against 28 + 28 us for the two passes.  Queries of repeated issuers follow all others, in any
// order.  The order only decides which queries share a wavefront; results
// do not depend on it.  The table is back to kNoOwner after each call.
__global__ void k_order_mark(const uint32_t *__restrict__ pos, uint32_t nq,
                             uint32_t *__restrict__ owner)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) owner[pos[q]] = q;
}

__global__ void k_order_repeats(const uint32_t *__restrict__ pos, uint32_t nq,
                                const uint32_t *__restrict__ owner,
                                uint32_t *__restrict__ repeats, uint32_t *__restrict__ words)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq && owner[pos[q]] != q) repeats[atomicAdd(&words[0], 1u)] = q;
}

// Marked positions per run of 64 (one wavefront each); the repeat count
// moves to words[1] and its counter restarts at zero for the next call.
__global__ __launch_bounds__(256) void k_order_counts(const uint32_t *__restrict__ owner,
                                                      uint32_t n, uint32_t *__restrict__ popc,
                                                      uint32_t *__restrict__ words)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) {
        words[1] = words[0];
        words[0] = 0u;
    }
    const bool marked = p < n && owner[p] != kNoOwner;
    const unsigned long long m = __ballot(marked);
    if ((threadIdx.x & (kWave - 1)) == 0 && p < n) popc[p / kWave] = (uint32_t)__popcll(m);
}

// Every marked position takes rank base[run] + (marked positions before it
// in its run) and is reset to kNoOwner; the repeats follow the words[2]
// marked positions.
__global__ __launch_bounds__(256) void k_order_emit(
    uint32_t *__restrict__ owner, uint32_t n, const uint32_t *__restrict__ base,
    const uint32_t *__restrict__ repeats, const uint32_t *__restrict__ pos,
    const uint32_t *__restrict__ words, uint32_t *__restrict__ out_pos,
    uint32_t *__restrict__ out_row)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t o = p < n ? owner[p] : kNoOwner;
    const bool marked = o != kNoOwner;
    const unsigned long long m = __ballot(marked);
    if (marked) {
        const uint32_t lane = threadIdx.x & (kWave - 1);
        const uint32_t r = base[p / kWave] + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        out_pos[r] = p;
        out_row[r] = o;
        owner[p] = kNoOwner;
    }
    const uint32_t marked_total = words[2], nrep = words[1];
    for (uint32_t j = p; j < nrep; j += gridDim.x * blockDim.x) {
        const uint32_t q = repeats[j];
        out_pos[marked_total + j] = pos[q];
        out_row[marked_total + j] = q;
    }
}

// The owner-table order pays when the queries are many against the
// objects (its passes read the table once per 4 bytes of it); its scan then
// also fits the query workspace's second scan space (one item per 64
// positions, at most nq + 1 of them).
bool order_by_marks(int64_t n, int64_t nq) { return n > 0 && nq > 0 && (n + 63) / 64 <= nq + 1; }

// pos: sorted position of each query's issuer (nq, each below c->n); the
// ordered positions and query indexes go to out_pos / out_row; `repeats`
// (nq) is scratch.
void launch_marks_order(mknn_ctx *c, const uint32_t *pos, uint32_t nq, uint32_t *repeats,
                        const ScanSpace &sp, uint32_t *out_pos, uint32_t *out_row)
{
    const int T = 256;
    const uint32_t n = (uint32_t)c->n;
    const uint32_t runs = (n + kWave - 1) / kWave;
    const uint32_t gq = (nq + T - 1) / T, gn = (n + T - 1) / T;
    k_order_mark<<<gq, T, 0, c->stream>>>(pos, nq, c->qowner);
    k_order_repeats<<<gq, T, 0, c->stream>>>(pos, nq, c->qowner, repeats, c->qorder);
    k_order_counts<<<gn, T, 0, c->stream>>>(c->qowner, n, c->qpopc, c->qorder);
    launch_exclusive_scan(c->qpopc, c->qbase, runs, sp, c->qorder + 2, c->stream);
    k_order_emit<<<gn, T, 0, c->stream>>>(c->qowner, n, c->qbase, repeats, pos, c->qorder,
                                          out_pos, out_row);
}

int read_counters(mknn_ctx *c, IndexCounters *h)
{
    HIP_OR_FAIL(c, hipMemcpyAsync(h, c->ix.ctr, sizeof *h, hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return MKNN_OK;
}

// Error words are sticky: a kernel that meets bad input raises its word to
// a nonzero value, and the word keeps it -- whichever launch, eager or
// replayed from a graph, raised it -- until the host has read and reported
// it here; then every error word is cleared (by a kernel, so that nothing
// here records a memset) and the first error found is returned.
__global__ void k_clear_flags(IndexCounters *ctr)
{
    ctr->bad_coord = 0;
    ctr->bad_nodes = 0;
    ctr->bad_issuer = 0;
    ctr->bad_k = 0;
    ctr->bad_sync_build = 0;
    ctr->bad_sync_query = 0;
    ctr->bad_centre = 0;
}

int check_deferred(mknn_ctx *c)
{
    if (!c->ticked) return MKNN_OK;
    IndexCounters h{};
    int rc = read_counters(c, &h);
    if (rc) return rc;
    if (!(h.bad_coord | h.bad_nodes | h.bad_sync_build | h.bad_sync_query | h.bad_issuer |
          h.bad_k | h.bad_centre))
        return MKNN_OK;
    k_clear_flags<<<1, 1, 0, c->stream>>>(c->ix.ctr);
    rc = check_launch(c, "clear error words");
    if (!rc) {
        const hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = hip_fail(c, e, "hipStreamSynchronize");
    }
    if (rc) return rc;
    if (h.bad_nodes) return fail(c, MKNN_E_DEVICE, "node table capacity exceeded%s");
    if (h.bad_sync_build) return fail(c, MKNN_E_DEVICE, "index build: a look-back wait gave up%s");
    if (h.bad_sync_query)
        return fail(c, MKNN_E_DEVICE, "query indexing: a look-back wait gave up%s");
    if (h.bad_coord)
        return fail(c, MKNN_E_RANGE, "a device coordinate is not finite or outside [0,1)%s");
    if (h.bad_issuer) return fail(c, MKNN_E_INVAL, "a device issuer is outside [0,n)%s");
    if (h.bad_k) return fail(c, MKNN_E_INVAL, "a device k is outside [1,k_max]%s");
    return fail(c, MKNN_E_RANGE, "a device query centre is not finite or outside [0,1)%s");
}

bool valid_where(int32_t w) { return w == MKNN_HOST || w == MKNN_DEVICE; }

// Every device buffer of a context and its element count, in one list:
// mknn_create allocates from it and mknn_footprint sums it.
template <class F>
void for_each_buffer(mknn_ctx *c, F &&f)
{
    const int64_t N = c->cfg.n_max, Q = c->cfg.q_max;
    const int64_t node_cap = c->ix.node_cap;
    f(c->x, N);
    f(c->y, N);
    f(c->ix.sort.keys[0], N);
    f(c->ix.sort.keys[1], N);
    f(c->ix.sort.vals[0], N);
    f(c->ix.sort.vals[1], N);
    f(c->ix.ws.base, c->ix.ws.cap_words);
    f(c->qws.base, c->qws.cap_words);
    f(c->ix.xy, N);
    f(c->ix.anchor, N);
    f(c->ix.pts, N);
    f(c->ix.inv, N);
    f(c->ix.leaf_of, N);
    f(c->ix.leaf_begin, N);
    f(c->ix.leaf_end, N);
    f(c->ix.leaf_level, N);
    f(c->ix.leaf_code, N);
    f(c->ix.cnt_f, N);
    f(c->ix.cnt_r, N);
    f(c->ix.leaf_node_f, N);
    f(c->ix.leaf_node_r, N);
    f(c->ix.fwd, node_cap);
    f(c->ix.rev, node_cap);
    f(c->ix.ctr, 1);
    f(c->qowner, N);
    f(c->qpopc, N / 64 + 2);
    f(c->qbase, N / 64 + 2);
    f(c->qorder, 4);
    f(c->qs.keys[0], Q);
    f(c->qs.keys[1], Q);
    f(c->qs.vals[0], Q);
    f(c->qs.vals[1], Q);
    f(c->issuers, Q);
    f(c->ks, Q);
    f(c->qcx, Q);
    f(c->qcy, Q);
    f(c->qpts, Q);
    f(c->class_bounds, 8);
    f(c->kcount, Q);
    f(c->kscan, Q);
    f(c->ktotal, 1);
    f(c->offsets, Q + 1);
    f(c->out_ids, Q * c->k_max);
    f(c->out_d2, Q * c->k_max);
    f(c->out_cnt, Q);
    f(c->counters, 8);
}

void size_context(mknn_ctx *c)
{
    const int64_t N = c->cfg.n_max, Q = c->cfg.q_max;
    c->ix.n_cap = N;
    c->ix.node_cap = node_capacity(N, c->th, c->L);
    c->ix.ws.cap_words = workspace_words(N);
    c->qws.cap_words = workspace_words(Q + 1);
}

bool valid_config(const mknn_config *cfg)
{
    return cfg->n_max >= 1 && cfg->n_max < ((int64_t)1 << 31) && cfg->q_max >= 1 &&
           cfg->q_max < ((int64_t)1 << 31) && cfg->k_max >= 1 && cfg->k_max <= MKNN_K_LIMIT &&
           cfg->max_level >= 0 && cfg->max_level <= kCodeLevels && cfg->leaf_capacity >= 0 &&
           cfg->k_hint >= 0 && cfg->k_hint <= MKNN_K_LIMIT;
}

void configure(mknn_ctx *c, const mknn_config *cfg)
{
    c->cfg = *cfg;
    c->L = cfg->max_level ? cfg->max_level : kCodeLevels;
    c->k_max = cfg->k_max;
    const int kh = cfg->k_hint ? cfg->k_hint : cfg->k_max;
    c->th = cfg->leaf_capacity ? cfg->leaf_capacity : mknn_default_leaf_capacity(kh);
    c->sweep = (cfg->flags & MKNN_FLAG_SWEEP_WAVE) ? MKNN_SWEEP_WAVE : MKNN_SWEEP_AUTO;
    c->group_k = (cfg->flags & MKNN_FLAG_GROUP_K) != 0;
    size_context(c);
}


// Record timing mark i (0..4, as mknn_ctx::ring) in the current build's or
// query's ring slot.
int mark(mknn_ctx *c, int i)
{
    if (!((c->cfg.flags & MKNN_FLAG_TIMING) && c->have_ring)) return MKNN_OK;
    const int64_t slot = (i < 2 ? c->build_slot : c->query_slot) % mknn_ctx::kRing;
    HIP_OR_FAIL(c, hipEventRecord(c->ring[slot][i], c->stream));
    return MKNN_OK;
}

// Start of the leaf-sweep kernel: a mark of its own only if preparation
// work was enqueued since the query started.
int mark_main(mknn_ctx *c, bool prepared)
{
    if (!((c->cfg.flags & MKNN_FLAG_TIMING) && c->have_ring)) return MKNN_OK;
    c->main_is_start[c->query_slot % mknn_ctx::kRing] = !prepared;
    return prepared ? mark(c, 3) : MKNN_OK;
}

// The flavour a query runs with: the schedule's, except that the lane
// flavour hands lists above its 128 keys to the one-query-per-wavefront
// flavour.  AUTO takes one query per lane up to k = 32 and a group of lanes
// per query above: from k = 64 a lane-private list leaves at most two
// wavefronts per SIMD (query kernel at the 64-key class on network_4m:
// 1.06 ms grouped against 1.26 ms; k = 128 on mixed_16m: 24 ms against
// 45 ms), while at k = 32 one lane per query wins (0.37 against 0.45 ms on
// clustered_1m).
constexpr int kAutoLaneMaxK = 32;

int sweep_flavour(const mknn_ctx *c, int kmax_call)
{
    if (c->sweep == MKNN_SWEEP_GROUP || c->sweep == MKNN_SWEEP_WAVE) return c->sweep;
    if (c->sweep == MKNN_SWEEP_AUTO)
        return kmax_call > kAutoLaneMaxK ? MKNN_SWEEP_GROUP : MKNN_SWEEP_LANE;
    return kmax_call > 128 ? MKNN_SWEEP_WAVE : MKNN_SWEEP_LANE;
}

bool use_wave_sweep(const mknn_ctx *c, int kmax_call)
{
    return sweep_flavour(c, kmax_call) == MKNN_SWEEP_WAVE;
}

// One k class of queries (or all of them) with list size kclass_k.
void launch_class(const mknn_ctx *c, const QueryArgs &qa, int kclass_k, int flavour)
{
    if (flavour == MKNN_SWEEP_WAVE) launch_knn_wave(qa, k_class_wave(kclass_k), c->stream);
    else if (flavour == MKNN_SWEEP_GROUP) launch_knn_group(qa, k_class_group(kclass_k), c->stream);
    else launch_knn(qa, k_class(kclass_k), c->stream);
}

void launch_sweep(const mknn_ctx *c, const QueryArgs &qa, int kmax_call)
{
    launch_class(c, qa, kmax_call, sweep_flavour(c, kmax_call));
}

}  // namespace

extern "C" {

const char *mknn_status_str(int s)
{
    switch (s) {
    case MKNN_OK: return "MKNN_OK";
    case MKNN_E_INVAL: return "MKNN_E_INVAL";
    case MKNN_E_RANGE: return "MKNN_E_RANGE";
    case MKNN_E_STATE: return "MKNN_E_STATE";
    case MKNN_E_CAPACITY: return "MKNN_E_CAPACITY";
    case MKNN_E_NOMEM: return "MKNN_E_NOMEM";
    case MKNN_E_DEVICE: return "MKNN_E_DEVICE";
    default: return "MKNN_E_UNKNOWN";
    }
}

int32_t mknn_default_leaf_capacity(int32_t k)
{
    // Paper's setting (Sec. 6): 192 for k < 32, 12k for 32..128, 2048 above.
    if (k < 32) return 192;
    if (k <= 128) return 12 * k;
    return 2048;
}

const char *mknn_last_error(const mknn_ctx *c) { return c ? c->err.c_str() : "null context"; }

int mknn_destroy(mknn_ctx *c)
{
    if (!c) return MKNN_OK;
    {
        DeviceScope dev(c->cfg.device);
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        for (void *p : c->allocs) (void)hipFree(p);
        for (auto &slot : c->ring)
            for (auto &e : slot)
                if (e) (void)hipEventDestroy(e);
        if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    }
    delete c;
    return MKNN_OK;
}

int mknn_footprint(const mknn_config *cfg, int64_t *bytes)
{
    if (!cfg || !bytes) return MKNN_E_INVAL;
    if (!valid_config(cfg)) return MKNN_E_INVAL;
    mknn_ctx tmp;
    configure(&tmp, cfg);
    int64_t total = 0;
    for_each_buffer(&tmp, [&](auto &p, int64_t count) {
        if (count < 1) count = 1;
        // The runtime maps buffers of 2 MiB or more in whole 2 MiB pages;
        // smaller ones are counted in 256-byte units.
        const size_t b = (size_t)count * sizeof(*p);
        const size_t unit = b >= ((size_t)2 << 20) ? ((size_t)2 << 20) : 256;
        total += (int64_t)((b + unit - 1) / unit * unit);
    });
    *bytes = total;
    return MKNN_OK;
}

int mknn_create(const mknn_config *cfg, mknn_ctx **out)
{
    if (!out) return MKNN_E_INVAL;
    *out = nullptr;
    if (!cfg) return MKNN_E_INVAL;
    if (!valid_config(cfg)) return MKNN_E_INVAL;
    if ((double)cfg->q_max * cfg->k_max >= 4294967295.0) return MKNN_E_CAPACITY;

    mknn_ctx *c = new (std::nothrow) mknn_ctx;
    if (!c) return MKNN_E_NOMEM;
    configure(c, cfg);

    DeviceScope dev(cfg->device);
    if (dev.err != hipSuccess) {
        delete c;
        return MKNN_E_DEVICE;
    }
    int rc = MKNN_OK;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg->device) ==
                hipSuccess && cus > 0)
            c->compute_units = cus;
    }
    if (cfg->stream) {
        c->stream = (hipStream_t)cfg->stream;
    } else {
        const hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            return MKNN_E_DEVICE;
        }
        c->own_stream = true;
    }
    for_each_buffer(c, [&](auto &p, int64_t count) {
        if (!rc) rc = dalloc(c, &p, count);
    });
    if (!rc) {
        if (cfg->flags & MKNN_FLAG_TIMING) {
            // Timing only: no system-scope fence when an event is recorded
            // (its cache writeback would cost the following kernels time).
            c->have_ring = true;
            for (auto &slot : c->ring)
                for (auto &ev : slot)
                    if (hipEventCreateWithFlags(&ev, hipEventDisableSystemFence) != hipSuccess)
                        c->have_ring = false;
        }
        k_reset_counters<<<1, 1, 0, c->stream>>>(c->ix.ctr);
        k_zero_u64<<<1, 8, 0, c->stream>>>(c->counters, 8);
        {
            const int64_t N = c->cfg.n_max;
            const uint32_t g = (uint32_t)std::min<int64_t>((N + 255) / 256, 2048);
            k_fill_u32<<<g, 256, 0, c->stream>>>(c->qowner, (uint32_t)N, kNoOwner);
        }
        k_zero_u64<<<1, 2, 0, c->stream>>>((unsigned long long *)c->qorder, 2);
        rc = check_launch(c, "reset counters");
    }
    if (rc) {
        mknn_destroy(c);
        return rc;
    }
    *out = c;
    return MKNN_OK;
}

int mknn_load_positions(mknn_ctx *c, const float *x, const float *y, int64_t n, int32_t where)
{
    if (!c) return MKNN_E_INVAL;
    if (c->dead) return fail(c, MKNN_E_DEVICE, "context has a sticky device error%s");
    if (!valid_where(where)) return fail(c, MKNN_E_INVAL, "bad `where`%s");
    if (n < 0 || (n > 0 && (!x || !y))) return fail(c, MKNN_E_INVAL, "bad positions%s");
    if (n > c->cfg.n_max) return fail(c, MKNN_E_CAPACITY, "n exceeds n_max%s");
    if (where == MKNN_HOST) {
        for (int64_t i = 0; i < n; ++i) {
            const float a = x[i], b = y[i];
            if (!(a >= 0.0f && a < 1.0f && b >= 0.0f && b < 1.0f))
                return fail(c, MKNN_E_RANGE, "object %s: coordinate not finite or outside [0,1)",
                            std::to_string(i).c_str());
        }
    }
    DeviceScope dev(c->cfg.device);
    HIP_OR_FAIL(c, dev.err);
    if (where == MKNN_HOST) {
        if (n > 0) {
            HIP_OR_FAIL(c, hipMemcpyAsync(c->x, x, (size_t)n * sizeof(float),
                                          hipMemcpyHostToDevice, c->stream));
            HIP_OR_FAIL(c, hipMemcpyAsync(c->y, y, (size_t)n * sizeof(float),
                                          hipMemcpyHostToDevice, c->stream));
            HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
        }
        c->src_x = c->x;
        c->src_y = c->y;
    } else {
        // Read in place by the next index build.
        c->src_x = x;
        c->src_y = y;
    }
    c->n = n;
    c->loaded = true;
    c->ticked = false;
    c->queried = false;
    c->ticks = 0;
    return MKNN_OK;
}

int mknn_advance_tick(mknn_ctx *c)
{
    if (!c) return MKNN_E_INVAL;
    if (c->dead) return fail(c, MKNN_E_DEVICE, "context has a sticky device error%s");
    if (!c->loaded) return fail(c, MKNN_E_STATE, "advance_tick before load_positions%s");
    DeviceScope dev(c->cfg.device);
    HIP_OR_FAIL(c, dev.err);
    int rc = mark(c, 0);
    if (rc) return rc;
    c->build_epoch = next_epoch(c->build_epoch);
    launch_build_index(c->ix, c->src_x, c->src_y, c->n, c->th, c->L, c->build_epoch, c->stream);
    rc = check_launch(c, "index build");
    if (!rc) rc = mark(c, 1);
    if (rc) return rc;
    ++c->build_slot;
    ++c->builds_timed;
    c->ticked = true;
    c->queried = false;
    c->inv_ready = false;
    c->built = true;
    c->built_n = c->n;
    c->refits = 0;
    ++c->ticks;
    return MKNN_OK;
}

int mknn_refit_tick(mknn_ctx *c)
{
    if (!c) return MKNN_E_INVAL;
    if (c->dead) return fail(c, MKNN_E_DEVICE, "context has a sticky device error%s");
    if (!c->loaded) return fail(c, MKNN_E_STATE, "refit_tick before load_positions%s");
    if (!c->built) return fail(c, MKNN_E_STATE, "refit_tick needs a full build first%s");
    if (c->n != c->built_n)
        return fail(c, MKNN_E_STATE, "refit_tick needs the object count of the last build%s");
    DeviceScope dev(c->cfg.device);
    HIP_OR_FAIL(c, dev.err);
    int rc = mark(c, 0);
    if (rc) return rc;
    c->build_epoch = next_epoch(c->build_epoch);
    launch_refit(c->ix, c->src_x, c->src_y, c->n, c->build_epoch, c->stream);
    rc = check_launch(c, "refit");
    if (!rc) rc = mark(c, 1);
    if (rc) return rc;
    ++c->build_slot;
    ++c->builds_timed;
    c->ticked = true;
    c->queried = false;
    ++c->refits;
    ++c->ticks;
    return MKNN_OK;
}

namespace {

// Query-kernel arguments shared by both kinds of query.
QueryArgs base_query_args(mknn_ctx *c, int64_t nq, const int32_t *ks, int32_t k_uniform)
{
    QueryArgs qa{};
    qa.pts = c->ix.pts;
    qa.n = (uint32_t)c->n;
    qa.fwd = c->ix.fwd;
    qa.rev = c->ix.rev;
    qa.leaf_of = c->ix.leaf_of;
    qa.leaf_begin = c->ix.leaf_begin;
    qa.leaf_end = c->ix.leaf_end;
    qa.leaf_node_f = c->ix.leaf_node_f;
    qa.leaf_node_r = c->ix.leaf_node_r;
    qa.ctr = c->ix.ctr;
    qa.node_cap = (int32_t)c->ix.node_cap;
    qa.nq = (uint32_t)nq;
    qa.k_uniform = ks ? 0 : k_uniform;
    qa.out_ids = c->out_ids;
    qa.out_d2 = c->out_d2;
    qa.out_cnt = c->out_cnt;
    qa.counters = (c->cfg.flags & MKNN_FLAG_COUNTERS) ? c->counters : nullptr;
    qa.build_epoch = c->build_epoch;
    qa.pos_mask = 0xffffffffu;
    qa.class_bounds = nullptr;
    qa.klass = 0;
    qa.tile_queries = (uint32_t)c->tile_queries;
    qa.compute_units = (uint32_t)c->compute_units;
    return qa;
}

// Host-side description of the results of the query just enqueued.
void record_query(mknn_ctx *c, int64_t nq, const int32_t *ks, int32_t k_uniform, int32_t where)
{
    ++c->query_slot;
    ++c->queries_timed;
    c->queried = true;
    c->nq = nq;
    c->var_k = ks != nullptr;
    c->k_uniform = ks ? 0 : k_uniform;
    if (!ks) {
        c->entries = nq * (int64_t)k_uniform;
    } else if (where == MKNN_HOST) {
        int64_t s = 0;
        for (int64_t i = 0; i < nq; ++i) s += ks[i];
        c->entries = s;
    } else {
        c->entries = -1;  // known after synchronisation
    }
}

// Host-side checks of per-query k; *kmax gets the largest.
int check_host_ks(mknn_ctx *c, const int32_t *ks, int64_t nq, int *kmax)
{
    int kmx = 1;
    for (int64_t i = 0; i < nq; ++i) {
        if (ks[i] < 1 || ks[i] > c->k_max)
            return fail(c, MKNN_E_INVAL, "k of query %s outside [1,k_max]",
                        std::to_string(i).c_str());
        if (ks[i] > kmx) kmx = ks[i];
    }
    *kmax = kmx;
    return MKNN_OK;
}

}  // namespace

int mknn_query_points(mknn_ctx *c, const float *qx, const float *qy, const int32_t *exclude,
                      const int32_t *ks, int64_t nq, int32_t k_uniform, int32_t where)
{
    if (!c) return MKNN_E_INVAL;
    if (c->dead) return fail(c, MKNN_E_DEVICE, "context has a sticky device error%s");
    if (!valid_where(where)) return fail(c, MKNN_E_INVAL, "bad `where`%s");
    if (!c->ticked) return fail(c, MKNN_E_STATE, "query before advance_tick%s");
    if (nq < 0) return fail(c, MKNN_E_INVAL, "nq < 0%s");
    if (nq > c->cfg.q_max) return fail(c, MKNN_E_CAPACITY, "nq exceeds q_max%s");
    if (nq > 0 && (!qx || !qy)) return fail(c, MKNN_E_INVAL, "qx and qy are required%s");
    if (c->n == 0 && nq > 0) return fail(c, MKNN_E_INVAL, "queries need at least one object%s");
    if (!ks && (k_uniform < 1 || k_uniform > c->k_max))
        return fail(c, MKNN_E_INVAL, "k outside [1, k_max]%s");
    int kmax_call = ks ? c->k_max : k_uniform;
    if (where == MKNN_HOST) {
        for (int64_t i = 0; i < nq; ++i) {
            if (!(qx[i] >= 0.0f && qx[i] < 1.0f && qy[i] >= 0.0f && qy[i] < 1.0f))
                return fail(c, MKNN_E_RANGE, "query centre %s is not finite or outside [0,1)",
                            std::to_string(i).c_str());
            if (exclude && (exclude[i] < -1 || exclude[i] >= c->n))
                return fail(c, MKNN_E_INVAL, "exclude of query %s is not -1 or an object id",
                            std::to_string(i).c_str());
        }
        if (ks) {
            int rc = check_host_ks(c, ks, nq, &kmax_call);
            if (rc) return rc;
        }
    }
    DeviceScope dev(c->cfg.device);
    HIP_OR_FAIL(c, dev.err);
    const float *d_qx = qx, *d_qy = qy;
    const int32_t *d_ex = exclude, *d_ks = ks;
    if (where == MKNN_HOST && nq > 0) {
        HIP_OR_FAIL(c, hipMemcpyAsync(c->qcx, qx, (size_t)nq * 4, hipMemcpyHostToDevice,
                                      c->stream));
        HIP_OR_FAIL(c, hipMemcpyAsync(c->qcy, qy, (size_t)nq * 4, hipMemcpyHostToDevice,
                                      c->stream));
        d_qx = c->qcx;
        d_qy = c->qcy;
        if (exclude) {
            HIP_OR_FAIL(c, hipMemcpyAsync(c->issuers, exclude, (size_t)nq * 4,
                                          hipMemcpyHostToDevice, c->stream));
            d_ex = c->issuers;
        }
        if (ks) {
            HIP_OR_FAIL(c, hipMemcpyAsync(c->ks, ks, (size_t)nq * 4, hipMemcpyHostToDevice,
                                          c->stream));
            d_ks = c->ks;
        }
        // Host arrays are read before the call returns: the caller may
        // reuse them at once.
        HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    }
    int rc = mark(c, 2);
    if (rc) return rc;
    c->query_epoch = next_epoch(c->query_epoch);

    QueryArgs qa = base_query_args(c, nq, ks, k_uniform);
    if (nq > 0) {
        const int64_t words = carve_workspace(c->qws, nq + 1, &c->qs, &c->qscan, 1,
                                              &c->ix.ctr->bad_sync_query, c->query_epoch);
        PointPrep p{};
        p.qx = d_qx;
        p.qy = d_qy;
        p.exclude = d_ex;
        p.ks = d_ks;
        p.nq = (uint32_t)nq;
        p.n = (uint32_t)c->n;
        p.k_max = c->k_max;
        p.sort = c->qs;
        p.kcount = c->kcount;
        p.ctr = c->ix.ctr;
        p.ws = c->qws.base;
        p.ws_words = words;
        p.epoch = c->query_epoch;
        launch_point_prep(p, c->stream);
        const int res = launch_radix_sort(c->qs, nq, 2 * kCodeLevels, c->stream);
        launch_point_place(c->qs.keys[res], c->qs.vals[res], (uint32_t)nq, d_qx, d_qy, d_ex,
                           c->ix.pts, (uint32_t)c->n, c->qpts, c->stream);
        qa.qpts = c->qpts;
        qa.qrow = (const int32_t *)c->qs.vals[res];
        if (d_ks) {
            launch_offsets(c->kcount, (uint32_t)nq, c->kscan, c->qscan, c->ktotal, c->offsets,
                           c->stream);
            qa.ks = (const int32_t *)c->kcount;
            qa.row_off = c->offsets;
        }
    } else if (d_ks) {
        const int64_t words = carve_workspace(c->qws, 1, &c->qs, &c->qscan, 1,
                                              &c->ix.ctr->bad_sync_query, c->query_epoch);
        launch_zero_words(c->qws.base, words, c->stream);
        launch_offsets(c->kcount, 0, c->kscan, c->qscan, c->ktotal, c->offsets, c->stream);
    }
    rc = mark_main(c, nq > 0 || ks != nullptr);
    if (rc) return rc;
    launch_sweep(c, qa, kmax_call);
    rc = check_launch(c, "k-NN query");
    if (!rc) rc = mark(c, 4);
    if (rc) return rc;
    record_query(c, nq, ks, k_uniform, where);
    return MKNN_OK;
}

int mknn_query(mknn_ctx *c, const int32_t *issuers, const int32_t *ks, int64_t nq,
               int32_t k_uniform, int32_t where)
{
    if (!c) return MKNN_E_INVAL;
    if (c->dead) return fail(c, MKNN_E_DEVICE, "context has a sticky device error%s");
    if (!valid_where(where)) return fail(c, MKNN_E_INVAL, "bad `where`%s");
    if (!c->ticked) return fail(c, MKNN_E_STATE, "query before advance_tick%s");
    if (nq < 0) return fail(c, MKNN_E_INVAL, "nq < 0%s");
    if (nq > c->cfg.q_max) return fail(c, MKNN_E_CAPACITY, "nq exceeds q_max%s");
    if (!issuers && nq != c->n)
        return fail(c, MKNN_E_INVAL, "issuers NULL requires nq == n%s");
    if (c->n == 0 && nq > 0) return fail(c, MKNN_E_INVAL, "queries need at least one object%s");
    if (!ks && (k_uniform < 1 || k_uniform > c->k_max))
        return fail(c, MKNN_E_INVAL, "k outside [1, k_max]%s");
    int kmax_call = ks ? c->k_max : k_uniform;
    // k classes that occur (bit c: lists of 8 << c keys); unknown for device ks.
    unsigned present = 0x1fu;
    if (where == MKNN_HOST) {
        int kmx = 1;
        unsigned seen = 0;
        for (int64_t i = 0; i < nq; ++i) {
            if (issuers && (issuers[i] < 0 || issuers[i] >= c->n))
                return fail(c, MKNN_E_INVAL, "issuer %s outside [0,n)",
                            std::to_string(i).c_str());
            if (ks) {
                if (ks[i] < 1 || ks[i] > c->k_max)
                    return fail(c, MKNN_E_INVAL, "k of query %s outside [1,k_max]",
                                std::to_string(i).c_str());
                if (ks[i] > kmx) kmx = ks[i];
                seen |= 1u << class_slot(ks[i]);
            }
        }
        if (ks) {
            kmax_call = kmx;
            present = seen;
        }
    }
    DeviceScope dev(c->cfg.device);
    HIP_OR_FAIL(c, dev.err);
    const int32_t *d_iss = issuers, *d_ks = ks;
    if (where == MKNN_HOST && nq > 0) {
        if (issuers) {
            HIP_OR_FAIL(c, hipMemcpyAsync(c->issuers, issuers, (size_t)nq * 4,
                                          hipMemcpyHostToDevice, c->stream));
            d_iss = c->issuers;
        }
        if (ks) {
            HIP_OR_FAIL(c, hipMemcpyAsync(c->ks, ks, (size_t)nq * 4, hipMemcpyHostToDevice,
                                          c->stream));
            d_ks = c->ks;
        }
        // Host arrays are read before the call returns: the caller may
        // reuse them at once.
        if (issuers || ks) HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    }
    int rc = mark(c, 2);
    if (rc) return rc;
    c->query_epoch = next_epoch(c->query_epoch);

    QueryArgs qa = base_query_args(c, nq, ks, k_uniform);

    // Variable k with MKNN_FLAG_GROUP_K: queries are grouped by k class
    // (sorted by class, then by position) and each class runs with its own
    // list size, as long as class and position fit one 32-bit sort key.
    const int pbits = pos_bits(c->n);
    const bool grouped = c->group_k && d_ks && nq > 0 && pbits + 3 <= 32 &&
                         !use_wave_sweep(c, kmax_call);
    if ((d_iss || grouped) && nq > 0 && !c->inv_ready) {
        launch_inverse(c->ix, c->n, c->stream);
        c->inv_ready = true;
    }
    const bool marks = d_iss && !grouped && order_by_marks(c->n, nq);
    if ((d_iss || d_ks) && nq > 0) {
        ScanSpace scans[2]{};
        const int64_t words = carve_workspace(c->qws, nq + 1, &c->qs, scans, marks ? 2 : 1,
                                              &c->ix.ctr->bad_sync_query, c->query_epoch);
        c->qscan = scans[0];
        QueryPrep p{};
        p.issuers = d_iss;
        p.ks = d_ks;
        p.nq = (uint32_t)nq;
        p.n = (uint32_t)c->n;
        p.k_max = c->k_max;
        p.inv = c->ix.inv;
        p.class_shift = grouped ? pbits : -1;
        p.sort = c->qs;
        p.kcount = c->kcount;
        p.ctr = c->ix.ctr;
        p.ws = c->qws.base;
        p.ws_words = words;
        p.epoch = c->query_epoch;
        launch_query_prep(p, c->stream);
        if (marks) {
            launch_marks_order(c, c->qs.keys[0], (uint32_t)nq, c->qs.vals[0], scans[1],
                               c->qs.keys[1], c->qs.vals[1]);
            qa.qpos = (const int32_t *)c->qs.keys[1];
            qa.qrow = (const int32_t *)c->qs.vals[1];
        } else if (d_iss || grouped) {
            const int res =
                launch_radix_sort(c->qs, nq, grouped ? pbits + 3 : bits_for(c->n), c->stream);
            qa.qpos = (const int32_t *)c->qs.keys[res];
            qa.qrow = (const int32_t *)c->qs.vals[res];
            if (grouped) {
                qa.pos_mask = (1u << pbits) - 1u;
                launch_class_bounds(c->qs.keys[res], (uint32_t)nq, pbits, c->class_bounds,
                                    c->stream);
                qa.class_bounds = c->class_bounds;
            }
        }
        if (d_ks) {
            launch_offsets(c->kcount, (uint32_t)nq, c->kscan, c->qscan, c->ktotal, c->offsets,
                           c->stream);
            qa.ks = (const int32_t *)c->kcount;
            qa.row_off = c->offsets;
        }
    } else if (d_ks) {
        // nq == 0 with variable k: a single zero offset.
        const int64_t words = carve_workspace(c->qws, 1, &c->qs, &c->qscan, 1,
                                              &c->ix.ctr->bad_sync_query, c->query_epoch);
        launch_zero_words(c->qws.base, words, c->stream);
        launch_offsets(c->kcount, 0, c->kscan, c->qscan, c->ktotal, c->offsets, c->stream);
    }
    rc = mark_main(c, issuers != nullptr || ks != nullptr);
    if (rc) return rc;
    if (qa.class_bounds) {
        const int top = class_slot(kmax_call);
        for (int cls = 0; cls <= top; ++cls) {
            if (!(present & (1u << cls))) continue;
            qa.klass = cls;
            launch_class(c, qa, 8 << cls, sweep_flavour(c, kmax_call));
        }
    } else {
        launch_sweep(c, qa, kmax_call);
    }
    rc = check_launch(c, "k-NN query");
    if (!rc) rc = mark(c, 4);
    if (rc) return rc;
    record_query(c, nq, ks, k_uniform, where);
    return MKNN_OK;
}

static int resolve_entries(mknn_ctx *c)
{
    if (c->entries >= 0) return MKNN_OK;
    int64_t tot = 0;
    HIP_OR_FAIL(c, hipMemcpyAsync(&tot, c->offsets + c->nq, sizeof tot, hipMemcpyDeviceToHost,
                                  c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->entries = tot;
    return MKNN_OK;
}

int mknn_sync(mknn_ctx *c)
{
    if (!c) return MKNN_E_INVAL;
    if (c->dead) return fail(c, MKNN_E_DEVICE, "context has a sticky device error%s");
    DeviceScope dev(c->cfg.device);
    HIP_OR_FAIL(c, dev.err);
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return check_deferred(c);
}

int mknn_result_size(const mknn_ctx *cc, int64_t *nq, int64_t *entries)
{
    mknn_ctx *c = const_cast<mknn_ctx *>(cc);
    if (!c) return MKNN_E_INVAL;
    if (!c->queried) return fail(c, MKNN_E_STATE, "no query yet%s");
    DeviceScope dev(c->cfg.device);
    HIP_OR_FAIL(c, dev.err);
    int rc = resolve_entries(c);
    if (rc) return rc;
    if (nq) *nq = c->nq;
    if (entries) *entries = c->entries;
    return MKNN_OK;
}

int mknn_result_device(const mknn_ctx *cc, const int32_t **ids, const float **d2,
                       const int32_t **counts, const int64_t **offsets)
{
    mknn_ctx *c = const_cast<mknn_ctx *>(cc);
    if (!c) return MKNN_E_INVAL;
    if (!c->queried) return fail(c, MKNN_E_STATE, "no query yet%s");
    if (ids) *ids = c->out_ids;
    if (d2) *d2 = c->out_d2;
    if (counts) *counts = c->out_cnt;
    if (offsets) *offsets = c->var_k ? c->offsets : nullptr;
    return MKNN_OK;
}

int mknn_fetch(mknn_ctx *c, int32_t *ids, float *d2, int32_t *counts, int64_t *offsets,
               int32_t where)
{
    if (!c) return MKNN_E_INVAL;
    if (!valid_where(where)) return fail(c, MKNN_E_INVAL, "bad `where`%s");
    if (!c->queried) return fail(c, MKNN_E_STATE, "fetch before query%s");
    DeviceScope dev(c->cfg.device);
    HIP_OR_FAIL(c, dev.err);
    int rc = mknn_sync(c);
    if (rc) return rc;
    rc = resolve_entries(c);
    if (rc) return rc;
    const hipMemcpyKind kind = where == MKNN_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    const size_t ne = (size_t)c->entries, nq = (size_t)c->nq;
    if (ids && ne) HIP_OR_FAIL(c, hipMemcpyAsync(ids, c->out_ids, ne * 4, kind, c->stream));
    if (d2 && ne) HIP_OR_FAIL(c, hipMemcpyAsync(d2, c->out_d2, ne * 4, kind, c->stream));
    if (counts && nq) HIP_OR_FAIL(c, hipMemcpyAsync(counts, c->out_cnt, nq * 4, kind, c->stream));
    if (offsets) {
        if (c->var_k) {
            HIP_OR_FAIL(c, hipMemcpyAsync(offsets, c->offsets, (nq + 1) * 8, kind, c->stream));
        } else if (where == MKNN_HOST) {
            for (size_t i = 0; i <= nq; ++i) offsets[i] = (int64_t)i * c->k_uniform;
        } else {
            std::vector<int64_t> h(nq + 1);
            for (size_t i = 0; i <= nq; ++i) h[i] = (int64_t)i * c->k_uniform;
            HIP_OR_FAIL(c, hipMemcpyAsync(offsets, h.data(), (nq + 1) * 8,
                                          hipMemcpyHostToDevice, c->stream));
            HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
        }
    }
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return MKNN_OK;
}

int mknn_index_fetch(mknn_ctx *c, uint32_t *codes, int32_t *ids, int32_t *level, uint32_t *prefix,
                     int64_t *begin, int64_t *end, int64_t leaf_cap, int64_t *n_leaves)
{
    if (!c) return MKNN_E_INVAL;
    if (!c->ticked) return fail(c, MKNN_E_STATE, "no index yet%s");
    DeviceScope dev(c->cfg.device);
    HIP_OR_FAIL(c, dev.err);
    int rc = mknn_sync(c);
    if (rc) return rc;
    IndexCounters h{};
    rc = read_counters(c, &h);
    if (rc) return rc;
    const int64_t n = c->n, nl = c->n > 0 ? h.n_leaves : 0;
    if (n_leaves) *n_leaves = nl;
    std::vector<Point> pts((size_t)n);
    if (n) HIP_OR_FAIL(c, hipMemcpy(pts.data(), c->ix.pts, (size_t)n * sizeof(Point),
                                    hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) {
        if (codes) codes[i] = pts[(size_t)i].code;
        if (ids) ids[i] = (int32_t)pts[(size_t)i].id;
    }
    if (nl > leaf_cap) return fail(c, MKNN_E_CAPACITY, "leaf_cap too small%s");
    std::vector<int32_t> lb((size_t)nl), le((size_t)nl), lv((size_t)nl);
    if (nl) {
        HIP_OR_FAIL(c, hipMemcpy(lb.data(), c->ix.leaf_begin, (size_t)nl * 4, hipMemcpyDeviceToHost));
        HIP_OR_FAIL(c, hipMemcpy(le.data(), c->ix.leaf_end, (size_t)nl * 4, hipMemcpyDeviceToHost));
        HIP_OR_FAIL(c, hipMemcpy(lv.data(), c->ix.leaf_level, (size_t)nl * 4, hipMemcpyDeviceToHost));
    }
    for (int64_t j = 0; j < nl; ++j) {
        if (level) level[j] = lv[(size_t)j];
        if (begin) begin[j] = lb[(size_t)j];
        if (end) end[j] = le[(size_t)j];
        if (prefix) {
            const int l = lv[(size_t)j];
            const uint32_t code = pts[(size_t)lb[(size_t)j]].code;
            prefix[j] = l <= 0 ? 0u : code >> (2 * (kCodeLevels - l));
        }
    }
    return MKNN_OK;
}

int mknn_set_leaf_capacity(mknn_ctx *c, int32_t th)
{
    if (!c) return MKNN_E_INVAL;
    if (th < 1) return fail(c, MKNN_E_INVAL, "leaf capacity must be >= 1%s");
    if (node_capacity(c->cfg.n_max, th, c->L) > c->ix.node_cap)
        return fail(c, MKNN_E_CAPACITY, "leaf capacity %s needs larger node tables than allocated",
                    std::to_string(th).c_str());
    c->th = th;
    return MKNN_OK;
}

int mknn_get_schedule(const mknn_ctx *c, mknn_schedule *out)
{
    if (!c || !out) return MKNN_E_INVAL;
    out->leaf_capacity = c->th;
    out->max_level = c->L;
    out->sweep = c->sweep;
    out->group_k = c->group_k ? 1 : 0;
    out->tile_queries = c->tile_queries;
    return MKNN_OK;
}

int mknn_set_schedule(mknn_ctx *c, const mknn_schedule *sc)
{
    if (!c || !sc) return MKNN_E_INVAL;
    if (sc->leaf_capacity < 1) return fail(c, MKNN_E_INVAL, "leaf capacity must be >= 1%s");
    if (sc->max_level < 1 || sc->max_level > kCodeLevels)
        return fail(c, MKNN_E_INVAL, "max_level must be in 1..16%s");
    if (sc->sweep != MKNN_SWEEP_AUTO && sc->sweep != MKNN_SWEEP_LANE &&
        sc->sweep != MKNN_SWEEP_WAVE && sc->sweep != MKNN_SWEEP_GROUP)
        return fail(c, MKNN_E_INVAL, "unknown sweep flavour%s");
    if (sc->tile_queries != 0 && sc->tile_queries != 8 && sc->tile_queries != 16 &&
        sc->tile_queries != 32 && sc->tile_queries != 64)
        return fail(c, MKNN_E_INVAL, "tile_queries must be 0, 8, 16, 32 or 64%s");
    if (node_capacity(c->cfg.n_max, sc->leaf_capacity, sc->max_level) > c->ix.node_cap)
        return fail(c, MKNN_E_CAPACITY, "schedule needs larger node tables than allocated%s");
    c->th = sc->leaf_capacity;
    c->L = sc->max_level;
    c->sweep = sc->sweep;
    c->group_k = sc->group_k != 0;
    c->tile_queries = sc->tile_queries;
    return MKNN_OK;
}

int mknn_set_epochs(mknn_ctx *c, uint32_t build_epoch, uint32_t query_epoch)
{
    if (!c) return MKNN_E_INVAL;
    if (build_epoch < 1 || build_epoch >= (1u << 24) || query_epoch < 1 ||
        query_epoch >= (1u << 24))
        return fail(c, MKNN_E_INVAL, "epochs run 1 .. 2^24-1%s");
    c->build_epoch = build_epoch;
    c->query_epoch = query_epoch;
    return MKNN_OK;
}

int mknn_reset_timing(mknn_ctx *c)
{
    if (!c) return MKNN_E_INVAL;
    DeviceScope dev(c->cfg.device);
    HIP_OR_FAIL(c, dev.err);
    int rc = mknn_sync(c);
    if (rc) return rc;
    c->builds_timed = 0;
    c->queries_timed = 0;
    k_zero_u64<<<1, 8, 0, c->stream>>>(c->counters, 8);
    return check_launch(c, "reset counters");
}

int mknn_query_time(const mknn_ctx *cc, int32_t back, int32_t wait, float *ms)
{
    mknn_ctx *c = const_cast<mknn_ctx *>(cc);
    if (!c || !ms) return MKNN_E_INVAL;
    if (!((c->cfg.flags & MKNN_FLAG_TIMING) && c->have_ring))
        return fail(c, MKNN_E_INVAL, "query_time needs MKNN_FLAG_TIMING%s");
    if (back < 0 || back >= mknn_ctx::kRing || (int64_t)back >= c->query_slot)
        return fail(c, MKNN_E_INVAL, "no such query%s");
    const int64_t slot = (c->query_slot - 1 - back) % mknn_ctx::kRing;
    DeviceScope dev(c->cfg.device);
    if (dev.err != hipSuccess) return hip_fail(c, dev.err, "hipSetDevice");
    // Not finished (or never timed): report it without leaving a HIP error
    // behind for the next launch check to find.
    hipEvent_t end = c->ring[slot][4];
    float t = 0;
    if (wait) (void)hipEventSynchronize(end);
    if (hipEventQuery(end) != hipSuccess ||
        hipEventElapsedTime(&t, c->ring[slot][2], end) != hipSuccess) {
        (void)hipGetLastError();
        return MKNN_E_STATE;
    }
    *ms = t;
    return MKNN_OK;
}

int mknn_get_stats(const mknn_ctx *cc, mknn_stats *out)
{
    mknn_ctx *c = const_cast<mknn_ctx *>(cc);
    if (!c || !out) return MKNN_E_INVAL;
    memset(out, 0, sizeof *out);
    out->tick = c->ticks;
    out->n = c->n;
    out->nq = c->queried ? c->nq : 0;
    out->leaf_capacity = c->th;
    if (c->ticked && !c->dead) {
        DeviceScope dev(c->cfg.device);
        HIP_OR_FAIL(c, dev.err);
        IndexCounters h{};
        int rc = read_counters(c, &h);
        if (rc) return rc;
        if (c->cfg.flags & MKNN_FLAG_COUNTERS) {
            unsigned long long w[5] = {0, 0, 0, 0, 0};
            HIP_OR_FAIL(c, hipMemcpy(w, c->counters, sizeof w, hipMemcpyDeviceToHost));
            out->wave_candidate_steps = (int64_t)w[0];
            out->wave_merges = (int64_t)w[1];
            out->wave_node_visits = (int64_t)w[2];
            out->wave_leaf_sweeps = (int64_t)w[3];
            out->wavefronts = (int64_t)w[4];
        }
        out->leaves = c->n > 0 ? h.n_leaves : 0;
        out->nodes = c->n > 0 ? h.n_nodes : 0;
        out->deepest_level = (h.deepest >> 8) == c->build_epoch ? (int32_t)(h.deepest & 0xff) : 0;
        out->refits = c->refits;
        if ((uint32_t)(h.drift >> 32) == c->build_epoch) {
            const uint32_t bits = (uint32_t)h.drift;
            memcpy(&out->drift, &bits, sizeof bits);
        }
        if ((c->cfg.flags & MKNN_FLAG_TIMING) && c->have_ring) {
            const int R = mknn_ctx::kRing;
            float ms = 0;
            auto elapsed = [&](int64_t slot, int a, int b, double *acc) {
                hipEvent_t ea = c->ring[slot % R][a], eb = c->ring[slot % R][b];
                if (a == 3 && c->main_is_start[slot % R]) ea = c->ring[slot % R][2];
                if (hipEventElapsedTime(&ms, ea, eb) != hipSuccess) return false;
                *acc += ms;
                return true;
            };
            double v = 0;
            if (c->build_slot > 0 && elapsed(c->build_slot - 1, 0, 1, &v)) out->ms_build = (float)v;
            if (c->queried && c->query_slot > 0) {
                v = 0;
                if (elapsed(c->query_slot - 1, 2, 4, &v)) out->ms_query = (float)v;
                v = 0;
                if (elapsed(c->query_slot - 1, 3, 4, &v)) out->ms_query_main = (float)v;
            }
            // Means over the builds and queries since the last reset (at
            // most the ring's length, the most recent ones).
            const int64_t nb = c->builds_timed < R ? c->builds_timed : R;
            const int64_t nqr = c->queries_timed < R ? c->queries_timed : R;
            double sb = 0, sq = 0, sm = 0;
            for (int64_t i = 0; i < nb; ++i) elapsed(c->build_slot - 1 - i, 0, 1, &sb);
            for (int64_t i = 0; i < nqr; ++i) {
                elapsed(c->query_slot - 1 - i, 2, 4, &sq);
                elapsed(c->query_slot - 1 - i, 3, 4, &sm);
            }
            out->timed_ticks = (int32_t)(nb < nqr ? nb : nqr);
            if (nb) out->ms_build_mean = (float)(sb / nb);
            if (nqr) {
                out->ms_query_mean = (float)(sq / nqr);
                out->ms_query_main_mean = (float)(sm / nqr);
            }
            (void)hipGetLastError();
        }
    }
    return MKNN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// One tick without allocating (mknn_knn_noalloc): the index build and the
// all-objects query of the context path, with every intermediate buffer
// carved from one file-scope device array.
// ---------------------------------------------------------------------------
namespace {

// The array every mknn_knn_noalloc call on a GPU carves its buffers from.
// Each GPU holds its own copy at its own address.  In host code this name is
// a host-side stand-in, not a device address: host code uses only the
// address looked up per device below (kernel arguments, carving).
static __device__ __align__(256) unsigned char scratch[MKNN_NOALLOC_SCRATCH_BYTES];

constexpr int kScratchDevices = 64;
std::mutex scratch_mu;
unsigned char *scratch_dev[kScratchDevices];  // device address per device, or null

// Device address of `scratch` on device `dev`, which must be current: looked
// up on the first call on that device and kept.
hipError_t scratch_address(int dev, unsigned char **out)
{
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_dev[dev] = (unsigned char *)p;
    }
    *out = scratch_dev[dev];
    return hipSuccess;
}

// Consecutive 256-byte aligned pieces of the array; ok turns false when a
// piece does not fit.
struct ScratchCarve {
    unsigned char *base;
    size_t used = 0;
    bool ok = true;

    template <class T>
    T *take(int64_t count)
    {
        if (count < 1) count = 1;
        const size_t at = (used + 255) / 256 * 256;
        const size_t bytes = (size_t)count * sizeof(T);
        if (!ok || at + bytes > (size_t)MKNN_NOALLOC_SCRATCH_BYTES) {
            ok = false;
            return nullptr;
        }
        used = at + bytes;
        return (T *)(base + at);
    }
};

__global__ void k_noalloc_status(const IndexCounters *ctr, int32_t *status)
{
    const bool device_err = (ctr->bad_nodes | ctr->bad_sync_build) != 0;
    *status = ctr->bad_coord ? MKNN_E_RANGE : device_err ? MKNN_E_DEVICE : MKNN_OK;
}

__global__ void k_noalloc_ok(int32_t *status) { *status = MKNN_OK; }

}  // namespace

extern "C" int mknn_knn_noalloc(const float *x, const float *y, int64_t n, int32_t k,
                                int32_t leaf_capacity, int32_t *ids, float *d2, int32_t *counts,
                                int32_t *status, void *stream)
{
    if (n < 0 || k < 1 || k > MKNN_K_LIMIT || leaf_capacity < 0) return MKNN_E_INVAL;
    if (n > 0 && (!x || !y || !ids || !d2 || !counts)) return MKNN_E_INVAL;
    if (n > MKNN_NOALLOC_MAX_N) return MKNN_E_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) {
        (void)hipGetLastError();
        return MKNN_E_DEVICE;
    }
    unsigned char *base = nullptr;
    if (scratch_address(dev, &base) != hipSuccess) {
        (void)hipGetLastError();
        return MKNN_E_DEVICE;
    }
    if (n == 0) {
        if (status) k_noalloc_ok<<<1, 1, 0, s>>>(status);
        return hipGetLastError() == hipSuccess ? MKNN_OK : MKNN_E_DEVICE;
    }
    const int th = leaf_capacity ? leaf_capacity : mknn_default_leaf_capacity(k);
    const int L = kCodeLevels;

    // The buffers of one context's index, sized for this call's n.
    IndexBuffers ix{};
    ix.n_cap = n;
    ix.node_cap = node_capacity(n, th, L);
    ix.ws.cap_words = workspace_words(n);
    ScratchCarve cv{base};
    for (int i = 0; i < 2; ++i) {
        ix.sort.keys[i] = cv.take<uint32_t>(n);
        ix.sort.vals[i] = cv.take<uint32_t>(n);
    }
    ix.ws.base = cv.take<uint64_t>(ix.ws.cap_words);
    ix.xy = cv.take<float2>(n);
    ix.anchor = cv.take<float2>(n);
    ix.pts = cv.take<Point>(n);
    ix.inv = nullptr;  // only subset queries use it
    ix.leaf_of = cv.take<int32_t>(n);
    ix.leaf_begin = cv.take<int32_t>(n);
    ix.leaf_end = cv.take<int32_t>(n);
    ix.leaf_level = cv.take<int32_t>(n);
    ix.leaf_code = cv.take<uint32_t>(n);
    ix.cnt_f = cv.take<uint32_t>(n);
    ix.cnt_r = cv.take<uint32_t>(n);
    ix.leaf_node_f = cv.take<int32_t>(n);
    ix.leaf_node_r = cv.take<int32_t>(n);
    ix.fwd = cv.take<Node>(ix.node_cap);
    ix.rev = cv.take<Node>(ix.node_cap);
    ix.ctr = cv.take<IndexCounters>(1);
    if (!cv.ok) return MKNN_E_CAPACITY;

    // The counters and error words start at zero (the build's first kernel
    // zeroes its own look-back words); epoch 1 tags this build.
    const uint32_t epoch = 1;
    k_reset_counters<<<1, 1, 0, s>>>(ix.ctr);
    launch_build_index(ix, x, y, n, th, L, epoch, s);

    QueryArgs qa{};
    qa.pts = ix.pts;
    qa.n = (uint32_t)n;
    qa.fwd = ix.fwd;
    qa.rev = ix.rev;
    qa.leaf_of = ix.leaf_of;
    qa.leaf_begin = ix.leaf_begin;
    qa.leaf_end = ix.leaf_end;
    qa.leaf_node_f = ix.leaf_node_f;
    qa.leaf_node_r = ix.leaf_node_r;
    qa.ctr = ix.ctr;
    qa.node_cap = (int32_t)ix.node_cap;
    qa.nq = (uint32_t)n;
    qa.k_uniform = k;
    qa.out_ids = ids;
    qa.out_d2 = d2;
    qa.out_cnt = counts;
    qa.build_epoch = epoch;
    qa.pos_mask = 0xffffffffu;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
            qa.compute_units = (uint32_t)cus;
    }
    // The flavour mknn_query's AUTO schedule picks.
    if (k > kAutoLaneMaxK) launch_knn_group(qa, k_class_group(k), s);
    else launch_knn(qa, k_class(k), s);
    if (status) k_noalloc_status<<<1, 1, 0, s>>>(ix.ctr, status);
    return hipGetLastError() == hipSuccess ? MKNN_OK : MKNN_E_DEVICE;
}
