// Iterative k-NN query processing (arXiv 1412.6170, Sec. 4.2), gfx950.
//
// Queries are processed in Morton order of their centres, 64 per
// wavefront (one query per lane), so the queries of one wavefront are
// spatial neighbours, as the paper groups the queries of one leaf into one
// task.  Each lane keeps its current best keys (d2 bits << 32 | id) sorted
// in registers; the k-th key bounds what can still enter.
//
//   1. First iteration: every object of the leaves holding the wavefront's
//      queries is a candidate (Sec. 4.2.1, distance computations).
//   2. Subsequent iterations: two sub-visits leave the own leaves in Morton
//      order, one towards higher codes and one towards lower codes, taking
//      turns (Sec. 4.2.2).  A quadtree node is entered only if, for some
//      lane, the lower bound of d2 to the node's box is not above that
//      lane's k-th distance; otherwise the walk jumps over its subtree
//      (the node tables are depth-first with subtree-skip links, so the walk
//      needs neither a stack nor a lookup table).  A reached leaf is swept:
//      every lane evaluates every object of the leaf.
//
// The paper runs each iteration as separate kernels with a host loop and
// re-sorts the active queries between iterations; here a wavefront carries
// its 64 queries through all iterations without leaving the kernel, so no
// active-query sort or host round trip is needed and every candidate leaf is
// read with wave-uniform (scalar) loads.
//
// Exactness.  d2 = fl(fl(dx*dx) + fl(dy*dy)) with no contraction (this file
// is built with -ffp-contract=off and the pragma below).  A box is skipped
// only when its lower bound -- the same rounded operations applied to the
// nearest box edge -- is strictly above the k-th d2; rounding is monotone,
// so no object of a skipped box could have entered.  Keys order by (d2, id),
// so the kept set is exactly the first k of Definition 1 with id tie-breaks.
#include <float.h>

#include "mknn_internal.hpp"
#include "query.hpp"

#pragma clang fp contract(off)

namespace mknn {

// Keys are (d2 bits << 32 | id).  d2 is a non-negative finite float, so a
// key is also the bit pattern of a non-negative finite double, and doubles
// of that kind order exactly like their bit patterns (denormal doubles --
// keys with d2 = 0 -- included, as the kernel keeps fp64 denormals).  The
// selection networks therefore compare-exchange keys with one fp64 min and
// one fp64 max.  The empty-slot key is the largest finite double, above
// every real key (whose high word is at most 0x7f7fffff).
constexpr uint64_t kKeyMax = 0x7fefffffffffffffull;

__device__ __forceinline__ double as_f64(uint64_t k) { return __longlong_as_double((long long)k); }
__device__ __forceinline__ uint64_t as_key(double d) { return (uint64_t)__double_as_longlong(d); }
__device__ __forceinline__ uint64_t key_min(uint64_t a, uint64_t b)
{
    return as_key(__builtin_fmin(as_f64(a), as_f64(b)));
}
__device__ __forceinline__ uint64_t key_max(uint64_t a, uint64_t b)
{
    return as_key(__builtin_fmax(as_f64(a), as_f64(b)));
}
__device__ __forceinline__ bool key_less(uint64_t a, uint64_t b) { return as_f64(a) < as_f64(b); }

// A 64-bit word in LDS (address space 3), so queue accesses stay ds_* ops.
typedef __attribute__((address_space(3))) uint64_t lds_u64;

__device__ __forceinline__ float sq_dist(float qx, float qy, float px, float py)
{
    const float dx = qx - px;
    const float dy = qy - py;
    const float ax = dx * dx;
    const float ay = dy * dy;
    return ax + ay;
}

__device__ __forceinline__ float box_lower_bound(float qx, float qy, const Node &nd)
{
    const float gx = (qx < nd.x0) ? (nd.x0 - qx) : ((qx >= nd.x1) ? (qx - nd.x1) : 0.0f);
    const float gy = (qy < nd.y0) ? (nd.y0 - qy) : ((qy >= nd.y1) ? (qy - nd.y1) : 0.0f);
    const float ax = gx * gx;
    const float ay = gy * gy;
    return ax + ay;
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Compare-exchange on keys: afterwards lo <= hi.
__device__ __forceinline__ void cmp_swap(uint64_t &lo, uint64_t &hi)
{
    const uint64_t t = key_min(lo, hi);
    hi = key_max(lo, hi);
    lo = t;
}

// Bitonic sorting network on a register array (all indices static).
template <int N>
__device__ __forceinline__ void bitonic_sort(uint64_t (&b)[N])
{
#pragma unroll
    for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (int stride = size / 2; stride > 0; stride >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int j = i ^ stride;
                if (j > i) {
                    if ((i & size) == 0) cmp_swap(b[i], b[j]);
                    else cmp_swap(b[j], b[i]);
                }
            }
        }
    }
}

// Sort a bitonic register array ascending (half-cleaner cascade).
template <int N>
__device__ __forceinline__ void bitonic_merge(uint64_t (&a)[N])
{
#pragma unroll
    for (int stride = N / 2; stride > 0; stride >>= 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int j = i ^ stride;
            if (j > i) cmp_swap(a[i], a[j]);
        }
    }
}

// Lane-private selection of the K best keys (d2 bits << 32 | id).
//
// a[] holds the current best, sorted, in registers.  A lane asking for
// k < K keeps K-k permanent zero sentinels at the bottom, so its k-th key is
// always a[K-1] and one template serves a mix of k.
//
// Candidates below the lane's threshold are not inserted one by one (in a
// wavefront every lane would pay for any lane's insertion); they are
// appended to a lane-private queue of P keys in LDS.  When some lane's
// queue is full -- and once at the end -- every lane merges its queue into
// a[]: the queue is sorted with a bitonic network, the lower K keys of
// a[] and the queue are taken with one min against the reversed queue
// (which leaves a bitonic sequence) and a bitonic merge sorts them.
//
// The threshold is min(a[K-1], cap): cap is one above a key known not to be
// exceeded by the k-th key (the k-th smallest key of any k other objects
// bounds it from above), so filtering with it drops nothing that belongs to
// the answer.  Between merges the threshold may be stale, which only lets
// more keys into the queue.  The query's own object is queued like any
// other candidate (its key is (0, own id)) and is removed at merge time.
template <int K, int P>
struct Selector {
    uint64_t a[K];
    lds_u64 *q;        // this lane's queue: q[s * kWave], s < P
    uint32_t cnt;
    uint64_t cap;      // upper bound (exclusive) from the seed
    uint64_t thr;      // min(a[K-1], cap) at the last merge
    uint64_t self_key;

    __device__ __forceinline__ void init(int k, lds_u64 *lane_queue, uint32_t self_id)
    {
#pragma unroll
        for (int s = 0; s < K; ++s) a[s] = (s < K - k) ? 0ull : kKeyMax;
        q = lane_queue;
        cnt = 0;
        cap = kKeyMax;
        thr = kKeyMax;
        self_key = (uint64_t)self_id;  // d2 of the query to itself is +0
    }

    __device__ __forceinline__ void set_cap(uint64_t c)
    {
        cap = c;
        thr = key_min(a[K - 1], cap);
    }

    // Every lane writes its key to its next free slot; only lanes whose key
    // passes advance.  No branch, so no lane waits on another's insertion.
    __device__ __forceinline__ void offer(uint64_t key)
    {
        q[cnt * kWave] = key;
        cnt += key_less(key, thr) ? 1u : 0u;
    }

    __device__ __forceinline__ void merge()
    {
        // Read every slot (volatile keeps the loads unconditional: slots
        // past cnt hold stale keys and are masked after the load).
        const volatile lds_u64 *vq = q;
        uint64_t b[P];
#pragma unroll
        for (int s = 0; s < P; ++s) b[s] = vq[s * kWave];
#pragma unroll
        for (int s = 0; s < P; ++s) b[s] = ((uint32_t)s < cnt && b[s] != self_key) ? b[s] : kKeyMax;
        bitonic_sort<P>(b);
#pragma unroll
        for (int i = K - P; i < K; ++i) a[i] = key_min(a[i], b[K - 1 - i]);
        bitonic_merge<K>(a);
        cnt = 0;
        thr = key_min(a[K - 1], cap);
    }
};

template <int K, int P>
struct Lane {
    float qx, qy;
    bool active;
    Selector<K, P> sel;
    uint32_t n_cand = 0, n_merge = 0, n_node = 0, n_leaf = 0;  // wave-uniform

    __device__ __forceinline__ void offer(const Point &p)
    {
        const float d2 = sq_dist(qx, qy, p.x, p.y);
        sel.offer(((uint64_t)__float_as_uint(d2) << 32) | p.id);
    }

    __device__ __forceinline__ void merge_if(bool full)
    {
        if (wave_any(full)) {
            sel.merge();
            ++n_merge;
        }
    }

    // Every lane evaluates every object of the sorted range [b, e).  The
    // range is wave-uniform, so objects arrive through scalar loads, two per
    // step, with the next two requested before the current ones are used.
    // Invariant between steps (and between sweeps): every queue holds at
    // most P-2 keys, so a step's two writes stay inside the queue; a merge
    // runs as soon as a queue holds more.
    __device__ __forceinline__ void sweep(const Point *__restrict__ pts, int32_t b, int32_t e)
    {
        if (b >= e) return;
        n_cand += (uint32_t)(e - b);
        ++n_leaf;
        int32_t j = b;
        if (e - b >= 2) {
            Point c0 = pts[j], c1 = pts[j + 1];
            for (; j + 2 <= e; j += 2) {
                const int32_t jn = j + 4 <= e ? j + 2 : j;
                const Point n0 = pts[jn], n1 = pts[jn + 1];
                offer(c0);
                offer(c1);
                merge_if(sel.cnt > (uint32_t)(P - 2));
                c0 = n0;
                c1 = n1;
            }
        }
        if (j < e) {
            offer(pts[j]);
            merge_if(sel.cnt > (uint32_t)(P - 2));
        }
    }

    // A node is needed if its box may hold a key below some lane's
    // threshold (queued keys are not yet counted, so this errs on the side
    // of visiting).
    __device__ __forceinline__ bool wants(const Node &nd) const
    {
        return active &&
               __float_as_uint(box_lower_bound(qx, qy, nd)) <= (uint32_t)(sel.thr >> 32);
    }
};

// Positions only move forward (a skip link never points back) and sweep
// ranges are clamped to the object array, so the walk always terminates
// inside its buffers.
template <int K, int P>
__device__ __forceinline__ int32_t walk_step(Lane<K, P> &ln, const Node *__restrict__ tab,
                                             int32_t pos, int32_t total,
                                             const Point *__restrict__ pts, int32_t n)
{
    while (pos < total) {
        const Node nd = tab[pos];
        ++ln.n_node;
        const int32_t next = nd.skip > pos ? nd.skip : pos + 1;
        if (!wave_any(ln.wants(nd))) {
            pos = next;
            continue;
        }
        if (nd.leaf >= 0) {
            ln.sweep(pts, max(nd.begin, 0), min(nd.end, n));
            return next;
        }
        ++pos;
    }
    return total;
}

template <int K, int P>
__global__ __launch_bounds__(256) void k_knn_tiles(QueryArgs qa)
{
    __shared__ uint64_t s_queue[256 / kWave][P * kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wib = threadIdx.x / kWave;
    const uint32_t tile = blockIdx.x * (blockDim.x / kWave) + wib;
    const uint32_t t = tile * kWave + lane;
    if (tile * kWave >= qa.nq) return;  // whole wavefront idle

    Lane<K, P> ln;
    ln.active = t < qa.nq;
    const uint32_t tq = ln.active ? t : qa.nq - 1;
    const int32_t qp = qa.qpos ? qa.qpos[tq] : (int32_t)tq;
    const Point q = qa.pts[qp];
    ln.qx = q.x;
    ln.qy = q.y;
    const int32_t row = qa.qrow ? qa.qrow[tq] : (int32_t)q.id;
    int kq = qa.ks ? qa.ks[row] : qa.k_uniform;
    kq = kq < 1 ? 1 : (kq > K ? K : kq);
    ln.sel.init(kq, (lds_u64 *)&s_queue[wib][lane], q.id);

    // Seed: the kq objects around the query in Morton order (a window of
    // kq + 1 sorted positions holding the query) are kq other objects, so
    // the largest of their keys bounds the k-th key from above.  Inactive
    // lanes keep a zero threshold and never queue anything.
    {
        const int32_t n = (int32_t)qa.n;
        uint64_t seed = 0;
        if (n - 1 >= kq) {
            int32_t w0 = qp - kq / 2;
            w0 = w0 < 0 ? 0 : (w0 > n - 1 - kq ? n - 1 - kq : w0);
#pragma unroll 4
            for (int s = 0; s <= K; ++s) {
                if (s <= kq) {
                    const int32_t j = w0 + s;
                    if (j != qp) {
                        const Point p = qa.pts[j];
                        const float d2 = sq_dist(q.x, q.y, p.x, p.y);
                        seed = key_max(seed, ((uint64_t)__float_as_uint(d2) << 32) | p.id);
                    }
                }
            }
            ln.sel.set_cap(seed + 1);
        }
        if (!ln.active) ln.sel.set_cap(0);
    }

    // Own leaves of the wavefront's queries: a contiguous run of leaves.
    const int32_t my_leaf = qa.leaf_of[qp];
    int32_t l0 = my_leaf, l1 = my_leaf;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        l0 = min(l0, __shfl_xor(l0, d, kWave));
        l1 = max(l1, __shfl_xor(l1, d, kWave));
    }
    l0 = __builtin_amdgcn_readfirstlane(l0);
    l1 = __builtin_amdgcn_readfirstlane(l1);

    // First iteration: the own leaves.
    ln.sweep(qa.pts, max(qa.leaf_begin[l0], 0), min(qa.leaf_end[l1], (int32_t)qa.n));

    // Subsequent iterations: alternate the two sub-visits.
    const int32_t total = min((int32_t)qa.ctr->n_nodes, qa.node_cap);
    int32_t rf = qa.leaf_node_f[l1] + 1;
    int32_t rl = qa.leaf_node_r[l0] + 1;
    rf = (rf < 1 || rf > total) ? total : rf;
    rl = (rl < 1 || rl > total) ? total : rl;
    bool right = true;
    while (rf < total || rl < total) {
        // One code path for both directions (the table is picked uniformly),
        // so the list is not duplicated across two inlined sweeps.
        const bool fw = (right && rf < total) || rl >= total;
        const int32_t pos =
            walk_step<K, P>(ln, fw ? qa.fwd : qa.rev, fw ? rf : rl, total, qa.pts, (int32_t)qa.n);
        rf = fw ? pos : rf;
        rl = fw ? rl : pos;
        right = !right;
    }

    if (wave_any(ln.sel.cnt > 0)) {
        ln.sel.merge();
        ++ln.n_merge;
    }
    if (qa.counters && lane == 0) {
        atomicAdd(&qa.counters[0], (unsigned long long)ln.n_cand);
        atomicAdd(&qa.counters[1], (unsigned long long)ln.n_merge);
        atomicAdd(&qa.counters[2], (unsigned long long)ln.n_node);
        atomicAdd(&qa.counters[3], (unsigned long long)ln.n_leaf);
        atomicAdd(&qa.counters[4], 1ull);
    }

    if (!ln.active) return;
    const int64_t off = qa.row_off ? qa.row_off[row] : (int64_t)row * qa.k_uniform;
    int32_t *__restrict__ oi = qa.out_ids + off;
    float *__restrict__ od = qa.out_d2 + off;
    int cnt = 0;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int slot = s - (K - kq);
        if (slot >= 0) {
            const uint64_t v = ln.sel.a[s];
            const bool real = v != kKeyMax;
            oi[slot] = real ? (int32_t)(uint32_t)v : -1;
            od[slot] = real ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_inff();
            cnt += real ? 1 : 0;
        }
    }
    qa.out_cnt[row] = cnt;
}

int k_class(int k)
{
    if (k <= 8) return 8;
    if (k <= 16) return 16;
    if (k <= 32) return 32;
    if (k <= 64) return 64;
    return 128;
}

void launch_knn(const QueryArgs &qa, int kclass, hipStream_t s)
{
    if (qa.nq == 0) return;
    const uint32_t tiles = (qa.nq + kWave - 1) / kWave;
    const uint32_t waves_per_block = 4;
    const uint32_t blocks = (tiles + waves_per_block - 1) / waves_per_block;
    const dim3 grid(blocks), block(waves_per_block * kWave);
    switch (kclass) {
    case 8: k_knn_tiles<8, 8><<<grid, block, 0, s>>>(qa); break;
    case 16: k_knn_tiles<16, 16><<<grid, block, 0, s>>>(qa); break;
    case 32: k_knn_tiles<32, 16><<<grid, block, 0, s>>>(qa); break;
    case 64: k_knn_tiles<64, 16><<<grid, block, 0, s>>>(qa); break;
    default: k_knn_tiles<128, 16><<<grid, block, 0, s>>>(qa); break;
    }
}

// ---------------------------------------------------------------------------
// Query indexing for a subset of issuers (Sec. 4.2.1, query indexing): sort
// the queries by their centre's sorted position so wavefronts hold spatial
// neighbours.  Device-supplied issuers and ks are range-checked here.
// ---------------------------------------------------------------------------

__global__ void k_query_keys(const int32_t *__restrict__ issuers, const int32_t *__restrict__ ks,
                             uint32_t nq, uint32_t n, int k_max, const int32_t *__restrict__ inv,
                             uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                             uint32_t *__restrict__ kcount, IndexCounters *__restrict__ ctr,
                             uint64_t *__restrict__ ws, int64_t ws_words, uint32_t epoch)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    // The query sort and scan workspace starts at zero.
    for (int64_t w = q; w < ws_words; w += (int64_t)gridDim.x * blockDim.x) ws[w] = 0ull;
    if (q >= nq) return;
    if (issuers) {
        int32_t s = issuers[q];
        bool ok = s >= 0 && (uint32_t)s < n;
        if (!ok) atomicMax(&ctr->bad_issuer, epoch);
        keys[q] = ok ? (uint32_t)inv[s] : 0u;
        vals[q] = q;
    }
    if (ks) {
        int32_t k = ks[q];
        bool ok = k >= 1 && k <= k_max;
        if (!ok) atomicMax(&ctr->bad_k, epoch);
        kcount[q] = ok ? (uint32_t)k : 1u;
    }
}

__global__ void k_widen_offsets(const uint32_t *__restrict__ excl, const uint32_t *__restrict__ total,
                                uint32_t nq, int64_t *__restrict__ off)
{
    uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) off[q] = (int64_t)excl[q];
    if (q == 0) off[nq] = (int64_t)*total;
}

void launch_query_prep(const QueryPrep &p, hipStream_t s)
{
    const int T = 256;
    const uint32_t g = (p.nq + T - 1) / T;
    if (p.nq == 0) return;
    k_query_keys<<<g, T, 0, s>>>(p.issuers, p.ks, p.nq, p.n, p.k_max, p.inv, p.sort.keys[0],
                                 p.sort.vals[0], p.kcount, p.ctr, p.ws, p.ws_words, p.epoch);
}

void launch_offsets(const uint32_t *kcount, uint32_t nq, uint32_t *scan_out, const ScanSpace &sp,
                    uint32_t *total, int64_t *offsets, hipStream_t s)
{
    launch_exclusive_scan(kcount, scan_out, nq, sp, total, s);
    const int T = 256;
    k_widen_offsets<<<(nq + 1 + T - 1) / T, T, 0, s>>>(scan_out, total, nq, offsets);
}

}  // namespace mknn
