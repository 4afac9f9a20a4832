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
// active-query sort or host round trip is needed; a candidate leaf is read
// once per wavefront, 64 records at a time with coalesced 16-byte loads into
// LDS, from where every lane reads each record.
//
// Exactness.  d2 = fl(fl(dx*dx) + fl(dy*dy)) with no contraction (this file
// is built with -ffp-contract=off and the pragma below).  A box is skipped
// only when its lower bound -- the same rounded operations applied to the
// nearest box edge -- is strictly above the k-th d2; rounding is monotone,
// so no object of a skipped box could have entered.  Keys order by (d2, id),
// so the kept set is exactly the first k of Definition 1 with id tie-breaks.
#include <float.h>

#include <utility>

#include "mknn_internal.hpp"
#include "query.hpp"
#include "query_device.hpp"

#pragma clang fp contract(off)

namespace mknn {

// Sorting networks on register arrays.  They are expanded with templates
// (fold expressions over the element indices) rather than unrolled loops, so
// every index is a compile-time constant whatever the size: an array
// indexed at run time would be moved to scratch memory.

// One compare-exchange of a bitonic sort stage: blocks of SIZE elements,
// partner at distance STRIDE, ascending blocks where (I & SIZE) == 0.
template <int N, int SIZE, int STRIDE, int I>
__device__ __forceinline__ void sort_ce(uint64_t (&b)[N])
{
    constexpr int J = I ^ STRIDE;
    if constexpr (J > I) {
        if constexpr ((I & SIZE) == 0) cmp_swap(b[I], b[J]);
        else cmp_swap(b[J], b[I]);
    }
}

template <int N, int SIZE, int STRIDE, int... I>
__device__ __forceinline__ void sort_stage(uint64_t (&b)[N], std::integer_sequence<int, I...>)
{
    (sort_ce<N, SIZE, STRIDE, I>(b), ...);
}

template <int N, int SIZE, int STRIDE>
__device__ __forceinline__ void sort_strides(uint64_t (&b)[N])
{
    sort_stage<N, SIZE, STRIDE>(b, std::make_integer_sequence<int, N>{});
    if constexpr (STRIDE > 1) sort_strides<N, SIZE, STRIDE / 2>(b);
}

// Bitonic sorting network, ascending.
template <int N, int SIZE = 2>
__device__ __forceinline__ void bitonic_sort(uint64_t (&b)[N])
{
    if constexpr (SIZE <= N) {
        sort_strides<N, SIZE, SIZE / 2>(b);
        bitonic_sort<N, SIZE * 2>(b);
    }
}

template <int N, int OFF, int STRIDE, int I>
__device__ __forceinline__ void merge_ce(uint64_t (&a)[N])
{
    constexpr int J = I ^ STRIDE;
    if constexpr (J > I) cmp_swap(a[OFF + I], a[OFF + J]);
}

template <int N, int OFF, int STRIDE, int... I>
__device__ __forceinline__ void merge_stage(uint64_t (&a)[N], std::integer_sequence<int, I...>)
{
    (merge_ce<N, OFF, STRIDE, I>(a), ...);
}

// Sort the bitonic run a[OFF .. OFF+LEN) ascending (half-cleaner cascade).
template <int N, int OFF = 0, int LEN = N, int STRIDE = LEN / 2>
__device__ __forceinline__ void bitonic_merge(uint64_t (&a)[N])
{
    if constexpr (STRIDE > 0) {
        merge_stage<N, OFF, STRIDE>(a, std::make_integer_sequence<int, LEN>{});
        bitonic_merge<N, OFF, LEN, STRIDE / 2>(a);
    }
}

// Largest list filled straight from the own leaves (Lane::fill).
constexpr int kFillMaxK = 64;

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
// a[]: the queue is sorted with a sorting network, the lower K keys of
// a[] and the queue are taken with one min against the reversed queue
// (which leaves a bitonic sequence) and a bitonic merge sorts them.
//
// The threshold is min(a[K-1], cap), cap being zero for lanes without a
// query (they never queue anything) and the largest key otherwise.  Between
// merges the threshold may be stale, which only lets more keys into the
// queue.  The excluded object (the issuer of the query) must never enter
// the list: an issuer lies in its own leaf, so it is met only in the first
// sweep, whose candidates are checked by id as they are offered; a free
// centre may exclude any object, so then every merge masks it by id.
template <int K, int P>
struct Selector {
    static constexpr uint32_t kSlotBytes = kWave * sizeof(uint64_t);  // slot stride
    uint64_t a[K];
    lds_u64 *q;        // this lane's queue: q[s * kWave], s < P
    uint32_t q0;       // LDS byte address of slot 0 (that of q)
    uint32_t qnext;    // LDS byte address of the next free slot
    uint64_t cap;      // exclusive upper bound of the keys the lane takes
    uint64_t thr;      // min(a[K-1], cap) at the last merge
    uint32_t excl;     // id of the excluded object (the issuer), or kNoExclude

    __device__ __forceinline__ void init(int k, lds_u64 *lane_queue, uint32_t excl_id)
    {
#pragma unroll
        for (int s = 0; s < K; ++s) a[s] = (s < K - k) ? 0ull : kKeyMax;
        q = lane_queue;
        q0 = (uint32_t)(uintptr_t)lane_queue;
        qnext = q0;
        cap = kKeyMax;
        thr = kKeyMax;
        excl = excl_id;
    }

    __device__ __forceinline__ void set_cap(uint64_t c)
    {
        cap = c;
        thr = key_min(a[K - 1], cap);
    }

    // Keys in the queue.
    __device__ __forceinline__ uint32_t count() const { return (qnext - q0) / kSlotBytes; }
    // Whether the queue holds more than m keys.
    __device__ __forceinline__ bool holds_more_than(uint32_t m) const
    {
        return qnext > q0 + m * kSlotBytes;
    }

    // Every lane writes its key to its next free slot; only lanes whose key
    // passes advance.  No branch, so no lane waits on another's insertion.
    // The slot is tracked by its address, so a write needs no address
    // arithmetic.
    __device__ __forceinline__ void offer(uint64_t key)
    {
        *(lds_u64 *)(uintptr_t)qnext = key;
        qnext += key_less(key, thr) ? kSlotBytes : 0u;
    }

    template <bool MASK_EXCL>
    __device__ __forceinline__ void merge()
    {
        // Read every slot (volatile keeps the loads unconditional: slots
        // past the count hold stale keys).  A stale or excluded key gets the
        // high word of the largest key and keeps its low word: it then lies
        // above every key of a real distance (whose high word is at most
        // that of +inf), so it can only take the place of a largest-key
        // filler of the list, which it equals in every use (threshold,
        // pruning, output; see kFillHi).  One select per slot instead of two.
        const volatile lds_u64 *vq = q;
        const uint32_t cnt = count();
        uint64_t b[P];
#pragma unroll
        for (int s = 0; s < P; ++s) b[s] = vq[s * kWave];
#pragma unroll
        for (int s = 0; s < P; ++s) {
            const uint32_t lo = (uint32_t)b[s];
            const bool keep = (uint32_t)s < cnt && (!MASK_EXCL || lo != excl);
            const uint32_t hi = keep ? (uint32_t)(b[s] >> 32) : kFillHi;
            b[s] = ((uint64_t)hi << 32) | lo;
        }
        oddeven_sort<P>(b);
#pragma unroll
        for (int i = K - P; i < K; ++i) a[i] = key_min(a[i], b[K - 1 - i]);
        if constexpr (K == 2 * P) {
            // a[P .. K) is now bitonic and holds the P smallest of the old
            // upper half and the queue; the whole list is bitonic, and the
            // bitonic merge is its first half-cleaner stage followed by
            // independent merges of the two halves.  If no lane's smallest
            // queued key is below a[P-1], the upper half is already no lower
            // than the lower half: the first stage and the lower merge change
            // nothing and are skipped.
            if (wave_any(key_less(b[0], a[P - 1]))) {
                merge_stage<K, 0, P>(a, std::make_integer_sequence<int, K>{});
                bitonic_merge<K, 0, P>(a);
            }
            bitonic_merge<K, P, P>(a);
        } else {
            bitonic_merge<K>(a);
        }
        qnext = q0;
        thr = key_min(a[K - 1], cap);
    }
};

// FREE: the query has a free centre, whose excluded object may lie in any
// leaf.
template <int K, int P, bool FREE>
struct Lane {
    float qx, qy;
    float pad;   // growth of every node box (drift since the last full build)
    bool active;
    Selector<K, P> sel;
    uint32_t n_cand = 0, n_merge = 0, n_node = 0, n_leaf = 0;  // wave-uniform

    // CHECK: the candidate may be the excluded object; its key then gets
    // the exponent of an infinity (with a nonzero low word it is a NaN,
    // which compares below no threshold), so it is written but not counted.
    template <bool CHECK>
    __device__ __forceinline__ void offer(const Point &p)
    {
        const float d2 = sq_dist(qx, qy, p.x, p.y);
        uint32_t hi = __float_as_uint(d2);
        if constexpr (CHECK) hi = p.id == sel.excl ? 0x7ff00000u : hi;
        sel.offer(((uint64_t)hi << 32) | p.id);
    }

    __device__ __forceinline__ void merge_if(bool full)
    {
        if (wave_any(full)) {
            sel.template merge<FREE>();
            ++n_merge;
        }
    }

    // The list starts from the keys of the first K objects of the own
    // leaves [b, b + K), sorted (K <= kWave: one staged chunk).  With an
    // empty list every key passes, so queueing those objects would fill
    // every queue in a few steps and cost several merges.  The excluded
    // object gets a filler key.  Lanes asking for kq < K keep their K - kq
    // zero sentinels: the kq smallest keys go above them in reverse order,
    // which leaves a bitonic sequence for a bitonic merge to sort.
    __device__ __forceinline__ void fill(const Point *__restrict__ pts, int32_t b, int kq,
                                         Point *stage)
    {
        static_assert(K <= kWave, "one staged chunk");
        const int lane = threadIdx.x & (kWave - 1);
        reinterpret_cast<uint4 *>(stage)[lane] =
            reinterpret_cast<const uint4 *>(pts)[b + min(lane, K - 1)];
        uint64_t (&a)[K] = sel.a;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const Point p = stage[s];
            const float d2 = sq_dist(qx, qy, p.x, p.y);
            const uint32_t hi = p.id == sel.excl ? kFillHi : __float_as_uint(d2);
            a[s] = ((uint64_t)hi << 32) | p.id;
        }
        oddeven_sort<K>(a);
        if (wave_any(kq < K)) {
            const int z = K - kq;  // sentinels
#pragma unroll
            for (int s = 0; s < K / 2; ++s) {
                const uint64_t lo = a[s], hi = a[K - 1 - s];
                a[s] = s < z ? 0ull : hi;
                a[K - 1 - s] = K - 1 - s < z ? 0ull : lo;
            }
            bitonic_merge<K>(a);
        }
        sel.thr = key_min(a[K - 1], sel.cap);
        n_cand += K;
    }

    // Every lane evaluates every object of the sorted range [b, e).  The
    // range is wave-uniform; it is staged through LDS in chunks of 64
    // records (one 16-byte load per lane, the next chunk requested before
    // the current one is evaluated), and each record is then read by all
    // lanes at once (an LDS broadcast), two per step.
    // Invariant between steps (and between sweeps): every queue holds at
    // most P-2 keys, so a step's two writes stay inside the queue; a merge
    // runs as soon as a queue holds more.
    // OWN: the first sweep (the leaves holding the queries' centres).
    template <bool OWN>
    __device__ __forceinline__ void sweep(const Point *__restrict__ pts, int32_t b, int32_t e,
                                          Point *stage)
    {
        constexpr bool CHECK = OWN && !FREE;
        if (b >= e) return;
        n_cand += (uint32_t)(e - b);
        ++n_leaf;
        const int lane = threadIdx.x & (kWave - 1);
        const uint4 *src = reinterpret_cast<const uint4 *>(pts);
        uint4 *dst = reinterpret_cast<uint4 *>(stage);
        uint4 next = src[b + min(lane, e - b - 1)];
        for (int32_t c0 = b; c0 < e; c0 += kWave) {
            const int32_t m = min(kWave, e - c0);
            dst[lane] = next;
            const int32_t c1 = c0 + kWave;
            if (c1 < e) next = src[c1 + min(lane, e - c1 - 1)];
            int32_t j = 0;
            for (; j + 2 <= m; j += 2) {
                const Point p0 = stage[j], p1 = stage[j + 1];
                offer<CHECK>(p0);
                offer<CHECK>(p1);
                merge_if(sel.holds_more_than(P - 2));
            }
            if (j < m) {
                const Point p0 = stage[j];
                offer<CHECK>(p0);
                merge_if(sel.holds_more_than(P - 2));
            }
        }
    }

    // A node is needed if its box may hold a key below some lane's
    // threshold (queued keys are not yet counted, so this errs on the side
    // of visiting).  A lane without a query has a zero threshold and the
    // centre of its tile's last query, which is in the same wavefront: it
    // wants a node only if that box contains the centre, and then so does
    // the lane of that query, so it adds no visit and needs no test of its
    // own.
    // After refit ticks inner boxes are grown by pad; leaf boxes already
    // bound their objects' current positions and are taken as they are.
    __device__ __forceinline__ bool wants(const Node &nd) const
    {
        const float lb = nd.leaf >= 0 ? box_lower_bound_exact(qx, qy, nd)
                                      : box_lower_bound(qx, qy, nd, pad);
        return __float_as_uint(lb) <= (uint32_t)(sel.thr >> 32);
    }
    // The same with unpadded boxes (right after a full build): x - 0 = x, so
    // the bound is identical, with four fewer operations.
    __device__ __forceinline__ bool wants_exact(const Node &nd) const
    {
        return __float_as_uint(box_lower_bound_exact(qx, qy, nd)) <= (uint32_t)(sel.thr >> 32);
    }
};

// Positions only move forward (a skip link never points back) and sweep
// ranges are clamped to the object array, so the walk always terminates
// inside its buffers.
template <int K, int P, bool FREE>
__device__ __forceinline__ int32_t walk_step(Lane<K, P, FREE> &ln, const Node *__restrict__ tab,
                                             int32_t pos, int32_t total,
                                             const Point *__restrict__ pts, int32_t n,
                                             Point *stage)
{
    while (pos < total) {
        const Node nd = tab[pos];
        ++ln.n_node;
        const int32_t next = nd.skip > pos ? nd.skip : pos + 1;
        const bool want = ln.pad == 0.0f ? wave_any(ln.wants_exact(nd)) : wave_any(ln.wants(nd));
        if (!want) {
            pos = next;
            continue;
        }
        if (nd.leaf >= 0) {
            ln.template sweep<false>(pts, max(nd.begin, 0), min(nd.end, n), stage);
            return next;
        }
        ++pos;
    }
    return total;
}

// One wavefront per workgroup, so a finished wavefront frees its registers
// and LDS at once instead of waiting for the slowest wavefront of a larger
// group (wavefront run times differ several-fold between dense and sparse
// regions).  Tiles are dealt to the XCDs as xcd_tile describes.
template <int K, int P, bool FREE>
__global__ __launch_bounds__(kWave) void k_knn_tiles(QueryArgs qa)
{
    __shared__ uint64_t s_queue[P * kWave];
    __shared__ Point s_stage[kWave];
    Point *stage = s_stage;
    const int lane = threadIdx.x;
    // The queries of this launch: all of them, or one k class of them.
    uint32_t q_begin = 0, q_count = qa.nq;
    if (qa.class_bounds) {
        q_begin = qa.class_bounds[qa.klass];
        q_count = qa.class_bounds[qa.klass + 1] - q_begin;
    }
    // Tiles of qt consecutive queries, one per wavefront; lanes from qt on
    // take the tile's last query, like the lanes past the last query.
    const uint32_t qt = qa.tile_queries;
    const uint32_t tiles = (q_count + qt - 1) / qt;
    const uint32_t tile = xcd_tile(blockIdx.x, tiles);
    if (tile >= tiles) return;  // whole wavefront idle
    const uint32_t t = tile * qt + lane;
    const uint32_t tile_last = min(tile * qt + qt, q_count) - 1;

    Lane<K, P, FREE> ln;
    ln.active = (uint32_t)lane < qt && t < q_count;
    // After refit ticks the objects have moved by up to D per axis since the
    // quadrant boxes were made; grow the inner nodes' boxes by D plus a
    // margin that covers the rounding of D and of the grown edges (2^-23 >
    // 2 * 2^-25, the largest rounding error of a difference or a sum below
    // 1).  Leaf boxes are recomputed by the refit and not grown.
    ln.pad = 0.0f;
    {
        const unsigned long long dw = qa.ctr->drift;
        const float d = __uint_as_float((uint32_t)dw);
        if ((uint32_t)(dw >> 32) == qa.build_epoch && d > 0.0f) ln.pad = d + 0x1p-23f;
        // The same in every lane; keep it scalar so the choice of bound per
        // node is a wavefront-uniform branch.
        ln.pad = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(ln.pad)));
    }
    const uint32_t tq = q_begin + (ln.active ? t : tile_last);
    // Query centre, excluded object and sorted position to start from: an
    // object's own position and id, or a free centre's insertion position.
    int32_t qp, row;
    uint32_t excl;
    if (qa.qpts) {
        const QPoint c = qa.qpts[tq];
        ln.qx = c.x;
        ln.qy = c.y;
        excl = c.excl;
        qp = min(max(c.pos, 0), (int32_t)qa.n - 1);
        row = qa.qrow[tq];
    } else {
        qp = qa.qpos ? (int32_t)((uint32_t)qa.qpos[tq] & qa.pos_mask) : (int32_t)tq;
        const Point q = qa.pts[qp];
        ln.qx = q.x;
        ln.qy = q.y;
        excl = q.id;
        row = qa.qrow ? qa.qrow[tq] : (int32_t)q.id;
    }
    int kq = qa.ks ? qa.ks[row] : qa.k_uniform;
    kq = kq < 1 ? 1 : (kq > K ? K : kq);
    ln.sel.init(kq, (lds_u64 *)&s_queue[lane], excl);

    // Lanes without a query keep a zero threshold and never queue anything.
    // (A bound on the k-th key from a few nearby objects, tried as a start
    // threshold, left the merge count unchanged: merges are triggered by
    // whichever lane's queue fills first.)
    ln.sel.set_cap(ln.active ? kKeyMax : 0ull);

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

    // First iteration: the own leaves (their first K objects straight into
    // the list when there are enough of them).
    int32_t own_b = max(qa.leaf_begin[l0], 0);
    const int32_t own_e = min(qa.leaf_end[l1], (int32_t)qa.n);
    if constexpr (K <= kFillMaxK) {
        if (own_e - own_b >= K) {
            ln.fill(qa.pts, own_b, kq, stage);
            own_b += K;
        }
    }
    ln.template sweep<true>(qa.pts, own_b, own_e, stage);

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
            walk_step<K, P, FREE>(ln, fw ? qa.fwd : qa.rev, fw ? rf : rl, total, qa.pts, (int32_t)qa.n,
                            stage);
        rf = fw ? pos : rf;
        rl = fw ? rl : pos;
        right = !right;
    }

    if (wave_any(ln.sel.holds_more_than(0))) {
        ln.sel.template merge<FREE>();
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
    if (kq == K && (off & 3) == 0) {
        // Full-width row starting on a 16-byte boundary: 16-byte stores, so
        // each 128-byte line of the row is written by a few consecutive
        // stores of the lane instead of K separate 4-byte ones.
#pragma unroll
        for (int s = 0; s < K; s += 4) {
            int4 vi;
            float4 vd;
            int32_t *pi = &vi.x;
            float *pd = &vd.x;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint64_t v = ln.sel.a[s + u];
                const bool real = (uint32_t)(v >> 32) < kFillHi;
                pi[u] = real ? (int32_t)(uint32_t)v : -1;
                pd[u] = real ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_inff();
                cnt += real ? 1 : 0;
            }
            *reinterpret_cast<int4 *>(oi + s) = vi;
            *reinterpret_cast<float4 *>(od + s) = vd;
        }
    } else {
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int slot = s - (K - kq);
            if (slot >= 0) {
                const uint64_t v = ln.sel.a[s];
                const bool real = (uint32_t)(v >> 32) < kFillHi;
                oi[slot] = real ? (int32_t)(uint32_t)v : -1;
                od[slot] = real ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_inff();
                cnt += real ? 1 : 0;
            }
        }
    }
    qa.out_cnt[row] = cnt;
}

// ---------------------------------------------------------------------------
// Free-centre queries (Definition 1: q = (x, y, k) with any centre): the
// centres are validated and given level-16 Morton codes, sorted by code with
// the query radix sort, then each is placed among the sorted objects (the
// position its code would take), which gives the wavefront's starting leaf
// and the seed window.  Any starting position is correct -- the two walks
// reach every leaf outside the swept ones -- the code order only keeps the
// wavefront's queries and candidates close together.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t spread16(uint32_t v)
{
    v &= 0x0000ffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__global__ void k_point_keys(const float *__restrict__ qx, const float *__restrict__ qy,
                             const int32_t *__restrict__ exclude, const int32_t *__restrict__ ks,
                             uint32_t nq, uint32_t n, int k_max, uint32_t *__restrict__ keys,
                             uint32_t *__restrict__ vals, uint32_t *__restrict__ kcount,
                             IndexCounters *__restrict__ ctr, uint64_t *__restrict__ ws,
                             int64_t ws_words, uint32_t epoch)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t w = q; w < ws_words; w += (int64_t)gridDim.x * blockDim.x) ws[w] = 0ull;
    if (q >= nq) return;
    const float px = qx[q], py = qy[q];
    const bool ok = (px >= 0.0f) && (px < 1.0f) && (py >= 0.0f) && (py < 1.0f);
    if (!ok) atomicMax(&ctr->bad_centre, epoch);
    const uint32_t cx = min(ok ? (uint32_t)(px * 65536.0f) : 0u, 65535u);
    const uint32_t cy = min(ok ? (uint32_t)(py * 65536.0f) : 0u, 65535u);
    keys[q] = spread16(cx) | (spread16(cy) << 1);
    vals[q] = q;
    if (exclude) {
        const int32_t e = exclude[q];
        if (e < -1 || e >= (int32_t)n) atomicMax(&ctr->bad_issuer, epoch);
    }
    if (ks) {
        const int32_t k = ks[q];
        const bool kok = k >= 1 && k <= k_max;
        if (!kok) atomicMax(&ctr->bad_k, epoch);
        kcount[q] = kok ? (uint32_t)k : 1u;
    }
}

__global__ void k_point_place(const uint32_t *__restrict__ codes, const uint32_t *__restrict__ rows,
                              uint32_t nq, const float *__restrict__ qx,
                              const float *__restrict__ qy, const int32_t *__restrict__ exclude,
                              const Point *__restrict__ pts, uint32_t n,
                              QPoint *__restrict__ qpts)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const uint32_t q = rows[i], code = codes[i];
    // First sorted object whose code is not below the centre's code.
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pts[mid].code < code) lo = mid + 1;
        else hi = mid;
    }
    QPoint c;
    c.x = qx[q];
    c.y = qy[q];
    const int32_t e = exclude ? exclude[q] : -1;
    c.excl = (e >= 0 && e < (int32_t)n) ? (uint32_t)e : kNoExclude;
    c.pos = (int32_t)lo;
    qpts[i] = c;
}

void launch_point_prep(const PointPrep &p, hipStream_t s)
{
    const int T = 256;
    if (p.nq == 0) return;
    k_point_keys<<<(p.nq + T - 1) / T, T, 0, s>>>(p.qx, p.qy, p.exclude, p.ks, p.nq, p.n, p.k_max,
                                                 p.sort.keys[0], p.sort.vals[0], p.kcount, p.ctr,
                                                 p.ws, p.ws_words, p.epoch);
}

void launch_point_place(const uint32_t *codes, const uint32_t *rows, uint32_t nq, const float *qx,
                        const float *qy, const int32_t *exclude, const Point *pts, uint32_t n,
                        QPoint *qpts, hipStream_t s)
{
    const int T = 256;
    if (nq == 0) return;
    k_point_place<<<(nq + T - 1) / T, T, 0, s>>>(codes, rows, nq, qx, qy, exclude, pts, n, qpts);
}

int k_class(int k)
{
    if (k <= 8) return 8;
    if (k <= 16) return 16;
    if (k <= 32) return 32;
    if (k <= 64) return 64;
    return 128;
}

// Queries per wavefront of a lane-flavour launch.  Automatic: 64, halved
// (down to 8) while the halved tiles still fit the wavefronts the GPU holds
// at once for this list size (compute units x 4 SIMDs x the wavefronts per
// SIMD the kernel's registers allow), i.e. while the launch stays a single
// round: its time is then that of its longest wavefront, which shrinks with
// the tile's candidate set.  A per-class launch (query count known only on
// the device) keeps 64.
static uint32_t tile_queries_for(const QueryArgs &qa, int kclass)
{
    if (qa.tile_queries) return qa.tile_queries;
    if (qa.class_bounds) return kWave;
    const uint32_t per_simd = kclass <= 32 ? 4u : kclass == 64 ? 2u : 1u;
    const uint64_t cus = qa.compute_units ? qa.compute_units : 256u;
    const uint64_t slots = cus * 4ull * per_simd;
    uint32_t qt = kWave;
    while (qt > 8 && ((uint64_t)qa.nq + qt / 2 - 1) / (qt / 2) <= slots) qt /= 2;
    return qt;
}

void launch_knn(const QueryArgs &qa_in, int kclass, hipStream_t s)
{
    if (qa_in.nq == 0) return;
    QueryArgs qa = qa_in;
    qa.tile_queries = tile_queries_for(qa_in, kclass);
    const uint32_t tiles = (qa.nq + qa.tile_queries - 1) / qa.tile_queries;
    const uint32_t groups = (tiles + kXcds - 1) / kXcds * kXcds;
    const dim3 grid(groups), block(kWave);
    if (qa.qpts) {
        switch (kclass) {
        case 8: k_knn_tiles<8, 8, true><<<grid, block, 0, s>>>(qa); break;
        case 16: k_knn_tiles<16, 16, true><<<grid, block, 0, s>>>(qa); break;
        case 32: k_knn_tiles<32, 16, true><<<grid, block, 0, s>>>(qa); break;
        case 64: k_knn_tiles<64, 32, true><<<grid, block, 0, s>>>(qa); break;
        default: k_knn_tiles<128, 64, true><<<grid, block, 0, s>>>(qa); break;
        }
        return;
    }
    switch (kclass) {
    case 8: k_knn_tiles<8, 8, false><<<grid, block, 0, s>>>(qa); break;
    case 16: k_knn_tiles<16, 16, false><<<grid, block, 0, s>>>(qa); break;
    case 32: k_knn_tiles<32, 16, false><<<grid, block, 0, s>>>(qa); break;
    case 64: k_knn_tiles<64, 32, false><<<grid, block, 0, s>>>(qa); break;
    default: k_knn_tiles<128, 64, false><<<grid, block, 0, s>>>(qa); break;
    }
}

// ---------------------------------------------------------------------------
// Query indexing for a subset of issuers (Sec. 4.2.1, query indexing): sort
// the queries by their centre's sorted position so wavefronts hold spatial
// neighbours.  Device-supplied issuers and ks are range-checked here.
// ---------------------------------------------------------------------------

// Index of the selection-list size class of a k (classes of 8, 16, 32, 64
// and 128 keys).
__device__ __forceinline__ uint32_t class_index(int k)
{
    return k <= 8 ? 0u : k <= 16 ? 1u : k <= 32 ? 2u : k <= 64 ? 3u : 4u;
}

// Sort keys of the queries: the sorted position of the issuer, and with
// class_shift >= 0 the query's k class above it, so that the sorted
// queries are grouped by class and Morton-ordered within each class (each
// class then runs with its own list size).  Without issuers, query q is
// issued by object q.
__global__ void k_query_keys(const int32_t *__restrict__ issuers, const int32_t *__restrict__ ks,
                             uint32_t nq, uint32_t n, int k_max, const int32_t *__restrict__ inv,
                             int class_shift, uint32_t *__restrict__ keys,
                             uint32_t *__restrict__ vals, uint32_t *__restrict__ kcount,
                             IndexCounters *__restrict__ ctr, uint64_t *__restrict__ ws,
                             int64_t ws_words, uint32_t epoch)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    // The query sort and scan workspace starts at zero.
    for (int64_t w = q; w < ws_words; w += (int64_t)gridDim.x * blockDim.x) ws[w] = 0ull;
    if (q >= nq) return;
    uint32_t cls = 0;
    if (ks) {
        int32_t k = ks[q];
        bool ok = k >= 1 && k <= k_max;
        if (!ok) atomicMax(&ctr->bad_k, epoch);
        kcount[q] = ok ? (uint32_t)k : 1u;
        cls = class_index(ok ? k : 1);
    }
    if (issuers || class_shift >= 0) {
        int32_t s = issuers ? issuers[q] : (int32_t)q;
        bool ok = s >= 0 && (uint32_t)s < n;
        if (!ok) atomicMax(&ctr->bad_issuer, epoch);
        const uint32_t pos = ok ? (uint32_t)inv[s] : 0u;
        keys[q] = class_shift >= 0 ? (pos | (cls << class_shift)) : pos;
        vals[q] = q;
    }
}

// First sorted query of each class (bounds[c] .. bounds[c+1] is class c).
__global__ void k_class_bounds(const uint32_t *__restrict__ keys, uint32_t nq, int class_shift,
                               uint32_t *__restrict__ bounds)
{
    const uint32_t c = threadIdx.x;
    if (c > kQueryClasses) return;
    const uint32_t target = c << class_shift;
    uint32_t lo = 0, hi = nq;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (keys[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    bounds[c] = lo;
}

void launch_class_bounds(const uint32_t *keys, uint32_t nq, int class_shift, uint32_t *bounds,
                         hipStream_t s)
{
    k_class_bounds<<<1, kWave, 0, s>>>(keys, nq, class_shift, bounds);
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
    k_query_keys<<<g, T, 0, s>>>(p.issuers, p.ks, p.nq, p.n, p.k_max, p.inv, p.class_shift,
                                 p.sort.keys[0], p.sort.vals[0], p.kcount, p.ctr, p.ws,
                                 p.ws_words, p.epoch);
}

void launch_offsets(const uint32_t *kcount, uint32_t nq, uint32_t *scan_out, const ScanSpace &sp,
                    uint32_t *total, int64_t *offsets, hipStream_t s)
{
    launch_exclusive_scan(kcount, scan_out, nq, sp, total, s);
    const int T = 256;
    k_widen_offsets<<<(nq + 1 + T - 1) / T, T, 0, s>>>(scan_out, total, nq, offsets);
}

}  // namespace mknn
