// A group of G lanes per k-NN query: the query's list is spread over the
// group, so lists of 64 and 128 keys do not take all registers (arXiv
// 1412.6170, Sec. 4.2.1, the "coalesced writes" flavour of the distance
// computations, with a query per group of lanes instead of a warp), gfx950.
//
// A wavefront answers 64 / G Morton-consecutive queries.  The list of query
// g holds its K = 16 G best keys (d2 bits << 32 | id) in the blocked layout
// over the group's lanes: key i in lane i / 16 of the group, register i % 16,
// ascending; its last key (lane G-1, register 15) is the k-th.  The
// candidates are the wavefront's (the union of what its queries need, as in
// query.hip): 64 records at a time are staged in LDS, and each step deals G
// of them to every group, one per lane, so a query sees 64 candidates in
// 64 / G steps.  A lane appends a candidate below its query's threshold to
// a private LDS queue of 16 slots without branching; when some queue is
// full -- and once at the end -- every group merges: the group's 16 G
// queued keys are sorted by a bitonic network spread over its lanes (cross-
// lane stages exchange registers with the lane whose index differs in one
// bit), the k-th smallest of list and queue are taken with one minimum of
// the list against the reversed sorted queue (a bitonic sequence), and a
// bitonic merge over the group sorts the list again.
//
// The walk, the pruning and the exactness arguments are those of query.hip:
// d2 = fl(fl(dx*dx) + fl(dy*dy)) with no contraction, boxes skipped only when
// their lower bound is strictly above every lane's threshold, keys compared
// as doubles, the issuer excluded by id in the first sweep (free centres:
// at every merge).
#include <utility>

#include "mknn_internal.hpp"
#include "query.hpp"
#include "query_device.hpp"

#pragma clang fp contract(off)

namespace mknn {

constexpr int kGroupPL = 16;  // list keys per lane = queue slots per lane

// The sorted runs of PL keys held by the lanes of a group of G lanes become
// one sorted sequence over the group, runs of H lanes merging pairwise at
// each level: the half-cleaner of two sorted runs pairs element i of the
// lower run with element H PL - 1 - i of the upper one, which sits in lane
// r ^ (2H - 1), register PL - 1 - s; the lower run keeps the minima and the
// upper the maxima (reversed, so both are bitonic), then a bitonic merge
// over each run's H lanes sorts it.  Every direction is fixed at compile
// time except which side a lane keeps.
template <int PL, int H, int G>
__device__ __forceinline__ void merge_runs(uint64_t (&b)[PL], int r)
{
    if constexpr (H < G) {
        const bool lower = (r & H) == 0;
#pragma unroll
        for (int s = 0; s < PL / 2; ++s) {
            const uint64_t w1 = xor_key<2 * H - 1>(b[PL - 1 - s]);
            const uint64_t w2 = xor_key<2 * H - 1>(b[s]);
            // Both results, then a select (a choice between two asm
            // statements compiles to a branch around each).
            const uint64_t lo1 = key_min(b[s], w1), hi1 = key_max(b[s], w1);
            const uint64_t lo2 = key_min(b[PL - 1 - s], w2), hi2 = key_max(b[PL - 1 - s], w2);
            b[s] = lower ? lo1 : hi1;
            b[PL - 1 - s] = lower ? lo2 : hi2;
        }
        net_merge<PL, H * PL>(b, r);
        merge_runs<PL, 2 * H, G>(b, r);
    }
}

template <int G, bool FREE>
struct GroupQuery {
    static constexpr int PL = kGroupPL;
    static constexpr int K = G * PL;

    uint64_t a[PL];    // this lane's part of the list
    lds_u64 *q;        // this lane's queue: q[s * kWave], s < PL
    static constexpr uint32_t kSlotBytes = kWave * sizeof(uint64_t);  // slot stride
    uint32_t q0;       // LDS byte address of slot 0 (that of q)
    uint32_t qnext;    // LDS byte address of this lane's next free slot
    uint64_t cap;      // zero for lanes without a query, else the largest key
    uint64_t thr;      // min(the list's last key, cap) at the last merge
    uint32_t excl;     // the excluded object, or kNoExclude
    float qx, qy, pad;
    bool active;       // the lane's group has a query
    int r;             // index of the lane in its group
    int last_lane;     // lane holding the list's last key
    uint32_t n_cand = 0, n_merge = 0, n_node = 0, n_leaf = 0;  // wave-uniform

    __device__ __forceinline__ void init(int k, lds_u64 *lane_queue, uint32_t excl_id, int lane,
                                         bool has_query)
    {
        r = lane & (G - 1);
        last_lane = (lane & ~(G - 1)) + G - 1;
#pragma unroll
        for (int s = 0; s < PL; ++s) a[s] = (r * PL + s < K - k) ? 0ull : kKeyMax;
        q = lane_queue;
        q0 = (uint32_t)(uintptr_t)lane_queue;
        qnext = q0;
        active = has_query;
        cap = has_query ? kKeyMax : 0ull;
        thr = cap;
        excl = excl_id;
    }

    __device__ __forceinline__ uint32_t count() const { return (qnext - q0) / kSlotBytes; }
    __device__ __forceinline__ bool holds_more_than(uint32_t m) const
    {
        return qnext > q0 + m * kSlotBytes;
    }

    // One candidate: written to the next free slot, counted if it passes.
    __device__ __forceinline__ void offer(uint64_t key)
    {
        *(lds_u64 *)(uintptr_t)qnext = key;
        qnext += key_less(key, thr) ? kSlotBytes : 0u;
    }

    __device__ __forceinline__ void merge()
    {
        const volatile lds_u64 *vq = q;
        uint64_t b[PL];
#pragma unroll
        for (int s = 0; s < PL; ++s) b[s] = vq[s * kWave];
        // Stale and excluded keys get the filler high word (as in the lane
        // flavour's merge).
        const uint32_t cnt = count();
#pragma unroll
        for (int s = 0; s < PL; ++s) {
            const uint32_t lo = (uint32_t)b[s];
            const bool keep = (uint32_t)s < cnt && (!FREE || lo != excl);
            const uint32_t hi = keep ? (uint32_t)(b[s] >> 32) : kFillHi;
            b[s] = ((uint64_t)hi << 32) | lo;
        }
        // The group's queued keys, sorted over the group: each lane's run,
        // then the runs merged.
        oddeven_sort<PL>(b);
        merge_runs<PL, 1, G>(b, r);
        // Key i of the list against key K-1-i of the sorted queue, which sits
        // in the mirrored lane of the group, mirrored register.
#pragma unroll
        for (int s = 0; s < PL; ++s) a[s] = key_min(a[s], xor_key<G - 1>(b[PL - 1 - s]));
        net_merge<PL, K>(a, r);
        qnext = q0;
        thr = key_min(shfl_key(a[PL - 1], last_lane), cap);
    }

    __device__ __forceinline__ void merge_if(bool full)
    {
        if (wave_any(full)) {
            merge();
            ++n_merge;
        }
    }

    // The list starts from the keys of the first K objects of the own
    // leaves [b, b + K), sorted over the group, instead of from a first
    // merge of queues that every key passes.  Lane r of a group reads
    // objects s G + r (consecutive lanes, consecutive records).  The
    // excluded object gets a filler key.  Groups asking for kq < K keep
    // K - kq zero sentinels: the kq smallest keys go above them in reverse
    // order (mirrored lane, mirrored register), and a bitonic merge over
    // the group sorts the result.  (Starting from fewer objects, with
    // fillers for the rest, measured slower: the threshold stays open and
    // the first merge still comes.)
    __device__ __forceinline__ void fill(const Point *__restrict__ pts, int32_t b, int kq)
    {
#pragma unroll
        for (int s = 0; s < PL; ++s) {
            const Point p = pts[b + s * G + r];
            const float d2 = sq_dist(qx, qy, p.x, p.y);
            const uint32_t hi = p.id == excl ? kFillHi : __float_as_uint(d2);
            a[s] = ((uint64_t)hi << 32) | p.id;
        }
        oddeven_sort<PL>(a);
        merge_runs<PL, 1, G>(a, r);
        if (wave_any(kq < K)) {
            const int z = K - kq;  // sentinels
#pragma unroll
            for (int s = 0; s < PL / 2; ++s) {
                // Key K-1-i for i = r PL + s and for i = r PL + PL-1-s.
                const uint64_t m1 = xor_key<G - 1>(a[PL - 1 - s]);
                const uint64_t m2 = xor_key<G - 1>(a[s]);
                a[s] = r * PL + s < z ? 0ull : m1;
                a[PL - 1 - s] = r * PL + PL - 1 - s < z ? 0ull : m2;
            }
            net_merge<PL, K>(a, r);
        }
        thr = key_min(shfl_key(a[PL - 1], last_lane), cap);
        n_cand += (uint32_t)K;
    }

    // Every object of the sorted range [b, e): 64 records at a time staged in
    // LDS, G of them per step to every group (lane r of a group takes record
    // step * G + r).  Lanes past the range offer a key that passes no
    // threshold.  Between steps every queue holds at most PL - 1 keys.
    template <bool OWN>
    __device__ __forceinline__ void sweep(const Point *__restrict__ pts, int32_t b, int32_t e,
                                          Point *stage, int lane)
    {
        if (b >= e) return;
        constexpr bool CHECK = OWN && !FREE;
        n_cand += (uint32_t)(e - b);
        ++n_leaf;
        const uint4 *src = reinterpret_cast<const uint4 *>(pts);
        uint4 *dst = reinterpret_cast<uint4 *>(stage);
        uint4 next = src[b + min(lane, e - b - 1)];
        for (int32_t c0 = b; c0 < e; c0 += kWave) {
            const int32_t m = min(kWave, e - c0);
            dst[lane] = next;
            const int32_t c1 = c0 + kWave;
            if (c1 < e) next = src[c1 + min(lane, e - c1 - 1)];
            const int32_t steps = (m + G - 1) / G;
            for (int32_t j = 0; j < steps; ++j) {
                const int32_t i = j * G + r;
                const Point p = stage[i < m ? i : 0];
                const float d2 = sq_dist(qx, qy, p.x, p.y);
                uint32_t hi = __float_as_uint(d2);
                // A key with an infinity's exponent (an infinity or a NaN as a
                // double) passes no threshold.
                hi = i < m ? hi : 0x7ff00000u;
                if constexpr (CHECK) hi = p.id == excl ? 0x7ff00000u : hi;
                offer(((uint64_t)hi << 32) | p.id);
                merge_if(holds_more_than(PL - 1));
            }
        }
    }

    // Groups without a query have a zero threshold and the centre of the
    // launch's last query, whose group is in the same wavefront, so they
    // add no visit (see the lane flavour) and are not tested apart.
    __device__ __forceinline__ bool wants(const Node &nd) const
    {
        // Leaf boxes after a refit bound their objects as they are.
        const float lb = (pad == 0.0f || nd.leaf >= 0) ? box_lower_bound_exact(qx, qy, nd)
                                                       : box_lower_bound(qx, qy, nd, pad);
        return __float_as_uint(lb) <= (uint32_t)(thr >> 32);
    }

    // The next leaf of the table from pos that some lane wants is swept;
    // returns the position after it (or total).
    __device__ __forceinline__ int32_t walk_step(const Node *__restrict__ tab, int32_t pos,
                                                 int32_t total, const Point *__restrict__ pts,
                                                 int32_t n, Point *stage, int lane)
    {
        while (pos < total) {
            const Node nd = tab[pos];
            ++n_node;
            const int32_t next = nd.skip > pos ? nd.skip : pos + 1;
            if (!wave_any(wants(nd))) {
                pos = next;
                continue;
            }
            if (nd.leaf >= 0) {
                sweep<false>(pts, max(nd.begin, 0), min(nd.end, n), stage, lane);
                return next;
            }
            ++pos;
        }
        return total;
    }
};

// One wavefront per workgroup, tiles of 64 / G queries dealt to the XCDs as
// in query.hip.
template <int G, bool FREE>
__global__ __launch_bounds__(kWave) void k_knn_group(QueryArgs qa)
{
    constexpr int QW = kWave / G;
    constexpr int PL = kGroupPL;
    constexpr int K = G * PL;
    __shared__ uint64_t s_queue[PL * kWave];
    __shared__ Point s_stage[kWave];
    const int lane = threadIdx.x;
    uint32_t q_begin = 0, q_count = qa.nq;
    if (qa.class_bounds) {
        q_begin = qa.class_bounds[qa.klass];
        q_count = qa.class_bounds[qa.klass + 1] - q_begin;
    }
    const uint32_t tiles = (q_count + QW - 1) / QW;
    const uint32_t tile = xcd_tile(blockIdx.x, tiles);
    if (tile >= tiles) return;  // whole wavefront idle
    const uint32_t t = tile * QW + (uint32_t)(lane / G);
    const bool active = t < q_count;

    GroupQuery<G, FREE> w;
    // Drift since the last full build (refit ticks), as in query.hip.
    w.pad = 0.0f;
    {
        const unsigned long long dw = qa.ctr->drift;
        const float d = __uint_as_float((uint32_t)dw);
        if ((uint32_t)(dw >> 32) == qa.build_epoch && d > 0.0f) w.pad = d + 0x1p-23f;
        w.pad = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(w.pad)));
    }
    const uint32_t tq = q_begin + (active ? t : q_count - 1);
    int32_t qp, row;
    uint32_t excl;
    if (qa.qpts) {
        const QPoint c = qa.qpts[tq];
        w.qx = c.x;
        w.qy = c.y;
        excl = c.excl;
        qp = min(max(c.pos, 0), (int32_t)qa.n - 1);
        row = qa.qrow[tq];
    } else {
        qp = qa.qpos ? (int32_t)((uint32_t)qa.qpos[tq] & qa.pos_mask) : (int32_t)tq;
        const Point q = qa.pts[qp];
        w.qx = q.x;
        w.qy = q.y;
        excl = q.id;
        row = qa.qrow ? qa.qrow[tq] : (int32_t)q.id;
    }
    int kq = qa.ks ? qa.ks[row] : qa.k_uniform;
    kq = kq < 1 ? 1 : (kq > K ? K : kq);
    w.init(kq, (lds_u64 *)&s_queue[lane], excl, lane, active);

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
    if (own_e - own_b >= K) {
        w.fill(qa.pts, own_b, kq);
        own_b += K;
    }
    w.template sweep<true>(qa.pts, own_b, own_e, s_stage, lane);

    // Subsequent iterations: the two Morton-order sub-visits in turn.
    const int32_t total = min((int32_t)qa.ctr->n_nodes, qa.node_cap);
    int32_t rf = qa.leaf_node_f[l1] + 1;
    int32_t rl = qa.leaf_node_r[l0] + 1;
    rf = (rf < 1 || rf > total) ? total : rf;
    rl = (rl < 1 || rl > total) ? total : rl;
    bool right = true;
    while (rf < total || rl < total) {
        const bool fw = (right && rf < total) || rl >= total;
        const int32_t pos = w.walk_step(fw ? qa.fwd : qa.rev, fw ? rf : rl, total, qa.pts,
                                        (int32_t)qa.n, s_stage, lane);
        rf = fw ? pos : rf;
        rl = fw ? rl : pos;
        right = !right;
    }
    if (wave_any(w.holds_more_than(0))) {
        w.merge();
        ++w.n_merge;
    }
    if (qa.counters && lane == 0) {
        atomicAdd(&qa.counters[0], (unsigned long long)w.n_cand);
        atomicAdd(&qa.counters[1], (unsigned long long)w.n_merge);
        atomicAdd(&qa.counters[2], (unsigned long long)w.n_node);
        atomicAdd(&qa.counters[3], (unsigned long long)w.n_leaf);
        atomicAdd(&qa.counters[4], 1ull);
    }

    // The row: list slots K - kq .. K - 1, lane r of the group holding slots
    // 16 r .. 16 r + 15 of the list.
    int cnt = 0;
    if (active) {
        const int64_t off = qa.row_off ? qa.row_off[row] : (int64_t)row * qa.k_uniform;
        int32_t *__restrict__ oi = qa.out_ids + off;
        float *__restrict__ od = qa.out_d2 + off;
        const int first = w.r * PL - (K - kq);  // row slot of a[0]
        if (kq == K && (off & 3) == 0) {
#pragma unroll
            for (int s = 0; s < PL; s += 4) {
                int4 vi;
                float4 vd;
                int32_t *pi = &vi.x;
                float *pd = &vd.x;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint64_t v = w.a[s + u];
                    const bool real = (uint32_t)(v >> 32) < kFillHi;
                    pi[u] = real ? (int32_t)(uint32_t)v : -1;
                    pd[u] = real ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_inff();
                    cnt += real ? 1 : 0;
                }
                *reinterpret_cast<int4 *>(oi + first + s) = vi;
                *reinterpret_cast<float4 *>(od + first + s) = vd;
            }
        } else {
#pragma unroll
            for (int s = 0; s < PL; ++s) {
                const int slot = first + s;
                if (slot >= 0) {
                    const uint64_t v = w.a[s];
                    const bool real = (uint32_t)(v >> 32) < kFillHi;
                    oi[slot] = real ? (int32_t)(uint32_t)v : -1;
                    od[slot] = real ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_inff();
                    cnt += real ? 1 : 0;
                }
            }
        }
    }
#pragma unroll
    for (int d = 1; d < G; d <<= 1) cnt += __shfl_xor(cnt, d, kWave);
    if (active && w.r == 0) qa.out_cnt[row] = cnt;
}

int k_class_group(int k)
{
    if (k <= 32) return 32;
    if (k <= 64) return 64;
    if (k <= 128) return 128;
    if (k <= 256) return 256;
    if (k <= 512) return 512;
    return 1024;
}

template <bool FREE>
static void launch_group(const QueryArgs &qa, int kclass, hipStream_t s)
{
    const int G = kclass / kGroupPL;
    const uint32_t per = kWave / G;
    const uint32_t tiles = (qa.nq + per - 1) / per;
    const uint32_t groups = (tiles + kXcds - 1) / kXcds * kXcds;
    const dim3 grid(groups), block(kWave);
    switch (G) {
    case 2: k_knn_group<2, FREE><<<grid, block, 0, s>>>(qa); break;
    case 4: k_knn_group<4, FREE><<<grid, block, 0, s>>>(qa); break;
    case 8: k_knn_group<8, FREE><<<grid, block, 0, s>>>(qa); break;
    case 16: k_knn_group<16, FREE><<<grid, block, 0, s>>>(qa); break;
    case 32: k_knn_group<32, FREE><<<grid, block, 0, s>>>(qa); break;
    default: k_knn_group<64, FREE><<<grid, block, 0, s>>>(qa); break;
    }
}

void launch_knn_group(const QueryArgs &qa, int kclass, hipStream_t s)
{
    if (qa.nq == 0) return;
    if (qa.qpts) launch_group<true>(qa, kclass, s);
    else launch_group<false>(qa, kclass, s);
}

}  // namespace mknn
