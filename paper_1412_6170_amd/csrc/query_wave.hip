// One k-NN query per wavefront: the "coalesced writes" flavour of the
// distance computations (arXiv 1412.6170, Sec. 4.2.1), gfx950.
//
// The paper assigns a query to a warp: its threads check candidates side by
// side, and the list updates are orchestrated for the whole warp with
// ballots through a buffer in shared memory, so that writes are coalesced.
// Here a wavefront answers one query at a time (a few Morton-consecutive
// queries in turn):
//
//   * 64 candidates per step, one per lane, loaded with one coalesced
//     16-byte load per lane straight from the sorted records;
//   * a candidate whose key is below the query's threshold is appended to
//     an LDS buffer: a ballot gives the passing lanes, their rank among
//     them gives each one its slot, and the count advances by the ballot's
//     population -- no atomics, no barrier;
//   * when the buffer is nearly full (and once at the end) it is sorted by
//     a bitonic network spread over the wavefront and merged into the
//     query's list of K = 64 * KPL best keys, held KPL per lane in
//     ascending order across the lanes; the threshold is the list's last
//     key (or the seed bound, if lower);
//   * the candidates are the objects of the query's own leaf (first
//     iteration), then of the leaves the two Morton-order sub-visits reach
//     (Sec. 4.2.2), a subtree being skipped when its box cannot hold a key
//     below the threshold -- the same walk as the one-query-per-lane
//     kernel, for one query;
//   * the final list is written with consecutive lanes holding consecutive
//     slots of the row.
//
// This flavour holds lists of up to 1024 keys (16 per lane), where the
// lane-private lists of query.hip stop at 128; it also answers smaller k
// when asked to (the sweep flavour is a tuning dimension).
//
// Exactness is that of query.hip: d2 = fl(fl(dx*dx) + fl(dy*dy)) with no
// contraction, keys (d2 bits << 32 | id) compared as doubles, boxes
// skipped only when their lower bound is strictly above the threshold.
#include <utility>

#include "mknn_internal.hpp"
#include "query.hpp"
#include "query_device.hpp"

#pragma clang fp contract(off)

namespace mknn {

// Selection state of the wavefront's current query: its K = 64 * KPL best
// keys in the blocked layout, and an LDS buffer of B = 64 * BPL keys that
// candidates below the threshold are appended to.  A query asking for
// k < K keeps K - k zero sentinels at the bottom of the list, so its k-th
// key is always the list's last (an equal real key is indistinguishable
// from a sentinel, so the top k slots are exact either way).
template <int KPL, int BPL>
struct WaveSel {
    static constexpr int K = kWave * KPL;
    static constexpr int B = kWave * BPL;
    static_assert(BPL >= KPL, "the buffer holds at least a list of keys");

    uint64_t a[KPL];
    lds_u64 *buf;
    uint32_t cnt;      // keys in the buffer (wavefront-uniform)
    uint64_t cap;      // exclusive upper bound from the seed window
    uint64_t thr;      // min(k-th key, cap) at the last merge
    uint32_t merges;

    __device__ __forceinline__ void init(int k, lds_u64 *b, int lane)
    {
#pragma unroll
        for (int r = 0; r < KPL; ++r) a[r] = (lane * KPL + r < K - k) ? 0ull : kKeyMax;
        buf = b;
        cnt = 0;
        cap = kKeyMax;
        thr = kKeyMax;
        merges = 0;
    }

    __device__ __forceinline__ void set_cap(uint64_t c)
    {
        cap = c;
        thr = key_min(readlane_key(a[KPL - 1], kWave - 1), cap);
    }

    __device__ __forceinline__ void merge(int lane)
    {
        __syncthreads();  // appended keys visible to every lane
        uint64_t b[BPL];
#pragma unroll
        for (int r = 0; r < BPL; ++r) {
            const uint32_t s = (uint32_t)(lane * BPL + r);
            b[r] = s < cnt ? (uint64_t)buf[s] : kKeyMax;
        }
        net_sort<BPL, kWave * BPL>(b, lane);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < BPL; ++r) buf[lane * BPL + r] = b[r];
        __syncthreads();
        // The K smallest buffered keys, reversed against the list: the
        // element-wise minimum is a bitonic sequence holding the K smallest
        // of both, which the merge network sorts.
#pragma unroll
        for (int r = 0; r < KPL; ++r) a[r] = key_min(a[r], (uint64_t)buf[K - 1 - (lane * KPL + r)]);
        net_merge<KPL, kWave * KPL>(a, lane);
        __syncthreads();  // buffer reads done before new keys are appended
        cnt = 0;
        ++merges;
        thr = key_min(readlane_key(a[KPL - 1], kWave - 1), cap);
    }

    // One candidate per lane (ok: a real candidate, not the excluded object).
    __device__ __forceinline__ void offer(uint64_t key, bool ok, int lane)
    {
        const bool pass = ok && key_less(key, thr);
        const uint64_t m = __ballot(pass);
        if (m) {
            const uint32_t below = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            if (pass) buf[cnt + below] = key;
            cnt += (uint32_t)__popcll(m);
            if (cnt > (uint32_t)(B - kWave)) merge(lane);
        }
    }
};

template <int KPL, int BPL>
struct WaveQuery {
    float qx, qy, pad;
    uint32_t excl;
    WaveSel<KPL, BPL> sel;
    uint32_t n_cand = 0, n_node = 0, n_leaf = 0;

    // Every object of the sorted range [b, e), 64 per step.
    __device__ __forceinline__ void sweep(const Point *__restrict__ pts, int32_t b, int32_t e, int lane)
    {
        if (b >= e) return;
        n_cand += (uint32_t)(e - b);
        ++n_leaf;
        for (int32_t c0 = b; c0 < e; c0 += kWave) {
            const int32_t i = c0 + lane;
            const bool in = i < e;
            const Point p = pts[in ? i : b];
            const float d2 = sq_dist(qx, qy, p.x, p.y);
            sel.offer(((uint64_t)__float_as_uint(d2) << 32) | p.id, in && p.id != excl, lane);
        }
    }

    __device__ __forceinline__ bool wants(const Node &nd) const
    {
        // Leaf boxes after a refit bound their objects as they are.
        const float lb = (pad == 0.0f || nd.leaf >= 0) ? box_lower_bound_exact(qx, qy, nd)
                                                       : box_lower_bound(qx, qy, nd, pad);
        return __float_as_uint(lb) <= (uint32_t)(sel.thr >> 32);
    }

    // The next leaf of the table from pos whose box may hold a key below
    // the threshold is swept; returns the position after it.
    __device__ __forceinline__ int32_t walk_step(const Node *__restrict__ tab, int32_t pos,
                                                 int32_t total, const Point *__restrict__ pts,
                                                 int32_t n, int lane)
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
                sweep(pts, max(nd.begin, 0), min(nd.end, n), lane);
                return next;
            }
            ++pos;
        }
        return total;
    }
};

constexpr int kWaveQueries = 4;  // Morton-consecutive queries per wavefront

template <int KPL, int BPL>
__global__ __launch_bounds__(kWave) void k_knn_wave(QueryArgs qa)
{
    __shared__ uint64_t s_buf[kWave * BPL];
    const int lane = threadIdx.x;
    constexpr int K = kWave * KPL;
    uint32_t q_begin = 0, q_count = qa.nq;
    if (qa.class_bounds) {
        q_begin = qa.class_bounds[qa.klass];
        q_count = qa.class_bounds[qa.klass + 1] - q_begin;
    }
    const uint32_t tiles = (q_count + kWaveQueries - 1) / kWaveQueries;
    const uint32_t tile = xcd_tile(blockIdx.x, tiles);
    if (tile >= tiles) return;

    float pad = 0.0f;
    {
        const unsigned long long dw = qa.ctr->drift;
        const float d = __uint_as_float((uint32_t)dw);
        if ((uint32_t)(dw >> 32) == qa.build_epoch && d > 0.0f) pad = d + 0x1p-23f;
    }
    const int32_t n = (int32_t)qa.n;
    const int32_t total = min((int32_t)qa.ctr->n_nodes, qa.node_cap);
    uint32_t c_cand = 0, c_merge = 0, c_node = 0, c_leaf = 0, c_q = 0;

    for (int qi = 0; qi < kWaveQueries; ++qi) {
        const uint32_t t = tile * kWaveQueries + qi;
        if (t >= q_count) break;
        const uint32_t tq = q_begin + t;
        WaveQuery<KPL, BPL> w;
        w.pad = pad;
        int32_t qp, row;
        if (qa.qpts) {
            const QPoint c = qa.qpts[tq];
            w.qx = c.x;
            w.qy = c.y;
            w.excl = c.excl;
            qp = min(max(c.pos, 0), n - 1);
            row = qa.qrow[tq];
        } else {
            qp = qa.qpos ? (int32_t)((uint32_t)qa.qpos[tq] & qa.pos_mask) : (int32_t)tq;
            const Point q = qa.pts[qp];
            w.qx = q.x;
            w.qy = q.y;
            w.excl = q.id;
            row = qa.qrow ? qa.qrow[tq] : (int32_t)q.id;
        }
        int kq = qa.ks ? qa.ks[row] : qa.k_uniform;
        kq = kq < 1 ? 1 : (kq > K ? K : kq);
        w.sel.init(kq, (lds_u64 *)s_buf, lane);

        // Seed: the kq + 1 sorted positions around qp hold at least kq
        // objects other than the excluded one; the largest of their keys
        // bounds the k-th key from above.
        if (n - 1 >= kq) {
            int32_t w0 = qp - kq / 2;
            w0 = w0 < 0 ? 0 : (w0 > n - 1 - kq ? n - 1 - kq : w0);
            uint64_t seed = 0;
            for (int32_t s = lane; s <= kq; s += kWave) {
                const Point p = qa.pts[w0 + s];
                const float d2 = sq_dist(w.qx, w.qy, p.x, p.y);
                const uint64_t key = ((uint64_t)__float_as_uint(d2) << 32) | p.id;
                seed = key_max(seed, p.id != w.excl ? key : 0ull);
            }
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) seed = key_max(seed, shfl_xor_key(seed, d));
            w.sel.set_cap(seed + 1);
        }

        // First iteration: the own leaf; then the two sub-visits in turn.
        const int32_t leaf = qa.leaf_of[qp];
        w.sweep(qa.pts, max(qa.leaf_begin[leaf], 0), min(qa.leaf_end[leaf], n), lane);
        int32_t rf = qa.leaf_node_f[leaf] + 1;
        int32_t rl = qa.leaf_node_r[leaf] + 1;
        rf = (rf < 1 || rf > total) ? total : rf;
        rl = (rl < 1 || rl > total) ? total : rl;
        bool right = true;
        while (rf < total || rl < total) {
            const bool fw = (right && rf < total) || rl >= total;
            const int32_t pos = w.walk_step(fw ? qa.fwd : qa.rev, fw ? rf : rl, total, qa.pts, n, lane);
            rf = fw ? pos : rf;
            rl = fw ? rl : pos;
            right = !right;
        }
        if (w.sel.cnt > 0) w.sel.merge(lane);

        // The row: slots K - kq .. K - 1 of the list, consecutive lanes
        // writing consecutive slots.
        const int64_t off = qa.row_off ? qa.row_off[row] : (int64_t)row * qa.k_uniform;
        int32_t *__restrict__ oi = qa.out_ids + off;
        float *__restrict__ od = qa.out_d2 + off;
        int cnt = 0;
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
            const int slot = lane * KPL + r - (K - kq);
            if (slot >= 0) {
                const uint64_t v = w.sel.a[r];
                const bool real = v != kKeyMax;
                oi[slot] = real ? (int32_t)(uint32_t)v : -1;
                od[slot] = real ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_inff();
                cnt += real ? 1 : 0;
            }
        }
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) cnt += __shfl_xor(cnt, d, kWave);
        if (lane == 0) qa.out_cnt[row] = cnt;
        c_cand += w.n_cand;
        c_merge += w.sel.merges;
        c_node += w.n_node;
        c_leaf += w.n_leaf;
        ++c_q;
    }
    if (qa.counters && lane == 0) {
        atomicAdd(&qa.counters[0], (unsigned long long)c_cand);
        atomicAdd(&qa.counters[1], (unsigned long long)c_merge);
        atomicAdd(&qa.counters[2], (unsigned long long)c_node);
        atomicAdd(&qa.counters[3], (unsigned long long)c_leaf);
        atomicAdd(&qa.counters[4], (unsigned long long)c_q);
    }
}

int k_class_wave(int k)
{
    if (k <= 64) return 64;
    if (k <= 128) return 128;
    if (k <= 256) return 256;
    if (k <= 512) return 512;
    return 1024;
}

void launch_knn_wave(const QueryArgs &qa, int kclass, hipStream_t s)
{
    if (qa.nq == 0) return;
    const uint32_t tiles = (qa.nq + kWaveQueries - 1) / kWaveQueries;
    const uint32_t groups = (tiles + kXcds - 1) / kXcds * kXcds;
    const dim3 grid(groups), block(kWave);
    switch (kclass) {
    case 64: k_knn_wave<1, 4><<<grid, block, 0, s>>>(qa); break;
    case 128: k_knn_wave<2, 4><<<grid, block, 0, s>>>(qa); break;
    case 256: k_knn_wave<4, 4><<<grid, block, 0, s>>>(qa); break;
    case 512: k_knn_wave<8, 8><<<grid, block, 0, s>>>(qa); break;
    default: k_knn_wave<16, 16><<<grid, block, 0, s>>>(qa); break;
    }
}

}  // namespace mknn
