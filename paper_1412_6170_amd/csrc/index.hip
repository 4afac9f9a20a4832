// Index build for one tick (arXiv 1412.6170, Sec. 4.1), gfx950.
//
//   k_morton         level-16 Morton code per object (the virtual full
//                    quadtree at l_max = 16), x cell in the even bits;
//                    device-side range validation
//   radix sort       stable LSD sort of (code, id), 8-bit digits, tiles
//                    staged in LDS and written back in digit runs
//   k_gather         sorted objects as 16-byte records {x, y, id, code}
//   k_leaf_flags     which adjacent sorted objects fall in different leaves
//   k_leaf_emit      leaf ranges from the flags' exclusive scan
//   k_leaf_info      leaf level and the node count each leaf contributes
//   k_node_emit      depth-first node tables (forward and backward) with
//                    subtree-skip links, for stackless Morton-order walks
//
// The paper builds the tree level by level with a CPU decision per level;
// here every step stays on the device.  A quadrant (level l, prefix P) is
// split iff it holds more than th objects and l < L.  Because objects are
// sorted by code, the objects of any quadrant form one contiguous run
// (ancestor property, Sec. 4.1), so the leaf structure is decided pairwise:
// sorted objects i and i+1 lie in different leaves iff the deepest quadrant
// containing both (level c = their common-prefix level) is split, i.e. iff
// c < L and that quadrant holds more than th objects.  A leaf's level is
// one below the deeper of the two quadrants that separate it from its
// neighbours, or L when it still holds more than th objects.
#include "mknn_internal.hpp"

#pragma clang fp contract(off)

namespace mknn {

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t spread_bits16(uint32_t v)
{
    v &= 0x0000ffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ __forceinline__ uint32_t compact_bits16(uint32_t v)
{
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0f0f0f0fu;
    v = (v | (v >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0x0000ffffu;
    return v;
}

// Level of the deepest quadrant holding both codes (16 if equal).
__device__ __forceinline__ int common_level(uint32_t a, uint32_t b)
{
    uint32_t d = a ^ b;
    return d == 0 ? kCodeLevels : (__clz(d) >> 1);
}

// Do codes a and b lie in the same level-l quadrant?
__device__ __forceinline__ bool same_quadrant(uint32_t a, uint32_t b, int l)
{
    return l <= 0 || ((a ^ b) >> (2 * (kCodeLevels - l))) == 0;
}

__device__ __forceinline__ uint32_t quadrant_of(uint32_t code, int l)
{
    return l <= 0 ? 0u : code >> (2 * (kCodeLevels - l));
}

// Inclusive scan across one wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan across a workgroup of NT threads; *total gets the sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total)
{
    constexpr int NW = NT / kWave;
    __shared__ uint32_t s_w[NW];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        uint32_t t = s_w[i];
        before += (i < w) ? t : 0u;
        all += t;
    }
    __syncthreads();
    if (total) *total = all;
    return before + inc - v;
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of uint32 (three launches)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *__restrict__ in,
                                                             uint32_t n,
                                                             uint32_t *__restrict__ sums,
                                                             const uint32_t *__restrict__ n_dev)
{
    if (n_dev) n = min(n, *n_dev);
    const uint32_t base = blockIdx.x * (uint32_t)kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        uint32_t p = base + j * kScanThreads + threadIdx.x;
        s += (p < n) ? in[p] : 0u;
    }
    uint32_t total;
    block_excl_scan<kScanThreads>(s, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t *__restrict__ sums, uint32_t nb,
                                                  uint32_t *__restrict__ total_out)
{
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += 1024u * 4u) {
        uint32_t v[4], s = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t p = base + threadIdx.x * 4u + j;
            v[j] = (p < nb) ? sums[p] : 0u;
            s += v[j];
        }
        uint32_t tot;
        uint32_t pre = block_excl_scan<1024>(s, &tot) + carry;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t p = base + threadIdx.x * 4u + j;
            if (p < nb) sums[p] = pre;
            pre += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t *in, uint32_t *out,
                                                           uint32_t n,
                                                           const uint32_t *__restrict__ sums,
                                                           const uint32_t *__restrict__ n_dev)
{
    if (n_dev) n = min(n, *n_dev);
    if (blockIdx.x * (uint32_t)kScanTile >= n) return;
    // Blocked arrangement: thread t owns kScanItems consecutive elements.
    const uint32_t base = blockIdx.x * (uint32_t)kScanTile + threadIdx.x * (uint32_t)kScanItems;
    uint32_t v[kScanItems], s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        uint32_t p = base + j;
        v[j] = (p < n) ? in[p] : 0u;
        s += v[j];
    }
    uint32_t pre = block_excl_scan<kScanThreads>(s, nullptr) + sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        uint32_t p = base + j;
        if (p < n) out[p] = pre;
        pre += v[j];
    }
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__global__ void k_store_zero(uint32_t *p) { *p = 0u; }

void launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                           uint32_t *total, hipStream_t s, const uint32_t *n_dev)
{
    if (n <= 0) {
        if (total) k_store_zero<<<1, 1, 0, s>>>(total);
        return;
    }
    uint32_t nb = (uint32_t)((n + kScanTile - 1) / kScanTile);
    k_scan_reduce<<<nb, kScanThreads, 0, s>>>(in, (uint32_t)n, tmp, n_dev);
    k_scan_top<<<1, 1024, 0, s>>>(tmp, nb, total);
    k_scan_down<<<nb, kScanThreads, 0, s>>>(in, out, (uint32_t)n, tmp, n_dev);
}

// ---------------------------------------------------------------------------
// Morton codes (Sec. 4.1: quadrants of the virtual full quadtree at l_max)
// ---------------------------------------------------------------------------

__global__ void k_morton(const float *__restrict__ x, const float *__restrict__ y, uint32_t n,
                         uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                         IndexCounters *__restrict__ ctr)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float px = x[i], py = y[i];
    // NaN fails both comparisons; -0.0 passes.
    bool ok = (px >= 0.0f) && (px < 1.0f) && (py >= 0.0f) && (py < 1.0f);
    if (!ok) atomicOr(&ctr->bad_input, 1u);
    // Scaling by 2^16 is exact; truncation is the floor for x >= 0.  The
    // clamp only matters for rejected input.
    uint32_t cx = ok ? (uint32_t)(px * 65536.0f) : 0u;
    uint32_t cy = ok ? (uint32_t)(py * 65536.0f) : 0u;
    cx = min(cx, 65535u);
    cy = min(cy, 65535u);
    keys[i] = spread_bits16(cx) | (spread_bits16(cy) << 1);
    vals[i] = i;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                            uint32_t n, int shift,
                                                            uint32_t *__restrict__ hist,
                                                            uint32_t ntiles)
{
    __shared__ uint32_t s_h[kRadixBins];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * (uint32_t)kSortTile;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        uint32_t p = base + j * kSortThreads + threadIdx.x;
        if (p < n) atomicAdd(&s_h[(keys[p] >> shift) & (kRadixBins - 1)], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * ntiles + blockIdx.x] = s_h[threadIdx.x];
}

// Each tile is ranked stably in LDS (rounds of 256 keys in position order;
// within a wavefront, lanes holding the same digit are found with ballots),
// reordered by digit in LDS, then written to its global digit offsets in
// contiguous runs.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
    uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out, uint32_t n, int shift,
    const uint32_t *__restrict__ offs, uint32_t ntiles)
{
    constexpr int NW = kSortThreads / kWave;
    __shared__ uint32_t s_keys[kSortTile];
    __shared__ uint32_t s_vals[kSortTile];
    __shared__ uint32_t s_start[kRadixBins];
    __shared__ uint32_t s_run[kRadixBins];
    __shared__ uint32_t s_wcnt[NW][kRadixBins];
    __shared__ uint32_t s_wbase[NW][kRadixBins];

    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const uint32_t base = blockIdx.x * (uint32_t)kSortTile;
    const uint32_t n_valid = min((uint32_t)kSortTile, n - base);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));

    uint32_t key[kSortItems], val[kSortItems];
    int dig[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        uint32_t p = j * kSortThreads + t;
        bool v = p < n_valid;
        key[j] = v ? keys_in[base + p] : 0xffffffffu;
        val[j] = v ? vals_in[base + p] : 0u;
        // Padding takes the last digit; it sits at the end of the tile's
        // position order, so it ranks after every real key.
        dig[j] = v ? (int)((key[j] >> shift) & (kRadixBins - 1)) : kRadixBins - 1;
    }

    s_start[t] = 0;
    s_run[t] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) atomicAdd(&s_start[dig[j]], 1u);
    __syncthreads();
    uint32_t cnt = s_start[t];
    __syncthreads();
    s_start[t] = block_excl_scan<kSortThreads>(cnt, nullptr);

#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int d = dig[j];
        uint64_t peers = ~0ull;
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            uint64_t m = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
#pragma unroll
        for (int q = 0; q < NW; ++q) s_wcnt[q][t] = 0;
        __syncthreads();
        if (rank == 0) s_wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t r = s_run[t];
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                s_wbase[q][t] = r;
                r += s_wcnt[q][t];
            }
            s_run[t] = r;
        }
        __syncthreads();
        const uint32_t local = s_start[d] + s_wbase[w][d] + rank;
        s_keys[local] = key[j];
        s_vals[local] = val[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        uint32_t lp = j * kSortThreads + t;
        if (lp < n_valid) {
            uint32_t k = s_keys[lp];
            uint32_t d = (k >> shift) & (kRadixBins - 1);
            uint32_t dst = offs[d * ntiles + blockIdx.x] + (lp - s_start[d]);
            keys_out[dst] = k;
            vals_out[dst] = s_vals[lp];
        }
    }
}

int64_t radix_hist_elems(int64_t n)
{
    int64_t tiles = (n + kSortTile - 1) / kSortTile;
    return (tiles > 0 ? tiles : 1) * kRadixBins;
}

int launch_radix_sort(const SortBuffers &b, int64_t n, int bits, hipStream_t s)
{
    int cur = 0;
    if (n <= 1) return cur;
    const uint32_t ntiles = (uint32_t)((n + kSortTile - 1) / kSortTile);
    const int64_t nh = (int64_t)ntiles * kRadixBins;
    for (int shift = 0; shift < bits; shift += kRadixBits) {
        k_radix_hist<<<ntiles, kSortThreads, 0, s>>>(b.keys[cur], (uint32_t)n, shift, b.hist,
                                                     ntiles);
        launch_exclusive_scan(b.hist, b.hist, nh, b.scan_tmp, nullptr, s);
        k_radix_scatter<<<ntiles, kSortThreads, 0, s>>>(b.keys[cur], b.vals[cur],
                                                        b.keys[cur ^ 1], b.vals[cur ^ 1],
                                                        (uint32_t)n, shift, b.hist, ntiles);
        cur ^= 1;
    }
    return cur;
}

// ---------------------------------------------------------------------------
// Sorted objects, leaves and node tables
// ---------------------------------------------------------------------------

__global__ void k_gather(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                         const float *__restrict__ x, const float *__restrict__ y, uint32_t n,
                         Point *__restrict__ pts, int32_t *__restrict__ inv)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t id = vals[i];
    Point p;
    p.x = x[id];
    p.y = y[id];
    p.id = id;
    p.code = keys[i];
    pts[i] = p;
    inv[id] = (int32_t)i;
}

// flags[0] = 1; flags[i+1] = 1 iff sorted objects i and i+1 lie in different
// leaves, i.e. iff the deepest quadrant holding both (level c) is split:
// c < L and the quadrant holds more than th objects.  The quadrant is a run
// [lo, hi] of the sorted codes; it holds more than th objects iff
// codes[lo + th] still lies in it.  lo is found by a binary search over the
// last th positions up to i (if the run starts even earlier, the search
// returns i + 1 - th and the test still holds, since then i + 1 = lo + th).
__global__ void k_leaf_flags(const uint32_t *__restrict__ codes, uint32_t n, int th, int L,
                             uint32_t *__restrict__ flags)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0) flags[0] = 1u;
    if (i + 1 >= n) return;
    const uint32_t a = codes[i], b = codes[i + 1];
    const int c = common_level(a, b);
    uint32_t split = 0;
    if (c < L) {
        int64_t first = (int64_t)i + 1 - th;
        if (first < 0) first = 0;
        int64_t count = (int64_t)i - first;  // positions before i still to test
        while (count > 0) {
            const int64_t step = count >> 1;
            const int64_t mid = first + step;
            if (!same_quadrant(codes[mid], a, c)) {
                first = mid + 1;
                count -= step + 1;
            } else {
                count = step;
            }
        }
        const int64_t last = first + th;
        split = (last < (int64_t)n && same_quadrant(codes[last], a, c)) ? 1u : 0u;
    }
    flags[i + 1] = split;
}

// From the exclusive scan of the flags: leaf of every sorted object and the
// [begin, end) range of every leaf.
__global__ void k_leaf_emit(const uint32_t *__restrict__ flags, const uint32_t *__restrict__ excl,
                            uint32_t n, int32_t *__restrict__ leaf_of,
                            int32_t *__restrict__ leaf_begin, int32_t *__restrict__ leaf_end)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t f = flags[i];
    int32_t leaf = (int32_t)(excl[i] + f) - 1;
    leaf_of[i] = leaf;
    if (f) {
        leaf_begin[leaf] = (int32_t)i;
        if (leaf > 0) leaf_end[leaf - 1] = (int32_t)i;
    }
    if (i + 1 == n) leaf_end[leaf] = (int32_t)n;
}

// Leaf level, and the nodes each leaf contributes to the depth-first
// tables: its inner ancestors below the deepest quadrant it shares with the
// previous leaf (forward) or next leaf (backward), then itself.
__global__ void k_leaf_info(const uint32_t *__restrict__ codes, uint32_t n, int th, int L,
                            const int32_t *__restrict__ leaf_begin,
                            const int32_t *__restrict__ leaf_end, IndexCounters *__restrict__ ctr,
                            int32_t *__restrict__ leaf_level, uint32_t *__restrict__ cnt_f,
                            uint32_t *__restrict__ cnt_r)
{
    const uint32_t nl = ctr->n_leaves;
    const uint32_t j0 = blockIdx.x * blockDim.x;
    if (j0 >= nl) return;  // whole block past the last leaf
    const uint32_t j = j0 + threadIdx.x;
    int lev = 0;
    if (j < nl) {
        const int32_t b = leaf_begin[j], e = leaf_end[j];
        const int cl = b > 0 ? common_level(codes[b - 1], codes[b]) : -1;
        const int cr = (uint32_t)e < n ? common_level(codes[e - 1], codes[e]) : -1;
        lev = (e - b <= th) ? max(cl, cr) + 1 : L;
        leaf_level[j] = lev;
        cnt_f[j] = (uint32_t)(lev - cl);
        cnt_r[j] = (uint32_t)(lev - cr);
    }
    // Statistic only: one atomic per wavefront that holds leaves.
    int deepest = lev;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) deepest = max(deepest, __shfl_xor(deepest, d, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0 && j < nl) atomicMax(&ctr->deepest_level, (uint32_t)deepest);
}

__device__ __forceinline__ void node_box(uint32_t code, int l, Node &nd)
{
    const uint32_t full = l <= 0 ? 0u : (code >> (2 * (kCodeLevels - l))) << (2 * (kCodeLevels - l));
    const uint32_t cx = compact_bits16(full), cy = compact_bits16(full >> 1);
    const uint32_t side = 1u << (kCodeLevels - l);
    const float s = 1.0f / 65536.0f;  // exact power of two; edges are exact
    nd.x0 = (float)cx * s;
    nd.y0 = (float)cy * s;
    nd.x1 = (float)(cx + side) * s;
    nd.y1 = (float)(cy + side) * s;
}

// One work item per (leaf j, slot s): slot s of leaf j's forward nodes is
// its ancestor at level cl+1+s (the leaf itself for the last slot), slot s
// of its backward nodes the ancestor at level cr+1+s.  Inner nodes find the
// end of their subtree by a binary search over the leaves' first codes.
__global__ void k_node_emit(const uint32_t *__restrict__ codes, uint32_t n,
                            const int32_t *__restrict__ leaf_begin,
                            const int32_t *__restrict__ leaf_end,
                            const int32_t *__restrict__ leaf_level,
                            const uint32_t *__restrict__ off_f, const uint32_t *__restrict__ off_r,
                            IndexCounters *__restrict__ ctr, Node *__restrict__ fwd,
                            Node *__restrict__ rev, int32_t *__restrict__ leaf_node_f,
                            int32_t *__restrict__ leaf_node_r, uint32_t node_cap)
{
    constexpr uint32_t kSlots = kCodeLevels + 1;
    const uint32_t nl = ctr->n_leaves;
    const uint32_t total = ctr->n_nodes;
    if (total > node_cap) {
        // Cannot happen for a correct build (the capacity bounds the tree);
        // refuse to write rather than overrun.
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctr->bad_input, 8u);
        return;
    }
    const uint64_t items = (uint64_t)nl * kSlots;
    for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < items;
         it += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t j = (uint32_t)(it / kSlots);
        const int sl = (int)(it % kSlots);
        const int32_t b = leaf_begin[j], e = leaf_end[j];
        const int lev = leaf_level[j];
        const uint32_t code = codes[b];
        const int cl = b > 0 ? common_level(codes[b - 1], codes[b]) : -1;
        const int cr = (uint32_t)e < n ? common_level(codes[e - 1], codes[e]) : -1;

        const int lf = cl + 1 + sl;  // forward level of this slot
        if (lf <= lev) {
            Node nd;
            node_box(code, lf, nd);
            const uint32_t idx = off_f[j] + (uint32_t)sl;
            if (lf == lev) {
                nd.begin = b;
                nd.end = e;
                nd.skip = (int32_t)idx + 1;
                nd.leaf = (int32_t)j;
                leaf_node_f[j] = (int32_t)idx;
            } else {
                // First later leaf outside this quadrant.
                uint32_t lo = j + 1, hi = nl;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (same_quadrant(codes[leaf_begin[mid]], code, lf)) lo = mid + 1;
                    else hi = mid;
                }
                nd.begin = b;
                nd.end = lo < nl ? leaf_begin[lo] : (int32_t)n;
                nd.skip = lo < nl ? (int32_t)off_f[lo] : (int32_t)total;
                nd.leaf = -1;
            }
            if (idx < node_cap) fwd[idx] = nd;
        }
        const int lr = cr + 1 + sl;  // backward level of this slot
        if (lr <= lev) {
            Node nd;
            node_box(code, lr, nd);
            // Backward table: nodes of all later leaves come first.
            const uint32_t rbase = total - off_r[j] - (uint32_t)(lev - cr);
            const uint32_t idx = rbase + (uint32_t)sl;
            if (lr == lev) {
                nd.begin = b;
                nd.end = e;
                nd.skip = (int32_t)idx + 1;
                nd.leaf = (int32_t)j;
                leaf_node_r[j] = (int32_t)idx;
            } else {
                // First (lowest) leaf inside this quadrant.
                uint32_t lo = 0, hi = j;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (same_quadrant(codes[leaf_begin[mid]], code, lr)) hi = mid;
                    else lo = mid + 1;
                }
                nd.begin = leaf_begin[lo];
                nd.end = e;
                if (lo > 0) {
                    const int32_t pe = leaf_end[lo - 1];
                    const int pcr = common_level(codes[pe - 1], codes[pe]);
                    nd.skip = (int32_t)(total - off_r[lo - 1] - (uint32_t)(leaf_level[lo - 1] - pcr));
                } else {
                    nd.skip = (int32_t)total;
                }
                nd.leaf = -1;
            }
            if (idx < node_cap) rev[idx] = nd;
        }
    }
}

__global__ void k_set_leaf_count(IndexCounters *ctr, const uint32_t *flags_total)
{
    ctr->n_leaves = *flags_total;
}

int64_t node_capacity(int64_t n, int th, int L)
{
    if (n <= 0) return 1;
    // Inner quadrants hold more than th objects and are disjoint per level.
    int64_t inner = (int64_t)L * (n / ((int64_t)th + 1)) + 1;
    int64_t leaves = 4 * inner;
    if (leaves > n) leaves = n;
    return inner + leaves + 1;
}

void launch_build_index(IndexBuffers &b, const float *x, const float *y, int64_t n, int th,
                        int L, hipStream_t s)
{
    const uint32_t nn = (uint32_t)n;
    const int T = 256;
    const uint32_t g = (uint32_t)((n + T - 1) / T);
    if (n == 0) return;
    k_morton<<<g, T, 0, s>>>(x, y, nn, b.sort.keys[0], b.sort.vals[0], b.ctr);
    const int res = launch_radix_sort(b.sort, n, 2 * kCodeLevels, s);
    const uint32_t *codes = b.sort.keys[res];
    k_gather<<<g, T, 0, s>>>(codes, b.sort.vals[res], x, y, nn, b.pts, b.inv);
    k_leaf_flags<<<g, T, 0, s>>>(codes, nn, th, L, b.flags);
    // The exclusive scan goes to the other key buffer; its sum is the leaf
    // count.
    uint32_t *excl = b.sort.vals[res ^ 1];
    launch_exclusive_scan(b.flags, excl, n, b.sort.scan_tmp, &b.ctr->n_leaves, s);
    k_leaf_emit<<<g, T, 0, s>>>(b.flags, excl, nn, b.leaf_of, b.leaf_begin, b.leaf_end);
    k_leaf_info<<<g, T, 0, s>>>(codes, nn, th, L, b.leaf_begin, b.leaf_end, b.ctr, b.leaf_level,
                                b.cnt_f, b.cnt_r);
    launch_exclusive_scan(b.cnt_f, b.cnt_f, n, b.sort.scan_tmp, &b.ctr->n_nodes, s,
                          &b.ctr->n_leaves);
    launch_exclusive_scan(b.cnt_r, b.cnt_r, n, b.sort.scan_tmp, nullptr, s, &b.ctr->n_leaves);
    k_node_emit<<<1024, T, 0, s>>>(codes, nn, b.leaf_begin, b.leaf_end, b.leaf_level, b.cnt_f,
                                b.cnt_r, b.ctr, b.fwd, b.rev, b.leaf_node_f, b.leaf_node_r,
                                (uint32_t)b.node_cap);
}

}  // namespace mknn
