// Index build for one tick (arXiv 1412.6170, Sec. 4.1), gfx950.
//
//   k_morton         level-16 Morton code per object (the virtual full
//                    quadtree at l_max = 16), x cell in the even bits;
//                    device-side range validation
//   radix sort       stable LSD sort of (level-L code, id) -- the top 2L
//                    bits of the codes -- 8-bit digits, tiles staged in LDS
//                    and written back in digit runs; the last pass writes
//                    the sorted objects as 16-byte records {id, x, y, code}
//   k_leaves         which adjacent sorted objects fall in different leaves,
//                    scanned in the same pass into leaf ranges
//   k_leaf_nodes     leaf level and the node count each leaf contributes,
//                    scanned in the same pass into node positions
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

// Inclusive scan across one wavefront, with DPP adds that stay in the
// vector unit: shifts by 1, 2, 4 and 8 lanes inside each row of 16 (lanes
// whose source falls outside the row add zero), then the last lane of row
// 0 and of row 2 added to rows 1 and 3, then lane 31 added to rows 2 and 3.
// Every lane of the wavefront must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, true);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return (uint32_t)x;
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
// Decoupled look-back (the single-pass prefix scan of Merrill and Garland,
// "Single-pass Parallel Prefix Scan with Decoupled Look-back", NVIDIA
// technical report NVR-2016-002): tile t publishes its aggregate, then walks back over
// tiles t-1, t-2, ... adding aggregates until it meets an inclusive prefix,
// and publishes its own inclusive prefix.  A word holds a 2-bit flag and a
// 62-bit value, written and read as one 64-bit atomic.  Tiles take tickets
// in the order they start, so a tile only ever waits on tiles that are
// already running, and every tile publishes its aggregate before it waits:
// the waits always end.  A bounded spin records an error instead of
// hanging if that reasoning were ever violated.
// ---------------------------------------------------------------------------

constexpr uint64_t kLbAgg = 1ull << 62;
constexpr uint64_t kLbInc = 2ull << 62;
constexpr uint64_t kLbVal = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ __forceinline__ void lb_store(uint64_t *w, uint64_t v)
{
    __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lb_load(uint64_t *w)
{
    return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish the tile's aggregate (tile 0 publishes it as its inclusive prefix).
__device__ __forceinline__ void lb_publish(uint64_t *status, uint32_t stride, uint32_t tile,
                                           uint64_t agg)
{
    lb_store(status + (uint64_t)tile * stride, (tile == 0 ? kLbInc : kLbAgg) | agg);
}

// Exclusive prefix of the tile, then publish the inclusive prefix.  The
// predecessors' words are read kLbWindow at a time (independent loads in
// flight together), then consumed in order: aggregates are added until an
// inclusive prefix is met; a word not yet published stops the pass and the
// next read starts from it.
constexpr int kLbWindow = 16;

__device__ __forceinline__ uint64_t lb_resolve(uint64_t *status, uint32_t stride, uint32_t tile,
                                               uint64_t agg, uint32_t *err, uint32_t epoch)
{
    if (tile == 0) return 0;
    uint64_t excl = 0;
    int64_t t = (int64_t)tile - 1;  // next predecessor to add
    uint32_t spins = 0;
    bool done = false;
    while (!done) {
        uint64_t w[kLbWindow];
#pragma unroll
        for (int i = 0; i < kLbWindow; ++i)
            w[i] = (t - i >= 0) ? lb_load(status + (uint64_t)(t - i) * stride) : kLbInc;
        int used = 0;
        bool stalled = false;
#pragma unroll
        for (int i = 0; i < kLbWindow; ++i) {
            if (!done && !stalled) {
                const uint64_t flag = w[i] & ~kLbVal;
                if (flag == 0) {
                    stalled = true;
                } else {
                    excl += w[i] & kLbVal;
                    ++used;
                    // Tile 0 is always inclusive, so t - i < 0 is never
                    // reached; the kLbInc filler above only ends the walk.
                    if (flag == kLbInc) done = true;
                }
            }
        }
        t -= used;
        if (!done && used == 0) {
            if (++spins > kSpinLimit) {
                atomicMax(err, epoch);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    lb_store(status + (uint64_t)tile * stride, kLbInc | (excl + agg));
    return excl;
}

// The same for a single look-back word per tile, resolved by one whole
// wavefront: lane i reads predecessor t - i, so 64 words are read per round.
// Returns the exclusive prefix in every lane; lane 0 publishes the inclusive
// prefix.
__device__ __forceinline__ uint64_t lb_resolve_wave(uint64_t *status, uint32_t tile, uint64_t agg,
                                                    uint32_t *err, uint32_t epoch)
{
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t excl = 0;
    int64_t t = (int64_t)tile - 1;
    uint32_t spins = 0;
    while (t >= 0) {
        const int64_t mine = t - lane;
        // Below tile 0, a zero inclusive filler ends the walk.
        const uint64_t w = mine >= 0 ? lb_load(status + mine) : kLbInc;
        const uint64_t flag = w & ~kLbVal;
        const uint64_t inc = __ballot(flag == kLbInc);
        const uint64_t none = __ballot(flag == 0);
        const int first_inc = inc ? __builtin_ctzll(inc) : kWave;
        const int first_none = none ? __builtin_ctzll(none) : kWave;
        // Lanes [0, take) are consumed this round.
        const bool done = first_inc < first_none;
        const int take = done ? first_inc + 1 : first_none;
        uint64_t v = lane < take ? (w & kLbVal) : 0ull;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
        excl += v;
        if (done) break;
        t -= take;
        if (take == 0) {
            if (++spins > kSpinLimit) {
                if (lane == 0) atomicMax(err, epoch);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    if (lane == 0) lb_store(status + tile, kLbInc | (excl + agg));
    return excl;
}

__device__ __forceinline__ uint32_t take_ticket(uint32_t *ticket)
{
    __shared__ uint32_t s_ticket;
    if (threadIdx.x == 0) s_ticket = atomicAdd(ticket, 1u);
    __syncthreads();
    return s_ticket;
}

// ---------------------------------------------------------------------------
// Single-pass exclusive scan of uint32
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kScanThreads) void k_scan_lb(const uint32_t *in, uint32_t *out,
                                                         uint32_t n,
                                                         const uint32_t *__restrict__ n_dev,
                                                         ScanSpace sp,
                                                         uint32_t *__restrict__ total)
{
    __shared__ uint32_t s_excl;
    if (n_dev) n = min(n, *n_dev);
    const uint32_t tile = take_ticket(sp.ticket);
    const uint32_t base = tile * (uint32_t)kScanTile;
    if (base >= n && !(n == 0 && tile == 0)) return;  // past the data; nobody waits on it
    // Blocked arrangement: thread t owns kScanItems consecutive elements.
    const uint32_t mine = base + threadIdx.x * (uint32_t)kScanItems;
    uint32_t v[kScanItems], sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint32_t p = mine + j;
        v[j] = (p < n) ? in[p] : 0u;
        sum += v[j];
    }
    uint32_t agg;
    uint32_t pre = block_excl_scan<kScanThreads>(sum, &agg);
    if (threadIdx.x == 0) lb_publish(sp.status, 1, tile, agg);
    if (threadIdx.x < kWave) {
        const uint64_t e = lb_resolve_wave(sp.status, tile, agg, sp.err, sp.epoch);
        if (threadIdx.x == 0) {
            s_excl = (uint32_t)e;
            if (total && base + kScanTile >= n) *total = (uint32_t)e + agg;
        }
    }
    __syncthreads();
    pre += s_excl;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint32_t p = mine + j;
        if (p < n) out[p] = pre;
        pre += v[j];
    }
}

int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, const ScanSpace &sp,
                           uint32_t *total, hipStream_t s, const uint32_t *n_dev)
{
    // At least one tile, so *total is written even for n = 0.
    const uint32_t nb = (uint32_t)(n > 0 ? (n + kScanTile - 1) / kScanTile : 1);
    k_scan_lb<<<nb, kScanThreads, 0, s>>>(in, out, (uint32_t)(n > 0 ? n : 0), n_dev, sp, total);
}

__global__ void k_zero_words(uint64_t *__restrict__ p, int64_t words)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

void launch_zero_words(uint64_t *p, int64_t words, hipStream_t s)
{
    if (words <= 0) return;
    int64_t blocks = (words + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    k_zero_words<<<(uint32_t)blocks, 256, 0, s>>>(p, words);
}

// ---------------------------------------------------------------------------
// Morton codes (Sec. 4.1: quadrants of the virtual full quadtree at l_max)
// ---------------------------------------------------------------------------

__global__ void k_morton(const float *__restrict__ x, const float *__restrict__ y, uint32_t n,
                         uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                         float2 *__restrict__ xy, IndexCounters *__restrict__ ctr,
                         uint64_t *__restrict__ ws, int64_t ws_words, uint32_t epoch)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    // The build's scan and sort workspace starts at zero.
    for (int64_t w = i; w < ws_words; w += (int64_t)gridDim.x * blockDim.x) ws[w] = 0ull;
    // This build's deepest-level word starts at its own epoch (raised by
    // k_leaf_nodes, which runs after this kernel).
    if (i == 0) ctr->deepest = epoch << 8;
    if (i >= n) return;
    float px = x[i], py = y[i];
    // NaN fails both comparisons; -0.0 passes.
    bool ok = (px >= 0.0f) && (px < 1.0f) && (py >= 0.0f) && (py < 1.0f);
    if (!ok) atomicMax(&ctr->bad_coord, epoch);
    // Scaling by 2^16 is exact; truncation is the floor for x >= 0.  The
    // clamp only matters for rejected input.
    uint32_t cx = ok ? (uint32_t)(px * 65536.0f) : 0u;
    uint32_t cy = ok ? (uint32_t)(py * 65536.0f) : 0u;
    cx = min(cx, 65535u);
    cy = min(cy, 65535u);
    keys[i] = spread_bits16(cx) | (spread_bits16(cy) << 1);
    vals[i] = i;
    // Interleaved copy, so the sort's last pass fetches a position with one
    // 8-byte read.
    xy[i] = make_float2(px, py);
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits, one launch per pass
//
// k_radix_ghist counts every pass's digits over all keys in one read (keys
// do not change between passes, only their order), in LDS per workgroup.  Each pass then runs one
// kernel over tiles of 4096 keys (8192 for large sorts):
//   * wavefront w of the tile owns a contiguous quarter of it and ranks its
//     keys in rounds of 64 in position order; lanes holding the same digit
//     are found with ballots, and a wavefront-private LDS counter per digit
//     gives the rank (no workgroup barrier between rounds);
//   * per-digit counts of the tile are published for decoupled look-back
//     and the tile is reordered by digit in LDS;
//   * each digit's offset among earlier tiles is found by look-back (one
//     thread per digit) and the tile is written out in contiguous digit
//     runs.  The last pass of the index build writes the sorted 16-byte
//     object records directly (positions fetched by id), so no separate
//     gather follows.
// ---------------------------------------------------------------------------

constexpr int kGhistItems = 16;  // keys per thread in the histogram kernel
// Copies of the digit counts: workgroup b adds into copy b mod kGhistCopies,
// so each count takes kGhistCopies times fewer global atomics from
// different workgroups; a radix pass sums the copies of its digits.
constexpr int kGhistCopies = 8;
constexpr int kGhistStride = kMaxRadixPasses * kRadixBins;  // words per copy

// Lanes of the wavefront (among `valid`) holding the same 8-bit digit d.
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, uint64_t valid)
{
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const uint64_t m = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? m : ~m;
    }
    return peers;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_ghist(const uint32_t *__restrict__ keys,
                                                             uint32_t n, int passes, int low_bit,
                                                             uint32_t *__restrict__ ghist)
{
    __shared__ uint32_t s_h[kMaxRadixPasses][kRadixBins];
#pragma unroll
    for (int p = 0; p < kMaxRadixPasses; ++p) s_h[p][threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * (uint32_t)(kSortThreads * kGhistItems);
#pragma unroll
    for (int j = 0; j < kGhistItems; ++j) {
        const uint32_t i = base + j * kSortThreads + threadIdx.x;
        if (i < n) {
            const uint32_t k = keys[i];
            for (int p = 0; p < passes; ++p)
                atomicAdd(&s_h[p][(k >> (low_bit + kRadixBits * p)) & (kRadixBins - 1)], 1u);
        }
    }
    __syncthreads();
    ghist += (blockIdx.x % kGhistCopies) * kGhistStride;
    for (int p = 0; p < passes; ++p) {
        const uint32_t c = s_h[p][threadIdx.x];
        if (c) atomicAdd(&ghist[p * kRadixBins + threadIdx.x], c);
    }
}

template <int NT, int ITEMS, bool LAST>
__global__ __launch_bounds__(NT) void k_radix_pass(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
    uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out, uint32_t n, int shift,
    const uint32_t *__restrict__ ghist, uint64_t *__restrict__ status, uint32_t *__restrict__ ticket,
    uint32_t *__restrict__ err, uint32_t epoch, const float2 *__restrict__ xy,
    Point *__restrict__ pts, float2 *__restrict__ anchor)
{
    constexpr int NW = NT / kWave;
    constexpr int TILE = NT * ITEMS;
    constexpr int PER_WAVE = kWave * ITEMS;
    static_assert(NT >= 2 * kRadixBins, "one thread per digit, as many more gathering");
    __shared__ uint32_t s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];
    __shared__ uint32_t s_wc[NW][kRadixBins];  // per-wavefront digit counts, then bases
    __shared__ uint32_t s_start[kRadixBins];   // start of each digit's run in the tile
    __shared__ uint32_t s_base[kRadixBins];    // destination of each digit's run
    __shared__ float2 s_pos[LAST ? TILE : 1];  // last pass: positions in tile order

    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const bool digit_thread = t < kRadixBins;  // thread t < 256 owns digit t
    for (int i = t; i < NW * kRadixBins; i += NT) (&s_wc[0][0])[i] = 0;
    const uint32_t tile = take_ticket(ticket);  // also orders the clearing above
    // This pass's count of digit t over all keys (the copies summed),
    // fetched now so the loads overlap the ranking.
    uint32_t digit_total = 0;
    if (digit_thread) {
#pragma unroll
        for (int c = 0; c < kGhistCopies; ++c) digit_total += ghist[c * kGhistStride + t];
    }
    const uint32_t base = tile * (uint32_t)TILE;
    const uint32_t n_valid = min((uint32_t)TILE, n - base);
    const uint64_t lt_mask = (1ull << lane) - 1ull;

    // Wavefront w owns tile positions [w * PER_WAVE, (w + 1) * PER_WAVE);
    // round j of lane l holds position w * PER_WAVE + j * 64 + l.  Padding
    // keys (all ones) take the last digit and the last positions, so they
    // rank after every real key.
    uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t p = w * PER_WAVE + j * kWave + lane;
        const bool v = p < n_valid;
        key[j] = v ? keys_in[base + p] : 0xffffffffu;
        val[j] = v ? vals_in[base + p] : 0u;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t d = (key[j] >> shift) & (kRadixBins - 1);
        const uint64_t peers = digit_peers(d, ~0ull);
        const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
        const uint32_t prior = s_wc[w][d];
        rank[j] = prior + below;
        // The lowest lane of each digit group advances the counter; the
        // wavefront's LDS accesses complete in order, so the next round
        // reads the new value.
        if (below == 0) s_wc[w][d] = prior + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    // Thread t: digit t.  Per-wavefront counts become per-wavefront bases.
    uint32_t cnt = 0;
    if (digit_thread) {
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const uint32_t c = s_wc[q][t];
            s_wc[q][t] = cnt;
            cnt += c;
        }
    }
    // Publish this tile's count of digit t (padding excluded) before
    // anything else, so later tiles can resolve while this one reorders.
    const uint32_t real = cnt - (t == kRadixBins - 1 ? (uint32_t)TILE - n_valid : 0u);
    if (digit_thread) lb_publish(status + t, kRadixBins, tile, real);
    const uint32_t start = block_excl_scan<NT>(cnt, nullptr);
    if (digit_thread) s_start[t] = start;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t d = (key[j] >> shift) & (kRadixBins - 1);
        const uint32_t local = s_start[d] + s_wc[w][d] + rank[j];
        s_keys[local] = key[j];
        s_vals[local] = val[j];
    }

    // Offset of digit t: keys of smaller digits anywhere, plus keys of digit
    // t in earlier tiles.  The digit threads wait for the earlier tiles.
    // In the last pass the other threads meanwhile fetch the position of
    // every object of the tile by id (random reads) into LDS: in waves of
    // their own, so the waits of the look-back, which count that wave's
    // memory reads in order, do not wait for them too.
    {
        const uint32_t below = block_excl_scan<NT>(digit_total, nullptr);
        if (digit_thread) {
            const uint64_t before = lb_resolve(status + t, kRadixBins, tile, real, err, epoch);
            s_base[t] = below + (uint32_t)before;
        } else if constexpr (LAST) {
            for (uint32_t lp = t - kRadixBins; lp < n_valid; lp += NT - kRadixBins)
                s_pos[lp] = xy[s_vals[lp]];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t lp = j * NT + t;
        if (lp < n_valid) {
            const uint32_t k = s_keys[lp];
            const uint32_t d = (k >> shift) & (kRadixBins - 1);
            const uint32_t dst = s_base[d] + (lp - s_start[d]);
            const uint32_t v = s_vals[lp];
            // dst < n whenever the digit counts are consistent; a failed
            // look-back wait (err set) must not turn into a stray write.
            if (dst >= n) {
                atomicMax(err, epoch);
                continue;
            }
            keys_out[dst] = k;
            if constexpr (LAST) {
                const float2 q = s_pos[lp];
                Point r;
                r.x = q.x;
                r.y = q.y;
                r.id = v;
                r.code = k;
                pts[dst] = r;
                anchor[dst] = q;
            } else {
                vals_out[dst] = v;
            }
        }
    }
}

static int sort_items(int64_t n) { return n >= kSortLargeKeys ? kSortItemsLarge : kSortItems; }

int64_t radix_tiles(int64_t n)
{
    const int64_t tile = (int64_t)kPassThreads * sort_items(n);
    return n > 0 ? (n + tile - 1) / tile : 1;
}

// Look-back words are sized with the smaller tile, an upper bound of
// radix_tiles(m) for every m <= n (the tile count drops where the larger
// tiles start).
static int64_t radix_tiles_bound(int64_t n)
{
    const int64_t tile = (int64_t)kPassThreads * kSortItems;
    return n > 0 ? (n + tile - 1) / tile : 1;
}

int launch_radix_sort(const SortBuffers &b, int64_t n, int bits, hipStream_t s, const float2 *xy,
                      Point *pts, float2 *anchor, int low_bit)
{
    int cur = 0;
    if (n < 1 || (n == 1 && !pts)) return cur;
    const uint32_t ntiles = (uint32_t)radix_tiles(n);
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    const uint32_t gblocks = (uint32_t)((n + kSortThreads * kGhistItems - 1) / (kSortThreads * kGhistItems));
    k_radix_ghist<<<gblocks, kSortThreads, 0, s>>>(b.keys[0], (uint32_t)n, passes, low_bit,
                                                   b.ghist);
    const bool large = sort_items(n) == kSortItemsLarge;
    for (int p = 0; p < passes; ++p) {
        const bool last = p == passes - 1;
        const bool rec = last && pts;  // this pass writes the object records
        auto pass = large ? (rec ? k_radix_pass<kPassThreads, kSortItemsLarge, true>
                                 : k_radix_pass<kPassThreads, kSortItemsLarge, false>)
                          : (rec ? k_radix_pass<kPassThreads, kSortItems, true>
                                 : k_radix_pass<kPassThreads, kSortItems, false>);
        pass<<<ntiles, kPassThreads, 0, s>>>(
            b.keys[cur], b.vals[cur], b.keys[cur ^ 1], b.vals[cur ^ 1], (uint32_t)n,
            low_bit + kRadixBits * p, b.ghist + p * kRadixBins,
            b.status + (uint64_t)p * ntiles * kRadixBins, b.tickets + p, b.err, b.epoch,
            last ? xy : nullptr, last ? pts : nullptr, last ? anchor : nullptr);
        cur ^= 1;
    }
    return cur;
}

int64_t workspace_words(int64_t n)
{
    // ghist (u32) + tickets + err, then radix look-back words, then scans.
    const int64_t small = (kGhistCopies * kGhistStride + 16 + 8) / 2 + 8;
    return small + (int64_t)kMaxRadixPasses * radix_tiles_bound(n) * kRadixBins +
           4 * scan_tiles(n) + 16;
}

int64_t carve_workspace(const Workspace &ws, int64_t n, SortBuffers *sort, ScanSpace *scans,
                        int n_scans, uint32_t *err, uint32_t epoch)
{
    uint64_t *p = ws.base;
    uint32_t *small = (uint32_t *)p;
    sort->ghist = small;                                  // [copies][4][256]
    sort->tickets = small + kGhistCopies * kGhistStride;  // [4]
    sort->err = err;
    sort->epoch = epoch;
    uint32_t *scan_tickets = sort->tickets + kMaxRadixPasses + 1;  // [n_scans]
    p += (kGhistCopies * kGhistStride + 16 + 8) / 2 + 8;
    sort->status = p;
    p += (int64_t)kMaxRadixPasses * radix_tiles(n) * kRadixBins;
    for (int i = 0; i < n_scans; ++i) {
        scans[i].status = p;
        scans[i].ticket = scan_tickets + i;
        scans[i].err = err;
        scans[i].epoch = epoch;
        p += scan_tiles(n);
    }
    return (int64_t)(p - ws.base);
}

// ---------------------------------------------------------------------------
// Sorted objects, leaves and node tables
// ---------------------------------------------------------------------------

// Sorted position of every object id; only subset queries need it.
__global__ void k_inverse(const Point *__restrict__ pts, uint32_t n, int32_t *__restrict__ inv)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) inv[pts[i].id] = (int32_t)i;
}

void launch_inverse(const IndexBuffers &b, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    k_inverse<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(b.pts, (uint32_t)n, b.inv);
}

// A new leaf starts at sorted position p iff p = 0 or objects p-1 and p lie
// in different leaves, i.e. iff the deepest quadrant holding both (level c)
// is split: c < L and the quadrant holds more than th objects.  The
// quadrant is a run [lo, hi] of the sorted codes; it holds more than th
// objects iff codes[lo + th] still lies in it.  lo is found by a binary
// search over the last th positions up to p-1 (if the run starts even
// earlier, the search returns p - th and the test still holds, since then
// p = lo + th).
//
// k_leaves does this for kScanItems consecutive positions per thread, with
// the searches of a thread's positions advancing in lockstep (their loads
// are independent and in flight together), scans the flags in one pass
// with decoupled look-back, and writes the leaf of every position and the
// [begin, end) range of every leaf; the last tile writes the leaf count.
// The searches of a tile read codes within th positions of it only: up to
// kLeavesStageTh, that span is first copied to LDS with coalesced loads
// and every search step reads LDS (Staged); beyond it, global memory.
constexpr int kLeavesStageTh = 1024;
constexpr int kLeavesSpan = kScanTile + 2 * kLeavesStageTh;

// LDS slot of staged code i: one word of skew per 32, so lanes reading
// positions kScanItems apart fall in different banks.
__host__ __device__ constexpr int leaves_slot(int i) { return i + (i >> 5); }

template <bool Staged>
__global__ __launch_bounds__(kScanThreads) void k_leaves(
    const uint32_t *__restrict__ codes, uint32_t n, int th, int L, int search_steps, ScanSpace sp,
    IndexCounters *__restrict__ ctr, int32_t *__restrict__ leaf_of,
    int32_t *__restrict__ leaf_begin, int32_t *__restrict__ leaf_end)
{
    __shared__ uint32_t s_excl;
    __shared__ uint32_t s_codes[Staged ? leaves_slot(kLeavesSpan) : 1];
    const uint32_t tile = take_ticket(sp.ticket);
    const uint32_t base = tile * (uint32_t)kScanTile;
    if (base >= n) return;  // past the data; nobody waits on it
    const uint32_t mine = base + threadIdx.x * (uint32_t)kScanItems;

    // Every position read below lies in [lo, hi): a pair's two codes, its
    // search window [p - th, p - 1] and the test position, below p + th.
    const int64_t lo = max((int64_t)base - th, (int64_t)0);
    const int64_t hi = min((int64_t)base + kScanTile + th, (int64_t)n);
    if constexpr (Staged) {
        for (int64_t i = lo + threadIdx.x; i < hi; i += kScanThreads)
            s_codes[leaves_slot((int)(i - lo))] = codes[i];
        __syncthreads();
    }
    auto code_at = [&](int64_t i) -> uint32_t {
        if constexpr (Staged) return s_codes[leaves_slot((int)(i - lo))];
        else return codes[i];
    };

    uint32_t a[kScanItems];
    int c[kScanItems];
    int64_t first[kScanItems], count[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint32_t p = mine + j;
        const bool pair = p >= 1 && p < n;
        // Positions without a pair read (and search) nothing outside [lo, hi).
        const int64_t q = pair ? (int64_t)p - 1 : lo;
        a[j] = code_at(q);
        const uint32_t b = pair ? code_at(p) : a[j];
        c[j] = pair ? common_level(a[j], b) : kCodeLevels;
        first[j] = pair ? max(q + 1 - th, (int64_t)0) : lo;
        count[j] = (pair && c[j] < L) ? q - first[j] : 0;
    }
    for (int step = 0; step < search_steps; ++step) {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            const int64_t half = count[j] >> 1;
            const int64_t mid = first[j] + half;
            const bool out = count[j] > 0 && !same_quadrant(code_at(mid), a[j], c[j]);
            first[j] = out ? mid + 1 : first[j];
            count[j] = count[j] > 0 ? (out ? count[j] - half - 1 : half) : 0;
        }
    }
    uint32_t f[kScanItems], sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint32_t p = mine + j;
        uint32_t split = 0;
        if (p >= 1 && p < n && c[j] < L) {
            const int64_t last = first[j] + th;
            split = (last < (int64_t)n && same_quadrant(code_at(last), a[j], c[j])) ? 1u : 0u;
        }
        f[j] = p == 0 ? 1u : split;
        f[j] = p < n ? f[j] : 0u;
        sum += f[j];
    }
    uint32_t agg;
    uint32_t pre = block_excl_scan<kScanThreads>(sum, &agg);
    if (threadIdx.x == 0) lb_publish(sp.status, 1, tile, agg);
    if (threadIdx.x < kWave) {
        const uint64_t e = lb_resolve_wave(sp.status, tile, agg, sp.err, sp.epoch);
        if (threadIdx.x == 0) {
            s_excl = (uint32_t)e;
            if (base + kScanTile >= n) ctr->n_leaves = (uint32_t)e + agg;
        }
    }
    __syncthreads();
    pre += s_excl;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint32_t p = mine + j;
        if (p < n) {
            pre += f[j];
            const int32_t leaf = (int32_t)pre - 1;
            leaf_of[p] = leaf;
            if (f[j]) {
                leaf_begin[leaf] = (int32_t)p;
                if (leaf > 0) leaf_end[leaf - 1] = (int32_t)p;
            }
            if (p + 1 == n) leaf_end[leaf] = (int32_t)n;
        }
    }
}

constexpr uint32_t kLeafNodeGroups = 64;

// Leaf level, and the nodes each leaf contributes to the depth-first
// tables: its inner ancestors below the deepest quadrant it shares with the
// previous leaf (forward) or next leaf (backward), then itself.  Both node
// counts are scanned in the same pass (two look-back chains, resolved by
// two wavefronts side by side) into the leaves' first node positions; the
// last tile writes the node count.  Leaves are counted on the device, so
// the workgroups loop over tiles until they pass the last leaf.
__global__ __launch_bounds__(kScanThreads) void k_leaf_nodes(
    const uint32_t *__restrict__ codes, uint32_t n, int th, int L,
    const int32_t *__restrict__ leaf_begin, const int32_t *__restrict__ leaf_end, ScanSpace spf,
    ScanSpace spr, IndexCounters *__restrict__ ctr, int32_t *__restrict__ leaf_level,
    uint32_t *__restrict__ leaf_code, uint32_t *__restrict__ off_f, uint32_t *__restrict__ off_r,
    uint32_t epoch)
{
    __shared__ uint32_t s_excl[2];
    const uint32_t nl = ctr->n_leaves;
    int deepest = 0;
    // A small fixed grid takes tiles in ticket order until it passes the
    // leaves (their count is only known here): a grid sized for the worst
    // case would spend more time launching idle workgroups than working.
    for (;;) {
        const uint32_t tile = take_ticket(spf.ticket);
        const uint32_t base = tile * (uint32_t)kScanTile;
        if (base >= nl) break;
        const uint32_t mine = base + threadIdx.x * (uint32_t)kScanItems;
        uint32_t cf[kScanItems], cr[kScanItems], sf = 0, sr = 0;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            const uint32_t p = mine + j;
            cf[j] = cr[j] = 0;
            if (p < nl) {
                const int32_t b = leaf_begin[p], e = leaf_end[p];
                const int cl = b > 0 ? common_level(codes[b - 1], codes[b]) : -1;
                const int crl = (uint32_t)e < n ? common_level(codes[e - 1], codes[e]) : -1;
                const int lev = (e - b <= th) ? max(cl, crl) + 1 : L;
                leaf_level[p] = lev;
                leaf_code[p] = codes[b];
                cf[j] = (uint32_t)(lev - cl);
                cr[j] = (uint32_t)(lev - crl);
                deepest = max(deepest, lev);
            }
            sf += cf[j];
            sr += cr[j];
        }
        uint32_t agg_f, agg_r;
        uint32_t pre_f = block_excl_scan<kScanThreads>(sf, &agg_f);
        __syncthreads();  // the scan's shared partials are reused below
        uint32_t pre_r = block_excl_scan<kScanThreads>(sr, &agg_r);
        if (threadIdx.x == 0) {
            lb_publish(spf.status, 1, tile, agg_f);
            lb_publish(spr.status, 1, tile, agg_r);
        }
        if (threadIdx.x < kWave) {
            const uint64_t e = lb_resolve_wave(spf.status, tile, agg_f, spf.err, spf.epoch);
            if (threadIdx.x == 0) {
                s_excl[0] = (uint32_t)e;
                if (base + kScanTile >= nl) ctr->n_nodes = (uint32_t)e + agg_f;
            }
        } else if (threadIdx.x < 2 * kWave) {
            const uint64_t e = lb_resolve_wave(spr.status, tile, agg_r, spr.err, spr.epoch);
            if (threadIdx.x == kWave) s_excl[1] = (uint32_t)e;
        }
        __syncthreads();
        pre_f += s_excl[0];
        pre_r += s_excl[1];
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            const uint32_t p = mine + j;
            if (p < nl) {
                off_f[p] = pre_f;
                off_r[p] = pre_r;
            }
            pre_f += cf[j];
            pre_r += cr[j];
        }
        __syncthreads();  // s_excl and the scan partials are reused by the next tile
    }
    // Statistic only: one atomic per workgroup, skipped when the stored
    // value is already as large (every workgroup targets the same word).
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) deepest = max(deepest, __shfl_xor(deepest, d, kWave));
    __shared__ int s_deep[kScanThreads / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) s_deep[threadIdx.x / kWave] = deepest;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kScanThreads / kWave; ++w) deepest = max(deepest, s_deep[w]);
        const uint32_t v = (epoch << 8) | (uint32_t)deepest;
        if (deepest > 0 &&
            v > __hip_atomic_load(&ctr->deepest, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&ctr->deepest, v);
    }
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

// One thread per leaf j emits its forward nodes (its ancestors below the
// deepest quadrant shared with leaf j-1, then itself) and its backward
// nodes (likewise with leaf j+1).  An inner node's subtree ends where the
// leaves' first codes leave its quadrant; that boundary is found by a
// galloping search over the leaf codes (subtrees are mostly small), the
// forward and backward searches of a level running together.
__device__ __forceinline__ uint32_t gallop_up(const uint32_t *__restrict__ lc, uint32_t j,
                                              uint32_t nl, uint32_t code, int l)
{
    // First leaf index > j whose code leaves the level-l quadrant of code.
    uint32_t lo = j, step = 1, hi;
    for (;;) {
        const uint32_t p = j + step;
        if (p >= nl) { hi = nl; break; }
        if (!same_quadrant(lc[p], code, l)) { hi = p; break; }
        lo = p;
        step <<= 1;
    }
    ++lo;  // lo: first candidate not yet known inside
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (same_quadrant(lc[mid], code, l)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t gallop_down(const uint32_t *__restrict__ lc, uint32_t j,
                                                uint32_t code, int l)
{
    // Lowest leaf index <= j whose code lies in the level-l quadrant of code.
    uint32_t hi = j, step = 1, lo;
    for (;;) {
        if (step > j) { lo = 0; break; }
        const uint32_t p = j - step;
        if (!same_quadrant(lc[p], code, l)) { lo = p + 1; break; }
        hi = p;
        step <<= 1;
    }
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (same_quadrant(lc[mid], code, l)) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Leaf levels run from min(cl, cr) + 1 >= 0 to lev <= 16 (17 at most, and
// one to three for most leaves); a group of kLevelLanes lanes shares them
// round robin, so the searches of different levels of one leaf run side by
// side while a wavefront still serves several leaves.
constexpr int kLevelLanes = 8;
constexpr uint32_t kNodeEmitBlocks = 2048;  // of 256 threads: every SIMD filled

// The nodes leaf j contributes to either table: its forward nodes (its
// ancestors below the deepest quadrant shared with leaf j-1, then itself)
// and its backward nodes (likewise with leaf j+1).  Lane r of the leaf's
// group emits levels min(cl, cr) + 1 + r, + kLevelLanes, ...
__device__ __forceinline__ void emit_leaf_levels(
    const uint32_t *__restrict__ codes, uint32_t n, const int32_t *__restrict__ leaf_begin,
    const int32_t *__restrict__ leaf_end, const int32_t *__restrict__ leaf_level,
    const uint32_t *__restrict__ leaf_code, const uint32_t *__restrict__ off_f,
    const uint32_t *__restrict__ off_r, uint32_t nl, uint32_t total, Node *__restrict__ fwd,
    Node *__restrict__ rev, int32_t *__restrict__ leaf_node_f, int32_t *__restrict__ leaf_node_r,
    uint32_t node_cap, uint32_t j, int r)
{
    const int32_t b = leaf_begin[j], e = leaf_end[j];
    const int lev = leaf_level[j];
    const uint32_t code = leaf_code[j];
    const int cl = b > 0 ? common_level(codes[b - 1], code) : -1;
    const int cr = (uint32_t)e < n ? common_level(codes[e - 1], codes[e]) : -1;
    const uint32_t fbase = off_f[j];
    // Backward table: nodes of all later leaves come first.
    const uint32_t rbase = total - off_r[j] - (uint32_t)(lev - cr);
    for (int l = min(cl, cr) + 1 + r; l <= lev; l += kLevelLanes) {
        const bool do_f = l > cl, do_r = l > cr;
        Node nd;
        node_box(code, l, nd);
        if (l == lev) {
            nd.begin = b;
            nd.end = e;
            nd.leaf = (int32_t)j;
            const uint32_t fi = fbase + (uint32_t)(l - cl - 1);
            const uint32_t ri = rbase + (uint32_t)(l - cr - 1);
            nd.skip = (int32_t)fi + 1;
            if (fi < node_cap) fwd[fi] = nd;
            leaf_node_f[j] = (int32_t)fi;
            nd.skip = (int32_t)ri + 1;
            if (ri < node_cap) rev[ri] = nd;
            leaf_node_r[j] = (int32_t)ri;
            break;  // lev is the last level
        }
        nd.leaf = -1;
        if (do_f) {
            const uint32_t hi = gallop_up(leaf_code, j, nl, code, l);
            const uint32_t fi = fbase + (uint32_t)(l - cl - 1);
            nd.begin = b;
            nd.end = hi < nl ? leaf_begin[hi] : (int32_t)n;
            nd.skip = hi < nl ? (int32_t)off_f[hi] : (int32_t)total;
            if (fi < node_cap) fwd[fi] = nd;
        }
        if (do_r) {
            const uint32_t lo = gallop_down(leaf_code, j, code, l);
            const uint32_t ri = rbase + (uint32_t)(l - cr - 1);
            nd.begin = leaf_begin[lo];
            nd.end = e;
            if (lo > 0) {
                const int32_t pe = leaf_end[lo - 1];
                const int pcr = common_level(codes[pe - 1], codes[pe]);
                nd.skip = (int32_t)(total - off_r[lo - 1] - (uint32_t)(leaf_level[lo - 1] - pcr));
            } else {
                nd.skip = (int32_t)total;
            }
            if (ri < node_cap) rev[ri] = nd;
        }
    }
}

__global__ void k_node_emit(const uint32_t *__restrict__ codes, uint32_t n,
                            const int32_t *__restrict__ leaf_begin,
                            const int32_t *__restrict__ leaf_end,
                            const int32_t *__restrict__ leaf_level,
                            const uint32_t *__restrict__ leaf_code,
                            const uint32_t *__restrict__ off_f, const uint32_t *__restrict__ off_r,
                            IndexCounters *__restrict__ ctr, Node *__restrict__ fwd,
                            Node *__restrict__ rev, int32_t *__restrict__ leaf_node_f,
                            int32_t *__restrict__ leaf_node_r, uint32_t node_cap,
                            uint32_t epoch)
{
    const uint32_t nl = ctr->n_leaves;
    const uint32_t total = ctr->n_nodes;
    if (total > node_cap) {
        // Cannot happen for a correct build (the capacity bounds the tree);
        // refuse to write rather than overrun.
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(&ctr->bad_nodes, epoch);
        return;
    }
    const int r = (int)(threadIdx.x % kLevelLanes);
    const uint32_t per_block = blockDim.x / kLevelLanes;
    for (uint32_t j = blockIdx.x * per_block + threadIdx.x / kLevelLanes; j < nl;
         j += gridDim.x * per_block)
        emit_leaf_levels(codes, n, leaf_begin, leaf_end, leaf_level, leaf_code, off_f, off_r, nl,
                         total, fwd, rev, leaf_node_f, leaf_node_r, node_cap, j, r);
}


// ---------------------------------------------------------------------------
// Refit tick (reuse of the last full build's index).  Sec. 4.1 rebuilds the
// index only when the work of the last tick grows by some factor over recent
// ticks; between rebuilds, the objects keep their sorted positions and leaves,
// each record takes the object's new position, and the largest per-axis
// displacement D of any object since the build is recorded.  Every object of
// a node's range lay inside the node's quadrant at the build, so it now lies
// inside the quadrant grown by D on every side; the query kernels prune inner
// nodes with those grown boxes.  A leaf's box is recomputed instead, as the
// bounding box of its objects' current positions (a leaf holds few objects,
// and the distance computations happen at leaves), so results stay exact.
// ---------------------------------------------------------------------------

__global__ void k_refit(const float *__restrict__ x, const float *__restrict__ y, uint32_t n,
                        Point *__restrict__ pts, const float2 *__restrict__ anchor,
                        IndexCounters *__restrict__ ctr, uint32_t epoch)
{
    // A fixed grid strides over the objects, so few workgroups reach the
    // shared maximum below.
    float d = 0.0f;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t id = pts[i].id;
        const float px = x[id], py = y[id];
        const bool ok = (px >= 0.0f) && (px < 1.0f) && (py >= 0.0f) && (py < 1.0f);
        if (!ok) atomicMax(&ctr->bad_coord, epoch);
        pts[i].x = px;
        pts[i].y = py;
        const float2 a = anchor[i];
        d = fmaxf(d, ok ? fmaxf(fabsf(px - a.x), fabsf(py - a.y)) : 0.0f);
    }
    // Largest displacement of the workgroup; non-negative floats order like
    // their bit patterns, so a 64-bit atomicMax keeps the epoch's maximum.
    // The atomic is skipped when the stored value is already as large (all
    // workgroups hit one address, and most would not raise it).
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) d = fmaxf(d, __shfl_xor(d, s, kWave));
    __shared__ float s_d[256 / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) s_d[threadIdx.x / kWave] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / kWave); ++w) d = fmaxf(d, s_d[w]);
        const unsigned long long v = ((unsigned long long)epoch << 32) | __float_as_uint(d);
        const unsigned long long cur =
            __hip_atomic_load(&ctr->drift, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v > cur) atomicMax(&ctr->drift, v);
    }
}

// Leaf boxes of a refit tick: the box of each leaf's node, in both tables,
// becomes the bounding box [min, max] of its objects' current positions.
// Its edges are coordinates of the leaf's objects, and rounding is monotone,
// so the unpadded lower bound (gap to the box, squared and summed in fp32)
// never exceeds the computed d2 of any of them.  A group of kBoxLanes lanes
// per leaf strides over its objects, then reduces across the group.
constexpr int kBoxLanes = 8;
constexpr uint32_t kBoxBlocks = 2048;

__global__ __launch_bounds__(256) void k_refit_leaf_boxes(
    const Point *__restrict__ pts, const int32_t *__restrict__ leaf_begin,
    const int32_t *__restrict__ leaf_end, const int32_t *__restrict__ leaf_node_f,
    const int32_t *__restrict__ leaf_node_r, const IndexCounters *__restrict__ ctr,
    Node *__restrict__ fwd, Node *__restrict__ rev, uint32_t node_cap)
{
    const uint32_t nl = ctr->n_leaves;
    const int r = (int)(threadIdx.x % kBoxLanes);
    const uint32_t per_block = blockDim.x / kBoxLanes;
    // Every lane of a wavefront runs the same iterations (the shuffles below
    // need all of them); lanes past the last leaf reduce an empty box.
    for (uint32_t j0 = blockIdx.x * per_block; j0 < nl; j0 += gridDim.x * per_block) {
        const uint32_t j = j0 + threadIdx.x / kBoxLanes;
        float x0 = __builtin_inff(), y0 = __builtin_inff();
        float x1 = -__builtin_inff(), y1 = -__builtin_inff();
        if (j < nl) {
            const int32_t e = leaf_end[j];
            for (int32_t i = leaf_begin[j] + r; i < e; i += kBoxLanes) {
                const Point p = pts[i];
                x0 = fminf(x0, p.x);
                y0 = fminf(y0, p.y);
                x1 = fmaxf(x1, p.x);
                y1 = fmaxf(y1, p.y);
            }
        }
#pragma unroll
        for (int d = 1; d < kBoxLanes; d <<= 1) {
            x0 = fminf(x0, __shfl_xor(x0, d, kWave));
            y0 = fminf(y0, __shfl_xor(y0, d, kWave));
            x1 = fmaxf(x1, __shfl_xor(x1, d, kWave));
            y1 = fmaxf(y1, __shfl_xor(y1, d, kWave));
        }
        if (j < nl && r == 0) {
            const float4 box = make_float4(x0, y0, x1, y1);
            const uint32_t f = (uint32_t)leaf_node_f[j], b = (uint32_t)leaf_node_r[j];
            if (f < node_cap) *reinterpret_cast<float4 *>(&fwd[f].x0) = box;
            if (b < node_cap) *reinterpret_cast<float4 *>(&rev[b].x0) = box;
        }
    }
}

// The drift word starts at this refit's epoch with a zero displacement, by
// a plain store ahead of k_refit's maxima.
__global__ void k_drift_start(IndexCounters *ctr, uint32_t epoch)
{
    ctr->drift = (unsigned long long)epoch << 32;
}

void launch_refit(IndexBuffers &b, const float *x, const float *y, int64_t n, uint32_t epoch,
                  hipStream_t s)
{
    if (n <= 0) return;
    k_drift_start<<<1, 1, 0, s>>>(b.ctr, epoch);
    const int T = 256;
    const int64_t g = (n + T - 1) / T;
    k_refit<<<(uint32_t)(g < 1024 ? g : 1024), T, 0, s>>>(x, y, (uint32_t)n, b.pts, b.anchor, b.ctr,
                                                         epoch);
    // At most one leaf per object; the grid strides over the leaf count,
    // which is only known on the device.
    const int64_t gb = (n + T / kBoxLanes - 1) / (T / kBoxLanes);
    k_refit_leaf_boxes<<<(uint32_t)(gb < kBoxBlocks ? gb : kBoxBlocks), T, 0, s>>>(
        b.pts, b.leaf_begin, b.leaf_end, b.leaf_node_f, b.leaf_node_r, b.ctr, b.fwd, b.rev,
        (uint32_t)b.node_cap);
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
                        int L, uint32_t epoch, hipStream_t s)
{
    const uint32_t nn = (uint32_t)n;
    const int T = 256;
    const uint32_t g = (uint32_t)((n + T - 1) / T);
    if (n == 0) return;
    const int64_t words = carve_workspace(b.ws, n, &b.sort, b.scan, 3, &b.ctr->bad_sync_build,
                                          epoch);
    k_morton<<<g, T, 0, s>>>(x, y, nn, b.sort.keys[0], b.sort.vals[0], b.xy, b.ctr, b.ws.base,
                             words, epoch);
    // Objects are ordered by their Morton code at level L (the top 2L bits
    // of the level-16 code), ties by id: no leaf lies below L, so the lower
    // bits order nothing the index or the queries depend on.
    const int res = launch_radix_sort(b.sort, n, 2 * L, s, b.xy, b.pts, b.anchor,
                                      2 * (kCodeLevels - L));
    const uint32_t *codes = b.sort.keys[res];
    // Binary-search steps over a window of th positions.
    int steps = 1;
    while ((1ll << steps) <= (int64_t)th + 1) ++steps;
    const uint32_t ns = (uint32_t)((n + kScanTile - 1) / kScanTile);
    if (th <= kLeavesStageTh)
        k_leaves<true><<<ns, kScanThreads, 0, s>>>(codes, nn, th, L, steps, b.scan[0], b.ctr,
                                                   b.leaf_of, b.leaf_begin, b.leaf_end);
    else
        k_leaves<false><<<ns, kScanThreads, 0, s>>>(codes, nn, th, L, steps, b.scan[0], b.ctr,
                                                    b.leaf_of, b.leaf_begin, b.leaf_end);
    const uint32_t gl = ns < kLeafNodeGroups ? ns : kLeafNodeGroups;
    k_leaf_nodes<<<gl, kScanThreads, 0, s>>>(codes, nn, th, L, b.leaf_begin, b.leaf_end, b.scan[1],
                                             b.scan[2], b.ctr, b.leaf_level, b.leaf_code, b.cnt_f,
                                             b.cnt_r, epoch);
    const uint32_t gn = (uint32_t)((n + T / kLevelLanes - 1) / (T / kLevelLanes));
    k_node_emit<<<gn < kNodeEmitBlocks ? gn : kNodeEmitBlocks, T, 0, s>>>(codes, nn, b.leaf_begin, b.leaf_end,
                                                   b.leaf_level, b.leaf_code,
                                b.cnt_f, b.cnt_r, b.ctr, b.fwd, b.rev, b.leaf_node_f,
                                b.leaf_node_r, (uint32_t)b.node_cap, epoch);
}

}  // namespace mknn
