// Device helpers shared by the two query kernels (query.hip: one query per
// lane; query_wave.hip: one query per wavefront).  Built with
// -ffp-contract=off; the pragma below keeps every multiply and add of the
// distance and bound computations separately rounded.
#pragma once

#include <utility>

#include "mknn_internal.hpp"

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
// High word of kKeyMax.  Any key with this high word is a filler, not a
// neighbour, whatever its low word: it lies above every real key and at or
// below kKeyMax, so as a threshold or a pruning bound it admits everything.
constexpr uint32_t kFillHi = 0x7fefffffu;

__device__ __forceinline__ double as_f64(uint64_t k) { return __longlong_as_double((long long)k); }
__device__ __forceinline__ uint64_t as_key(double d) { return (uint64_t)__double_as_longlong(d); }
// v_min_f64 / v_max_f64 written directly: fmin/fmax on loaded or
// bit-assembled doubles make the compiler quiet possible signalling NaNs
// first (one more fp64 op per operand), and keys are never NaN (their
// exponent field is at most 0x7f7).
__device__ __forceinline__ uint64_t key_min(uint64_t a, uint64_t b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(as_f64(a)), "v"(as_f64(b)));
    return as_key(r);
}
__device__ __forceinline__ uint64_t key_max(uint64_t a, uint64_t b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(as_f64(a)), "v"(as_f64(b)));
    return as_key(r);
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

// Gap between a coordinate and the interval [lo, hi): lo - v below it,
// v - hi at or above hi, zero inside.  Exactly one of the two differences
// can be positive (lo < hi), so the largest of them and zero is that gap,
// computed without a branch.
__device__ __forceinline__ float interval_gap(float v, float lo, float hi)
{
    return fmaxf(fmaxf(lo - v, v - hi), 0.0f);
}

// Lower bound of d2 over the node's box.  Every object of the box lies on
// the far side of the gap's edge, and rounding is monotone, so its rounded
// squared distance is no smaller.
__device__ __forceinline__ float box_lower_bound_exact(float qx, float qy, const Node &nd)
{
    const float gx = interval_gap(qx, nd.x0, nd.x1);
    const float gy = interval_gap(qy, nd.y0, nd.y1);
    const float ax = gx * gx;
    const float ay = gy * gy;
    return ax + ay;
}

// Lower bound of d2 over the node's box grown by pad on every side (pad is 0
// right after a full build; after refit ticks it covers the objects' drift).
__device__ __forceinline__ float box_lower_bound(float qx, float qy, const Node &nd, float pad)
{
    const float gx = interval_gap(qx, nd.x0 - pad, nd.x1 + pad);
    const float gy = interval_gap(qy, nd.y0 - pad, nd.y1 + pad);
    const float ax = gx * gx;
    const float ay = gy * gy;
    return ax + ay;
}

// Compare-exchange on keys: afterwards lo <= hi.
__device__ __forceinline__ void cmp_swap(uint64_t &lo, uint64_t &hi)
{
    const uint64_t t = key_min(lo, hi);
    hi = key_max(lo, hi);
    lo = t;
}

// Batcher's odd-even merge sort (N a power of two): fewer compare-exchanges
// than the bitonic network (63 instead of 80 for N = 16), all ascending.
// The comparator list is generated at compile time.
template <int N>
struct OddEvenNet {
    int lo[N * N], hi[N * N];  // generous bound on the comparator count
    int count = 0;
    constexpr void add(int a, int b)
    {
        lo[count] = a;
        hi[count] = b;
        ++count;
    }
    constexpr void merge(int base, int n, int r)
    {
        const int m = r * 2;
        if (m < n) {
            merge(base, n, m);
            merge(base + r, n, m);
            for (int i = base + r; i + r < base + n; i += m) add(i, i + r);
        } else {
            add(base, base + r);
        }
    }
    constexpr void sort(int base, int n)
    {
        if (n > 1) {
            const int m = n / 2;
            sort(base, m);
            sort(base + m, m);
            merge(base, n, 1);
        }
    }
    constexpr OddEvenNet() : lo(), hi() { sort(0, N); }
};

template <int N>
struct OddEven {
    static constexpr OddEvenNet<N> net{};
};

template <int N, int... I>
__device__ __forceinline__ void oddeven_apply(uint64_t (&b)[N], std::integer_sequence<int, I...>)
{
    (cmp_swap(b[OddEven<N>::net.lo[I]], b[OddEven<N>::net.hi[I]]), ...);
}

template <int N>
__device__ __forceinline__ void oddeven_sort(uint64_t (&b)[N])
{
    oddeven_apply<N>(b, std::make_integer_sequence<int, OddEven<N>::net.count>{});
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

__device__ __forceinline__ uint64_t shfl_xor_key(uint64_t v, int m)
{
    const int lo = __shfl_xor((int)(uint32_t)v, m, kWave);
    const int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, kWave);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// The value of lane (lane ^ M), M a compile-time mask.  Patterns that stay
// inside a row of 16 lanes are DPP moves, one VALU instruction per dword
// with no trip through the LDS unit: quad permutes for 1, 2 and 3, the
// half-row and row mirrors for 7 and 15, a row rotation by 8 for 8, and for
// 4 two row shifts each writing the half of the lanes (banks of 4 lanes)
// it serves.  Other masks use the LDS permute.
template <int M>
__device__ __forceinline__ uint32_t xor_dword(uint32_t x)
{
    const int v = (int)x;
    // DPP controls: quad_perm [1,0,3,2] [2,3,0,1] [3,2,1,0]; row_half_mirror;
    // row_mirror; row_ror:8; row_shl:4 (lane i reads i + 4) into banks 0
    // and 2, row_shr:4 (reads i - 4) into banks 1 and 3.
    if constexpr (M == 1) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
    else if constexpr (M == 2) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
    else if constexpr (M == 3) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x1B, 0xF, 0xF, false);
    else if constexpr (M == 7) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);
    else if constexpr (M == 15) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);
    else if constexpr (M == 8) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);
    else if constexpr (M == 4) {
        const int t = __builtin_amdgcn_mov_dpp(v, 0x104, 0xF, 0x5, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(t, v, 0x114, 0xF, 0xA, false);
    } else {
        return (uint32_t)__shfl_xor(v, M, kWave);
    }
}

template <int M>
__device__ __forceinline__ uint64_t xor_key(uint64_t v)
{
    const uint32_t lo = xor_dword<M>((uint32_t)v);
    const uint32_t hi = xor_dword<M>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_key(uint64_t v, int src)
{
    const int lo = __shfl((int)(uint32_t)v, src, kWave);
    const int hi = __shfl((int)(uint32_t)(v >> 32), src, kWave);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ uint64_t readlane_key(uint64_t v, int lane)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Bitonic networks over N keys (a power of two) held PL per lane by N / PL
// consecutive lanes in the blocked layout: key i sits in lane i / PL of the
// group, register i % PL; `idx` is the lane's index in its group (groups
// are aligned, so partners found by xor-ing the lane id stay inside).  A
// stage pairs i with i ^ STRIDE and orders the pair ascending where
// (i & SIZE) == 0 (SIZE = 0: every pair ascending, as in the last stage of
// a sort and in a merge).  Partners at a distance below PL are in the same
// lane; farther partners are in lane idx ^ (STRIDE / PL), same register, and
// each side keeps the minimum or the maximum.  Expanded with templates so
// every register index is static.
template <int PL, int SIZE, int STRIDE, int R>
__device__ __forceinline__ void wstage_one(uint64_t (&v)[PL], int idx)
{
    bool asc;
    if constexpr (SIZE == 0) asc = true;
    else if constexpr (SIZE < PL) asc = (R & SIZE) == 0;
    else asc = ((idx * PL) & SIZE) == 0;  // R < PL <= SIZE: no carry into bit SIZE
    if constexpr (STRIDE < PL) {
        constexpr int R2 = R ^ STRIDE;
        if constexpr (R2 > R) {
            const uint64_t lo = key_min(v[R], v[R2]);
            const uint64_t hi = key_max(v[R], v[R2]);
            v[R] = asc ? lo : hi;
            v[R2] = asc ? hi : lo;
        }
    } else {
        constexpr int M = STRIDE / PL;
        const uint64_t w = xor_key<M>(v[R]);
        const bool lower = (idx & M) == 0;
        // Both results, then a select: a choice between the two asm
        // statements would be compiled as a branch around each.
        const uint64_t lo = key_min(v[R], w);
        const uint64_t hi = key_max(v[R], w);
        v[R] = (lower == asc) ? lo : hi;
    }
}

template <int PL, int SIZE, int STRIDE, int... R>
__device__ __forceinline__ void wstage(uint64_t (&v)[PL], int idx, std::integer_sequence<int, R...>)
{
    (wstage_one<PL, SIZE, STRIDE, R>(v, idx), ...);
}

template <int PL, int SIZE, int STRIDE>
__device__ __forceinline__ void wstrides(uint64_t (&v)[PL], int idx)
{
    wstage<PL, SIZE, STRIDE>(v, idx, std::make_integer_sequence<int, PL>{});
    if constexpr (STRIDE > 1) wstrides<PL, SIZE, STRIDE / 2>(v, idx);
}

// Sort all N keys of the group ascending.
template <int PL, int N, int SIZE = 2>
__device__ __forceinline__ void net_sort(uint64_t (&v)[PL], int idx)
{
    if constexpr (SIZE <= N) {
        wstrides<PL, (SIZE == N ? 0 : SIZE), SIZE / 2>(v, idx);
        net_sort<PL, N, SIZE * 2>(v, idx);
    }
}

// Sort a bitonic sequence of N keys ascending (half-cleaner cascade).
template <int PL, int N>
__device__ __forceinline__ void net_merge(uint64_t (&v)[PL], int idx)
{
    wstrides<PL, 0, N / 2>(v, idx);
}


// Tile order is XCD-aware: workgroups are dealt round-robin to the 8 XCDs
// (workgroup b runs on XCD b mod 8), so for T tiles workgroup b takes tile
// (b mod 8) * ceil(T / 8) + b / 8.  Each XCD then works through one
// contiguous eighth of the Morton-ordered queries, whose candidates are
// spatially close and stay in that XCD's L2.  T is the launch's own query
// count (known on the device for a k class), so the grid may be larger;
// workgroups past the tiles exit at once.  (Measured per wavefront, the
// eighths carry equal work; dealing smaller chunks to the XCDs in turn
// only cost L2 locality.)
constexpr uint32_t kXcds = 8;

__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t tiles)
{
    const uint32_t per = (tiles + kXcds - 1) / kXcds;
    const uint32_t slot = b / kXcds;
    return slot < per ? (b % kXcds) * per + slot : 0xffffffffu;
}

}  // namespace mknn
