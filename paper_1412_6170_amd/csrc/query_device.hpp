// Device helpers shared by the two query kernels (query.hip: one query per
// lane; query_wave.hip: one query per wavefront).  Built with
// -ffp-contract=off; the pragma below keeps every multiply and add of the
// distance and bound computations separately rounded.
#pragma once

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

__device__ __forceinline__ float box_lower_bound_exact(float qx, float qy, const Node &nd)
{
    const float gx = (qx < nd.x0) ? (nd.x0 - qx) : ((qx >= nd.x1) ? (qx - nd.x1) : 0.0f);
    const float gy = (qy < nd.y0) ? (nd.y0 - qy) : ((qy >= nd.y1) ? (qy - nd.y1) : 0.0f);
    const float ax = gx * gx;
    const float ay = gy * gy;
    return ax + ay;
}

// Lower bound of d2 over the node's box grown by pad on every side (pad is 0
// right after a full build; after refit ticks it covers the objects' drift).
__device__ __forceinline__ float box_lower_bound(float qx, float qy, const Node &nd, float pad)
{
    const float x0 = nd.x0 - pad, x1 = nd.x1 + pad;
    const float y0 = nd.y0 - pad, y1 = nd.y1 + pad;
    const float gx = (qx < x0) ? (x0 - qx) : ((qx >= x1) ? (qx - x1) : 0.0f);
    const float gy = (qy < y0) ? (y0 - qy) : ((qy >= y1) ? (qy - y1) : 0.0f);
    const float ax = gx * gx;
    const float ay = gy * gy;
    return ax + ay;
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

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
