// Internal declarations of the mknn HIP library (gfx950).  Data layout in
// HBM, the device records shared by the index build and the query kernels,
// and the host-side launchers each translation unit provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mknn {

constexpr int kCodeLevels = 16;       // Morton codes on the 2^16 x 2^16 grid
constexpr int kWave = 64;             // CDNA wavefront width
constexpr int kRadixBits = 8;         // LSD radix sort digit
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kSortThreads = 256;     // one workgroup = 4 waves
constexpr int kSortItems = 8;         // keys per thread per tile
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// One object in sorted (Morton) order.  Array of 16-byte records so one
// scalar load fetches a whole candidate during leaf sweeps.
struct __align__(16) Point {
    float x, y;
    uint32_t id;    // object id = its index in the caller's arrays
    uint32_t code;  // level-16 Morton code, x cell in the even bits
};

// One quadtree node in depth-first pre-order (children in Morton order for
// the forward table, reversed for the backward table).  [begin,end) is the
// range of sorted objects under the node; skip is the index of the first
// node after its subtree; leaf is the leaf index for leaves, -1 otherwise.
struct __align__(16) Node {
    float x0, y0, x1, y1;  // quadrant box [x0,x1) x [y0,y1), exact edges
    int32_t begin, end;
    int32_t skip;
    int32_t leaf;
};

// Device scalars written by the build and read by later kernels (no host
// round trip between the build and the queries).
struct IndexCounters {
    uint32_t n_leaves;
    uint32_t n_nodes;
    uint32_t deepest_level;
    uint32_t bad_input;     // set when a coordinate is outside [0,1)
};

// Ping-pong buffers of a radix sort of (key, val) pairs.
struct SortBuffers {
    uint32_t *keys[2];
    uint32_t *vals[2];
    uint32_t *hist;         // kRadixBins * tiles
    uint32_t *scan_tmp;     // block sums for device-wide scans
};

// Device memory of one context's index.  Sizes are capacities.
struct IndexBuffers {
    SortBuffers sort;
    // sorted objects
    Point *pts;
    int32_t *inv;           // sorted position of each object id
    int32_t *leaf_of;       // leaf index of each sorted position
    // leaves
    uint32_t *flags;        // leaf-start flags -> exclusive scan
    int32_t *leaf_begin, *leaf_end;
    int32_t *leaf_level;
    uint32_t *cnt_f, *cnt_r;   // nodes emitted per leaf -> offsets
    int32_t *leaf_node_f, *leaf_node_r;
    Node *fwd, *rev;
    IndexCounters *ctr;
    int64_t n_cap, node_cap, hist_cap, scan_tmp_cap;
};

// Host launchers -------------------------------------------------------------

// Scratch element counts needed for a device-wide exclusive scan of n items.
int64_t scan_tmp_elems(int64_t n);
// Exclusive scan of n uint32 values (in -> out may alias); *total, if not
// null, receives the sum on the device.
// If n_dev is given, only the first min(n, *n_dev) entries are scanned.
void launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                           uint32_t *total, hipStream_t s, const uint32_t *n_dev = nullptr);

// Number of histogram entries a radix sort of n keys needs.
int64_t radix_hist_elems(int64_t n);
// Stable LSD radix sort of (key, val) pairs by key bits [0, bits); the result
// ends in keys[res], vals[res] where res is returned (0 or 1).
int launch_radix_sort(const SortBuffers &b, int64_t n, int bits, hipStream_t s);

// Full index build over positions x, y (device, n objects).
void launch_build_index(IndexBuffers &b, const float *x, const float *y, int64_t n, int th,
                        int max_level, hipStream_t s);

// Node-table capacity needed for n objects, leaf capacity th, depth L.
int64_t node_capacity(int64_t n, int th, int L);

}  // namespace mknn
