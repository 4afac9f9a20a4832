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
constexpr int kSortThreads = 256;     // digit-count workgroup = 4 waves
// A radix pass tile: 8 waves, so each wave ranks its keys in 8 rounds.
constexpr int kPassThreads = 512;
// Keys per thread of a radix tile: 4096-key tiles, or 8192-key tiles from
// kSortLargeKeys keys on (fewer tiles shorten the look-back chains of large
// sorts; below it the larger tiles leave CUs idle).
constexpr int kSortItems = 8;
constexpr int kSortItemsLarge = 16;
constexpr int64_t kSortLargeKeys = int64_t(1) << 21;
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 2;
constexpr int kScanTile = kScanThreads * kScanItems;

// One object in sorted (Morton) order.  Array of 16-byte records so one
// load fetches a whole candidate during leaf sweeps; the id comes first so
// that, read into consecutive registers, it can sit next to the squared
// distance computed from x and y as the (d2, id) selection key.
struct __align__(16) Point {
    uint32_t id;    // object id = its index in the caller's arrays
    float x, y;
    uint32_t code;  // level-16 Morton code, x cell in the even bits
};

// One quadtree node in depth-first pre-order (children in Morton order for
// the forward table, reversed for the backward table).  [begin,end) is the
// range of sorted objects under the node; skip is the index of the first
// node after its subtree; leaf is the leaf index for leaves, -1 otherwise.
struct __align__(16) Node {
    float x0, y0, x1, y1;  // quadrant box [x0,x1) x [y0,y1), exact edges; after a refit
                           // tick a leaf's is its objects' bounding box
    int32_t begin, end;
    int32_t skip;
    int32_t leaf;
};

// Device scalars written by the build and read by later kernels (no host
// round trip between the build and the queries).  The error words are
// sticky: a kernel that meets bad input raises its word to its (nonzero)
// epoch with atomicMax, and the word stays nonzero until the host reads
// and clears it.  The deepest level and the drift are tagged with the
// build's epoch in their high bits; each build (refit) first stores its
// own epoch with a plain store, then raises the value with atomicMax, so a
// larger value from another epoch (after the epochs wrap, or from a graph
// replayed out of order) never shadows it.
struct IndexCounters {
    uint32_t n_leaves;
    uint32_t n_nodes;
    uint32_t deepest;        // (build epoch << 8) | deepest leaf level
    uint32_t bad_coord;      // nonzero: a coordinate was outside [0,1)
    uint32_t bad_nodes;      // nonzero: the node tables overflowed
    uint32_t bad_issuer;     // nonzero: an issuer was outside [0,n)
    uint32_t bad_k;          // nonzero: a k was outside [1,k_max]
    uint32_t bad_sync_build; // nonzero: a build look-back wait gave up
    uint32_t bad_sync_query; // nonzero: a query look-back wait gave up
    uint32_t bad_centre;     // nonzero: a free centre was outside [0,1)
    uint32_t pad;
    // (build epoch << 32) | fp32 bits of the largest per-axis displacement of
    // any object since the last full build, raised by each refit tick.
    unsigned long long drift;
};

// Workspace of single-pass scans and radix passes.  Each pass or scan
// owns one look-back word per tile (and, for radix passes, per digit) and a
// tile ticket; all of it must be zero when the pass is launched.  A build
// carves its workspace from one block of words that its first kernel zeroes.
struct ScanSpace {
    uint64_t *status;   // look-back words, one per tile
    uint32_t *ticket;   // tile ticket counter
    uint32_t *err;      // raised to `epoch` if a look-back wait gives up
    uint32_t epoch;
};

// Ping-pong buffers of a radix sort of (key, val) pairs and its workspace.
constexpr int kMaxRadixPasses = 4;
struct SortBuffers {
    uint32_t *keys[2];
    uint32_t *vals[2];
    uint32_t *ghist;    // global digit counts, [copies][kMaxRadixPasses][kRadixBins] (zeroed)
    uint64_t *status;   // [passes][tiles][kRadixBins] look-back words (zeroed)
    uint32_t *tickets;  // [kMaxRadixPasses] tile tickets (zeroed)
    uint32_t *err;      // raised to `epoch` if a look-back wait gives up
    uint32_t epoch;
};

// A block of workspace words and how a build or a query carves it.
struct Workspace {
    uint64_t *base;
    int64_t cap_words;
};

// Device memory of one context's index.  Sizes are capacities.
struct IndexBuffers {
    SortBuffers sort;
    // sorted objects
    float2 *xy;             // positions interleaved, id order (build staging)
    float2 *anchor;         // positions at the last full build, sorted order
    Point *pts;
    int32_t *inv;           // sorted position of each object id (built on demand)
    int32_t *leaf_of;       // leaf index of each sorted position
    // leaves
    int32_t *leaf_begin, *leaf_end;
    int32_t *leaf_level;
    uint32_t *leaf_code;       // code of each leaf's first object
    uint32_t *cnt_f, *cnt_r;   // nodes emitted per leaf -> offsets
    int32_t *leaf_node_f, *leaf_node_r;
    Node *fwd, *rev;
    IndexCounters *ctr;
    Workspace ws;
    ScanSpace scan[3];         // flags, forward and backward node counts
    int64_t n_cap, node_cap;
};

// Host launchers -------------------------------------------------------------

// Tiles of a single-pass scan over n items.
int64_t scan_tiles(int64_t n);
// Radix sort tiles for n keys (tile size chosen by n).
int64_t radix_tiles(int64_t n);
// Workspace words a build over n objects (or a query sort of n keys plus a
// scan of n values) needs.
int64_t workspace_words(int64_t n);

// Carve a sort workspace (n keys) and `n_scans` scan workspaces (n values
// each) from ws; look-back failures raise *err to epoch.  Returns the
// number of words used, which must be zeroed before the first pass runs.
int64_t carve_workspace(const Workspace &ws, int64_t n, SortBuffers *sort, ScanSpace *scans,
                        int n_scans, uint32_t *err, uint32_t epoch);

// Zero the first `words` words of a workspace.
void launch_zero_words(uint64_t *p, int64_t words, hipStream_t s);

// Exclusive scan of n uint32 values in one launch (in -> out may alias);
// *total, if not null, receives the sum.  If n_dev is given, only the first
// min(n, *n_dev) entries are scanned.  sp must be zero (it is consumed).
void launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, const ScanSpace &sp,
                           uint32_t *total, hipStream_t s, const uint32_t *n_dev = nullptr);

// Stable LSD radix sort of (key, val) pairs by key bits [low_bit, low_bit +
// bits) (at most 32; bits above are zero or past the top of the key); the
// result ends in keys[res], vals[res] where res is returned.  The workspace
// in b must be zero (it is consumed).  With pts, the last pass writes keys
// and, instead of vals, the records {xy[val], val, key} to pts (the index
// build's sorted objects).
int launch_radix_sort(const SortBuffers &b, int64_t n, int bits, hipStream_t s,
                      const float2 *xy = nullptr, Point *pts = nullptr,
                      float2 *anchor = nullptr, int low_bit = 0);
// Refit tick: new positions into the sorted records of the last full build
// (same objects, same order, same leaves) and the drift since that build.
void launch_refit(IndexBuffers &b, const float *x, const float *y, int64_t n, uint32_t epoch,
                  hipStream_t s);

// Full index build over positions x, y (device, n objects); epoch tags the
// build's flags (1 .. 2^24-1).
void launch_build_index(IndexBuffers &b, const float *x, const float *y, int64_t n, int th,
                        int max_level, uint32_t epoch, hipStream_t s);

// Sorted position of every object id (for subset queries).
void launch_inverse(const IndexBuffers &b, int64_t n, hipStream_t s);

// Node-table capacity needed for n objects, leaf capacity th, depth L.
int64_t node_capacity(int64_t n, int th, int L);

}  // namespace mknn
