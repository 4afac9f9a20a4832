// Arguments of the query kernels (see query.hip).
#pragma once

#include "mknn_internal.hpp"

namespace mknn {

// A free query centre in processing (Morton) order: its position, the id of
// the object it excludes (kNoExclude: none) and its insertion position among
// the sorted objects (where its code would sort).
constexpr uint32_t kNoExclude = 0xffffffffu;
struct __align__(16) QPoint {
    float x, y;
    uint32_t excl;
    int32_t pos;
};

struct QueryArgs {
    const Point *pts;            // sorted objects
    uint32_t n;                  // number of objects
    const Node *fwd, *rev;       // depth-first node tables
    const int32_t *leaf_of;      // leaf of each sorted position
    const int32_t *leaf_begin, *leaf_end;
    const int32_t *leaf_node_f, *leaf_node_r;
    const IndexCounters *ctr;
    int32_t node_cap;            // entries in each node table
    const int32_t *qpos;         // sorted position of each query centre, in
                                 // processing order; null = identity
    const int32_t *qrow;         // result row of each query, processing
                                 // order; null = object id (every object queries)
    const QPoint *qpts;          // free centres in processing order (then qpos
                                 // is unused); null = queries issued by objects
    uint32_t pos_mask;           // bits of a qpos entry holding the position
    const uint32_t *class_bounds;  // null, or first processing-order query of
                                   // each k class ([kQueryClasses + 1])
    int klass;                   // the class this launch answers
    uint32_t nq;
    const int32_t *ks;           // k per result row (range-checked); null = k_uniform
    int32_t k_uniform;
    const int64_t *row_off;      // first entry of each row; null = row * k_uniform
    int32_t *out_ids;
    float *out_d2;
    int32_t *out_cnt;
    uint32_t build_epoch;        // epoch of the current index (refit drift tag)
    unsigned long long *counters;  // null, or [candidate steps, merges,
                                   // node visits, leaf sweeps, wavefronts]
    uint32_t tile_queries;       // lane flavour: queries per wavefront (8..64;
                                 // 0 = chosen at launch)
    uint32_t compute_units;      // of the device (0 = 256); sizes automatic tiles
};

constexpr int kQueryClasses = 5;  // selection lists of 8, 16, 32, 64, 128 keys

struct QueryPrep {
    const int32_t *issuers;      // device, nq entries, or null
    const int32_t *ks;           // device, nq entries, or null
    uint32_t nq, n;
    int k_max;
    const int32_t *inv;
    int class_shift;             // >= 0: put the k class above bit class_shift
    SortBuffers sort;            // keys[0]/vals[0] receive (sorted position, query)
    uint32_t *kcount;            // range-checked k per query
    IndexCounters *ctr;
    uint64_t *ws;                // query workspace words to zero first
    int64_t ws_words;
    uint32_t epoch;              // query epoch for the error flags
};

// Free-centre queries: validate and encode the centres, then (after the
// query sort by code) place each one among the sorted objects.
struct PointPrep {
    const float *qx, *qy;        // device, nq entries
    const int32_t *exclude;      // device, nq entries (-1: none), or null
    const int32_t *ks;           // device, nq entries, or null
    uint32_t nq, n;
    int k_max;
    SortBuffers sort;            // keys[0]/vals[0] receive (code, query)
    uint32_t *kcount;
    IndexCounters *ctr;
    uint64_t *ws;
    int64_t ws_words;
    uint32_t epoch;
};

int k_class(int k);
// List size (64, 128, 256, 512 or 1024 keys) of the one-query-per-wavefront
// kernel for a largest k.
int k_class_wave(int k);
void launch_knn_wave(const QueryArgs &qa, int kclass, hipStream_t s);
// List size (32, 64, ..., 1024 keys: 16 per lane of a group of 2 to 64
// lanes) of the group-per-query kernel for a largest k.
int k_class_group(int k);
void launch_knn_group(const QueryArgs &qa, int kclass, hipStream_t s);
void launch_point_prep(const PointPrep &p, hipStream_t s);
void launch_point_place(const uint32_t *codes, const uint32_t *rows, uint32_t nq, const float *qx,
                        const float *qy, const int32_t *exclude, const Point *pts, uint32_t n,
                        QPoint *qpts, hipStream_t s);
void launch_knn(const QueryArgs &qa, int kclass, hipStream_t s);
void launch_query_prep(const QueryPrep &p, hipStream_t s);
void launch_class_bounds(const uint32_t *keys, uint32_t nq, int class_shift, uint32_t *bounds,
                         hipStream_t s);
void launch_offsets(const uint32_t *kcount, uint32_t nq, uint32_t *scan_out, const ScanSpace &sp,
                    uint32_t *total, int64_t *offsets, hipStream_t s);

}  // namespace mknn
