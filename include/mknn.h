/*
 * mknn.h -- repeated k-NN queries over massive sets of moving 2D objects,
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method: Lettich, Orlando, Silvestri, "Manycore processing of repeated k-NN
 * queries over massive moving objects observations" (arXiv 1412.6170).
 *
 * Time is split into ticks (Sec. 2.2).  Per tick the caller hands over the
 * latest position of every object (the snapshot P of the tick) and the
 * queries Q issued during it; the library returns, for every query, its
 * k nearest objects (Definition 1, Sec. 2.1) -- the "iterated batch
 * processing" problem of Sec. 2.3.  Per tick it rebuilds a point-region
 * quadtree over the snapshot (Sec. 4.1: Morton codes, radix sort, split of
 * every quadrant holding more than the leaf capacity) and answers the
 * queries in batched leaf sweeps that widen from each query's own leaf to
 * the neighbouring leaves in Morton order until no leaf can still hold a
 * nearer object (Sec. 4.2).
 *
 * Result contract (exact and unique):
 *   - A query is issued by an object s and is centred on s's position; s is
 *     excluded from its own result (by id: other objects at the same
 *     position are kept, at distance 0).
 *   - Objects are ranked by the squared fp32 distance
 *         d2 = fl( fl(fl(qx-px)*fl(qx-px)) + fl(fl(qy-py)*fl(qy-py)) )
 *     (IEEE binary32, round to nearest even, no fused multiply-add,
 *     denormals kept), ties broken by ascending object id.  Definition 1
 *     lets ties be broken arbitrarily; this choice makes the answer unique.
 *   - A row holds the first min(k, n-1) objects of that order, ascending,
 *     each with its d2; remaining slots hold id -1 and d2 +inf.  d2 is the
 *     SQUARED distance (no square root is taken).
 *
 * Coordinates must be finite and lie in [0,1) (the unit square; -0.0 counts
 * as 0).  Object ids are the positions 0..n-1 in the arrays passed to
 * mknn_load_positions.
 *
 * Conventions: every call returns MKNN_OK (0) or a negative MKNN_E_* code;
 * mknn_last_error gives the message.  No C++ exception crosses this
 * interface.  A context is not thread-safe; separate contexts are
 * independent.  A call that uses the GPU makes the context's device current
 * while it runs and restores the calling thread's current device before it
 * returns.  Pointers marked "device" are HIP device (or managed)
 * pointers on the context's device; "host" pointers are ordinary host
 * memory.  Work is enqueued on the context's stream and the calls return
 * before the GPU finishes, except where a call says it synchronises.
 */
#ifndef MKNN_H
#define MKNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Exported entry points (the library is built with hidden visibility). */
#if defined(__GNUC__) || defined(__clang__)
#define MKNN_API __attribute__((visibility("default")))
#else
#define MKNN_API
#endif

/* Status codes. */
#define MKNN_OK 0
#define MKNN_E_INVAL (-1)    /* NULL pointer, bad `where`, k < 1 or k > k_max, ... */
#define MKNN_E_RANGE (-2)    /* a coordinate is not finite or lies outside [0,1) */
#define MKNN_E_STATE (-3)    /* call out of order (e.g. query before advance_tick) */
#define MKNN_E_CAPACITY (-4) /* n > n_max, nq > q_max or result entries too many */
#define MKNN_E_NOMEM (-5)    /* device or host allocation failed */
#define MKNN_E_DEVICE (-6)   /* a HIP error; sticky: the context must be destroyed */

/* Where a buffer lives. */
#define MKNN_HOST 0
#define MKNN_DEVICE 1

/* Largest k any query may ask for. */
#define MKNN_K_LIMIT 1024

/* Sweep flavours (Sec. 4.2.1, distance computations).  LANE is the
 * "cached writes" flavour: one query per lane, its best keys in that lane's
 * registers (k <= 128).  WAVE is the "coalesced writes" flavour: one query
 * per wavefront, candidates checked by the lanes side by side, list updates
 * orchestrated with ballots through an LDS buffer, rows written by
 * consecutive lanes (any k up to MKNN_K_LIMIT).  GROUP is the coalesced-
 * writes flavour with a query per group of k/16 lanes (rounded up to a
 * power of two, at least 2): its list spread 16 keys per lane over the
 * group, 64 / group queries per wavefront sharing their candidates, lists
 * merged by bitonic networks across the group's lanes (any k up to
 * MKNN_K_LIMIT).  AUTO takes LANE up to k = 32 and GROUP above; LANE
 * itself hands k above 128 to WAVE.  Results are the same in every
 * flavour. */
#define MKNN_SWEEP_AUTO 0
#define MKNN_SWEEP_LANE 1
#define MKNN_SWEEP_WAVE 2
#define MKNN_SWEEP_GROUP 3

/* mknn_config.flags */
/* Record per-phase device times (mknn_stats): HIP events on the context's
 * stream around each build and query, up to four per tick, recorded without
 * a system-scope fence (timing only, so they cost the kernels around them
 * next to nothing). */
#define MKNN_FLAG_TIMING 1
#define MKNN_FLAG_COUNTERS 2 /* count the query kernel's work (mknn_stats) */
/* Variable-k queries: group the queries by the size class of their k
 * (lists of 8, 16, 32, 64, 128 keys) and answer each class with its own
 * list size, instead of one pass sized for the largest k.  Pays off when
 * queries with similar k are spatially close (each class stays dense);
 * when k is drawn independently per query, each class is sparse in space
 * and one pass is faster.  Results are the same either way. */
#define MKNN_FLAG_GROUP_K 4
/* Answer every query with the one-query-per-wavefront flavour
 * (MKNN_SWEEP_WAVE) instead of MKNN_SWEEP_AUTO. */
#define MKNN_FLAG_SWEEP_WAVE 8

typedef struct mknn_ctx mknn_ctx;

typedef struct mknn_config {
    int32_t device;        /* HIP device ordinal */
    int32_t leaf_capacity; /* th (th_quad, Sec. 4.1): a quadrant holding more
                              than th objects is split; 0 = automatic */
    int32_t max_level;     /* l_max (Sec. 4.1): deepest quadtree level, 1..16;
                              0 = 16.  Leaves at this level may exceed th. */
    int32_t k_max;         /* largest k of any query, 1..MKNN_K_LIMIT */
    int64_t n_max;         /* capacity in objects (< 2^31) */
    int64_t q_max;         /* capacity in queries per tick (< 2^31) */
    void *stream;          /* hipStream_t to enqueue on (borrowed, not owned);
                              NULL = a stream the context creates and owns */
    int32_t k_hint;        /* typical k, used by the automatic leaf capacity;
                              0 = k_max */
    int32_t flags;         /* MKNN_FLAG_* */
} mknn_config;

/* Counters and device times of the last advance_tick / query. */
typedef struct mknn_stats {
    int64_t tick;          /* ticks advanced since the last load */
    int64_t n;             /* objects in the snapshot */
    int64_t nq;            /* queries of the last mknn_query */
    int64_t leaves;        /* non-empty quadtree leaves (active cells, Sec. 4.1) */
    int64_t nodes;         /* quadtree nodes kept (inner + non-empty leaves) */
    int32_t leaf_capacity; /* th used for the current index */
    int32_t deepest_level; /* l_deep: deepest leaf level (Sec. 4.1) */
    float ms_build;        /* device time of the last index build (MKNN_FLAG_TIMING) */
    float ms_query;        /* device time of the last query, all kernels */
    float ms_query_main;   /* device time of the last query's leaf-sweep kernel */
    int32_t timed_ticks;   /* builds and queries timed since mknn_reset_timing
                              (at most the last 256 of each are kept) */
    float ms_build_mean;   /* means over those ticks */
    float ms_query_mean;
    float ms_query_main_mean;
    float reserved[4];
    /* MKNN_FLAG_COUNTERS: totals over the queries since mknn_reset_timing */
    int64_t wave_candidate_steps; /* candidates evaluated, counted once per wavefront */
    int64_t wave_merges;          /* queue merges, once per wavefront */
    int64_t wave_node_visits;     /* node-table entries examined, once per wavefront */
    int64_t wave_leaf_sweeps;     /* leaves swept, once per wavefront */
    int64_t wavefronts;           /* query wavefronts run */
    /* Index reuse: refit ticks since the last full build, and the largest
     * per-axis displacement of any object since that build (0 right after
     * it), by which inner node boxes are grown during queries (leaf boxes
     * are recomputed by each refit). */
    int64_t refits;
    float drift;
    float reserved2;
} mknn_stats;

/*
 * mknn_create -- allocate a context and all its device memory, sized by
 * cfg->n_max, cfg->q_max and cfg->k_max.  *out receives the context.
 * Errors: MKNN_E_INVAL (NULL, capacities out of range), MKNN_E_NOMEM,
 * MKNN_E_DEVICE (bad device).  On error *out is set to NULL.
 */
MKNN_API int mknn_create(const mknn_config *cfg, mknn_ctx **out);

/* mknn_footprint -- device bytes mknn_create takes for cfg (no device is
 * touched), for admission decisions: each buffer of 2 MiB or more rounded
 * up to whole 2 MiB pages, as the runtime maps them, smaller ones to 256
 * bytes (the runtime may carve those from memory it already holds).
 * Errors: MKNN_E_INVAL. */
MKNN_API int mknn_footprint(const mknn_config *cfg, int64_t *bytes);

/* mknn_destroy -- wait for the context's work and free everything.  NULL is
 * allowed.  A borrowed stream is left alone. */
MKNN_API int mknn_destroy(mknn_ctx *ctx);

/*
 * mknn_load_positions -- replace the snapshot with n objects (Sec. 2.2:
 * only the latest update of each object counts).  x[i], y[i] is object i's
 * position, two arrays of n floats, host or device memory per `where`.
 * Host arrays are copied into the context and may be reused when the call
 * returns.  Device arrays are not copied: the index build reads them in
 * place, so they must stay valid and unchanged until the context's stream
 * has passed the next mknn_advance_tick.
 * Host input is validated during the call (MKNN_E_RANGE leaves the previous
 * snapshot in place).  Device input is validated on the device; a bad value
 * makes the next mknn_sync / mknn_fetch return MKNN_E_RANGE.  Errors found
 * on the device (here and in the other calls) are kept until a
 * synchronising call reports them, whichever launch -- eager or replayed
 * from a captured graph -- found them.
 * Errors: MKNN_E_INVAL, MKNN_E_CAPACITY (n > n_max), MKNN_E_RANGE.
 * After a load, mknn_advance_tick must run before the next query.
 */
MKNN_API int mknn_load_positions(mknn_ctx *ctx, const float *x, const float *y, int64_t n,
                        int32_t where);

/*
 * mknn_advance_tick -- enqueue the index build over the current snapshot
 * (Sec. 4.1: Morton codes at level 16, a stable radix sort of the objects
 * by their code at max_level (its top 2 * max_level bits; objects of one
 * max_level cell stay in id order), split of every quadrant holding more
 * than the leaf capacity up to max_level, leaf and node tables).  A lower
 * max_level sorts fewer bits (one radix pass per 8).  Asynchronous.
 * Errors: MKNN_E_STATE (nothing loaded).
 */
MKNN_API int mknn_advance_tick(mknn_ctx *ctx);

/*
 * mknn_refit_tick -- the index reuse of Sec. 4.1 (the index need not be
 * rebuilt every tick): instead of a full build, keep the last full build's
 * object order, leaves and node tables, take every object's position from
 * the current snapshot and record the largest per-axis displacement D of
 * any object since that build.  Each leaf's node box becomes the bounding
 * box of its objects' current positions; queries prune with the inner node
 * boxes grown by D (plus a rounding margin), so results stay exact; they
 * only get slower as D grows, which is the caller's signal to run a full
 * mknn_advance_tick again (e.g. when query time grows by a chosen factor
 * over the time after the last build).  The snapshot must hold as many
 * objects as at the last full build (ids are positions, so they are the
 * same objects).  Asynchronous; a bad device coordinate is reported by
 * the next mknn_sync / mknn_fetch (MKNN_E_RANGE).  mknn_index_fetch after
 * a refit returns the build's codes and order.
 * Errors: MKNN_E_STATE (nothing loaded, no full build yet, or a different
 * object count).
 */
MKNN_API int mknn_refit_tick(mknn_ctx *ctx);

/*
 * mknn_query -- enqueue one k-NN query per entry (Sec. 4.2).  Query i is
 * issued by object issuers[i] (NULL = every object 0..n-1, in order, and
 * then nq must equal n), centred on its position and excluding it, and asks
 * for ks[i] results (NULL = k_uniform for all).  Every k must be in
 * [1, k_max].  issuers and ks are int32 arrays of nq entries in host or
 * device memory per `where`; they are read before the call returns (host:
 * the call copies them and waits for the context's stream to pass the
 * copy, i.e. for the work enqueued before it) or once the stream reaches
 * the query (device: no wait).  Results stay on the device,
 * owned by the context, until the next mknn_query.
 * Graph capture: a load/advance/query sequence with device inputs enqueues
 * kernels only, so it may be captured on the context's stream and
 * replayed.  The context's host-side description of the results (nq, k,
 * entries, used by mknn_fetch and mknn_result_size) is that of the last
 * call made on the host; after replaying a captured query, issue no eager
 * query of a different shape on the context before fetching.
 * Errors: MKNN_E_INVAL (bad issuer or k, host-side), MKNN_E_STATE (no tick
 * since the last load), MKNN_E_CAPACITY (nq > q_max or, for variable k, the
 * sum of ks above q_max * k_max).
 */
MKNN_API int mknn_query(mknn_ctx *ctx, const int32_t *issuers, const int32_t *ks, int64_t nq,
               int32_t k_uniform, int32_t where);

/*
 * mknn_query_points -- enqueue one k-NN query per entry with a free centre
 * (Definition 1, Sec. 2.1: a query is q = (x, y, k) for any location).
 * Query i is centred on (qx[i], qy[i]), which must be finite and inside
 * [0,1)^2 like the objects; object exclude[i] is left out of its answer
 * (exclude NULL, or entry -1: nothing is excluded).  ks / k_uniform as for
 * mknn_query.  qx, qy, exclude and ks are arrays of nq entries in host or
 * device memory per `where`, read as for mknn_query.  A query of object s
 * is the query with centre (x[s], y[s]) and exclude s.  Results, their
 * layout and their lifetime are those of mknn_query (the two share the
 * result buffers; the last call wins); counts[i] = min(k_i, n - 1) with an
 * exclusion, min(k_i, n) without.
 * Errors: MKNN_E_RANGE (bad host centre; a bad device centre is reported
 * by the next mknn_sync / mknn_fetch), MKNN_E_INVAL (bad exclude or k,
 * NULL qx or qy, no objects), MKNN_E_STATE, MKNN_E_CAPACITY (as mknn_query).
 */
MKNN_API int mknn_query_points(mknn_ctx *ctx, const float *qx, const float *qy,
                               const int32_t *exclude, const int32_t *ks, int64_t nq,
                               int32_t k_uniform, int32_t where);

/*
 * mknn_fetch -- synchronise, then copy the last query's results into
 * caller-owned buffers (host or device per `where`).  The layout is the
 * paper's k-NN result set (Sec. 3, "k-NN queries result set layout", and
 * Fig. 1): one linear list of k slots per query, query after query, each
 * slot an (object id, distance) pair -- the ID and DIST outputs of Alg. 1
 * -- with the number of valid slots per query kept apart (Alg. 1's
 * NUMRES).  Here the ids and the squared distances are two parallel
 * arrays of slots, and a list is sorted ascending by (d2, id).  Rows are
 * in query order.  Uniform k: ids and d2 are dense row-major [nq][k]; offsets may be
 * NULL.  Variable k: row i occupies entries offsets[i] .. offsets[i+1]-1
 * (offsets has nq+1 int64 entries, offsets[i+1]-offsets[i] = ks[i]).
 * counts[i] = min(k_i, n-1).  Any of ids, d2, counts, offsets may be NULL
 * to skip it.  Sizes: see mknn_result_size.
 * Errors: MKNN_E_STATE (no query yet), MKNN_E_RANGE (bad device input),
 * MKNN_E_DEVICE.
 */
MKNN_API int mknn_fetch(mknn_ctx *ctx, int32_t *ids, float *d2, int32_t *counts, int64_t *offsets,
               int32_t where);

/* mknn_result_size -- number of queries and of result entries (row slots)
 * of the last query. */
MKNN_API int mknn_result_size(const mknn_ctx *ctx, int64_t *nq, int64_t *entries);

/*
 * mknn_result_device -- device pointers to the last query's results inside
 * the context (valid until the next mknn_query or mknn_destroy; do not
 * free).  Same layout as mknn_fetch.  offsets is NULL for uniform k.  The
 * results are complete once the context's stream has passed the query.
 */
MKNN_API int mknn_result_device(const mknn_ctx *ctx, const int32_t **ids, const float **d2,
                       const int32_t **counts, const int64_t **offsets);

/*
 * mknn_index_fetch -- synchronise and copy the current index to host
 * buffers, for inspection and tests.  Objects: codes[n] (level-16 Morton
 * codes in sorted order: ascending by their top 2 * max_level bits, then by
 * id) and ids[n] (object id at each sorted position).
 * Leaves, in Morton order: level[L], prefix[L] (quadrant id at its level),
 * begin[L], end[L] (half-open range of sorted positions); leaf_cap is the
 * room in the leaf arrays, *n_leaves receives the leaf count (the call
 * returns MKNN_E_CAPACITY if it exceeds leaf_cap).  Any array may be NULL.
 */
MKNN_API int mknn_index_fetch(mknn_ctx *ctx, uint32_t *codes, int32_t *ids, int32_t *level,
                     uint32_t *prefix, int64_t *begin, int64_t *end, int64_t leaf_cap,
                     int64_t *n_leaves);

/* mknn_sync -- wait for all enqueued work; reports deferred errors. */
MKNN_API int mknn_sync(mknn_ctx *ctx);

/* mknn_get_stats -- counters of the current index and last query; device
 * times need MKNN_FLAG_TIMING and a prior mknn_sync. */
MKNN_API int mknn_get_stats(const mknn_ctx *ctx, mknn_stats *out);

/*
 * mknn_set_leaf_capacity -- use leaf capacity th (Sec. 4.1) for the next
 * index builds.  The node tables were sized at mknn_create for the
 * configured capacity; a smaller th may need more nodes, so th below the
 * configured value returns MKNN_E_CAPACITY unless the tables still fit
 * (create with the smallest th you intend to use).  Results never depend on
 * th.  Errors: MKNN_E_INVAL (th < 1), MKNN_E_CAPACITY.
 */
MKNN_API int mknn_set_leaf_capacity(mknn_ctx *ctx, int32_t th);

/*
 * Tuning knobs of a context, for an autotuner (results never depend on
 * them).  leaf_capacity is th (Sec. 4.1); max_level is l_max (Sec. 4.1,
 * 1..16); sweep is an MKNN_SWEEP_* flavour (LANE applies to k <= 128;
 * larger k then use WAVE); group_k != 0 behaves as MKNN_FLAG_GROUP_K
 * (variable-k queries answered per k class, lane or group flavour).
 * tile_queries is the number of queries a wavefront of the lane flavour
 * answers together (Sec. 4.2.1's grouping of nearby queries into one task):
 * 64, 32, 16 or 8, or 0 for automatic (64, halved down to 8 while the
 * launch still fits the GPU's resident wavefronts in one round: a launch
 * too small to fill the GPU then finishes sooner, since fewer queries per
 * wavefront share a smaller candidate set).  The index settings take
 * effect at the next mknn_advance_tick, the sweep settings at the next
 * query.
 */
typedef struct mknn_schedule {
    int32_t leaf_capacity;
    int32_t max_level;
    int32_t sweep;
    int32_t group_k;
    int32_t tile_queries;
} mknn_schedule;

/* mknn_get_schedule -- the settings in force.  Errors: MKNN_E_INVAL. */
MKNN_API int mknn_get_schedule(const mknn_ctx *ctx, mknn_schedule *out);

/*
 * mknn_set_schedule -- change every setting at once.  The node tables were
 * sized at mknn_create; a leaf capacity below, or a maximum level above,
 * the configured ones may need more nodes: such a schedule returns
 * MKNN_E_CAPACITY unless the tables still fit.  Errors: MKNN_E_INVAL
 * (leaf_capacity < 1, max_level outside 1..16, unknown sweep, tile_queries
 * not 0, 8, 16, 32 or 64), MKNN_E_CAPACITY.  On error nothing changes.
 */
MKNN_API int mknn_set_schedule(mknn_ctx *ctx, const mknn_schedule *s);

/*
 * mknn_set_epochs -- testing hook: the tags the next index step and query
 * will be one past (build_epoch, query_epoch), both in 1 .. 2^24-1.  Tags
 * wrap from 2^24-1 to 1; this lets a test cross the wrap without running
 * 2^24 ticks.  Results never depend on the tags.  Errors: MKNN_E_INVAL.
 */
MKNN_API int mknn_set_epochs(mknn_ctx *ctx, uint32_t build_epoch, uint32_t query_epoch);

/* mknn_reset_timing -- forget the device times and counters recorded so far
 * (the means and totals in mknn_stats restart). */
MKNN_API int mknn_reset_timing(mknn_ctx *ctx);

/*
 * mknn_query_time -- device time in ms (all kernels) of an earlier query:
 * back = 0 is the last query enqueued, 1 the one before, and so on (up to
 * 255).  With wait = 0 it never blocks; with wait != 0 it waits for that
 * query only (not for later work on the stream).  For decisions taken while
 * later ticks are still running, such as when to rebuild the index (Sec.
 * 4.1): waiting for the query two ticks back keeps the host at most two
 * ticks ahead without ever leaving the GPU idle, unlike mknn_get_stats,
 * which synchronises the stream.  Needs MKNN_FLAG_TIMING.
 * Errors: MKNN_E_INVAL (NULL, back out of range, no such query yet),
 * MKNN_E_STATE (wait = 0 and that query has not finished, or it was not
 * timed; *ms is left unchanged).
 */
MKNN_API int mknn_query_time(const mknn_ctx *ctx, int32_t back, int32_t wait, float *ms);

/* mknn_last_error -- message of the context's last error ("" if none). */
MKNN_API const char *mknn_last_error(const mknn_ctx *ctx);

/* mknn_status_str -- name of a status code. */
MKNN_API const char *mknn_status_str(int status);

/* mknn_default_leaf_capacity -- the automatic leaf capacity for a given k. */
MKNN_API int32_t mknn_default_leaf_capacity(int32_t k);

/* Largest object count and scratch size of mknn_knn_noalloc. */
#define MKNN_NOALLOC_MAX_N 65536
#define MKNN_NOALLOC_SCRATCH_BYTES (16 << 20)

/*
 * mknn_knn_noalloc -- one whole tick without allocating: the index build of
 * mknn_advance_tick and the query of mknn_query with every object querying
 * (issuers NULL, uniform k), in one call that calls no hipMalloc, hipFree or
 * other allocating routine.  For callers that cannot allocate device
 * memory: code being captured into a HIP graph, tight serving loops, hosts
 * that forbid allocation after start-up.
 *
 * x, y      device, n fp32 coordinates each, object id = index (as
 *           mknn_load_positions with MKNN_DEVICE); read in place.
 * n         0 .. MKNN_NOALLOC_MAX_N.
 * k         1 .. MKNN_K_LIMIT; lists of up to 32 keys run one query per
 *           lane, larger ones a group of lanes per query (the flavours
 *           mknn_query's AUTO schedule picks).
 * leaf_capacity  0 = mknn_default_leaf_capacity(k); the maximum level is 16.
 * ids, d2   device, n * k entries each: row i (object i's query, object i
 *           excluded) is the dense row mknn_fetch returns for uniform k.
 * counts    device, n entries: min(k, n - 1).
 * status    device, one int32, or NULL: set to 0 when the tick's device
 *           checks pass, else MKNN_E_RANGE (a coordinate not finite or
 *           outside [0,1)) or MKNN_E_DEVICE (a look-back wait gave up or a
 *           node table overflowed); the rows are then unspecified.
 * stream    hipStream_t the work is enqueued on (NULL: the null stream).
 *
 * Every intermediate buffer (sort buffers, leaves, node tables, look-back
 * words, counters) is carved from one device array of
 * MKNN_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends; its address is looked up once per device on the
 * first call there (the device current at the call).  The call only
 * enqueues work and returns; nothing is read back.  Every call on one GPU
 * shares that GPU's array: calls whose work overlaps on one GPU (on
 * different streams, or from different host threads) race and give wrong
 * rows.  Each call clears what must start at zero itself.
 *
 * Errors: MKNN_E_INVAL (NULL pointer with n > 0, n < 0, k outside
 * [1, MKNN_K_LIMIT], leaf_capacity < 0), MKNN_E_CAPACITY (n above
 * MKNN_NOALLOC_MAX_N, or the buffers for n and leaf_capacity do not fit the
 * array: leaf capacities of 16 or more always fit), MKNN_E_DEVICE (a HIP
 * error while looking up the array or launching).
 */
MKNN_API int mknn_knn_noalloc(const float *x, const float *y, int64_t n, int32_t k,
                              int32_t leaf_capacity, int32_t *ids, float *d2, int32_t *counts,
                              int32_t *status, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MKNN_H */
