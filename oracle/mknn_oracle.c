/*
 * mknn_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU reference for the per-tick k-NN join over
 * moving 2D objects (Lettich, Orlando, Silvestri, "Manycore processing of
 * repeated k-NN queries over massive moving objects observations",
 * arXiv 1412.6170).  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header or table
 * with the GPU library; the product path never calls it.
 *
 * What it computes
 * ----------------
 *   * The k-NN result of Definition 1 (Sec. 2.1): for a query issued by object
 *     s, centred on s's position, the k objects (s itself excluded) of lowest
 *     rank.  Ties are broken by ascending object id, so the answer is unique.
 *     Distances are ranked and returned as the squared fp32 distance
 *         d2 = fl( fl(fl(qx-px)*fl(qx-px)) + fl(fl(qy-py)*fl(qy-py)) )
 *     in IEEE binary32, round-to-nearest-even, denormals kept, no fused
 *     multiply-add (this file must be compiled with -ffp-contract=off and
 *     without -ffast-math).
 *   * oracle_brute_knn: that definition written out (every object is a
 *     candidate).  Pinned against closed forms and a numpy brute force.
 *   * oracle_build_index: the index of Sec. 4.1 -- Morton codes on the
 *     virtual full quadtree of height L (the maximum level; the level-L code
 *     is the level-16 code without its 2(16-L) low bits), a sort of the
 *     objects by (level-L code, id), and the level-by-level PR-quadtree split
 *     of every quadrant holding more than th objects, up to level L (leaves
 *     at L may exceed th).  The level-16 code of every object is kept: it
 *     places the object in its quadrant at every level.
 *   * oracle_brute_knn_points / oracle_knn_points: the same two searches
 *     for queries q = (x, y, k) with a free centre in [0,1)^2 (Definition
 *     1) and an optional excluded object id.
 *   * oracle_knn: a sequential quadtree k-NN over that index: a depth-first
 *     visit that enters children in ascending box lower bound and prunes a
 *     quadrant whose lower bound is strictly greater than the current k-th
 *     squared distance (Sec. 4.2.2: a leaf may hold neighbours only if its
 *     borders are nearer than the farthest object found so far).  It returns
 *     exactly the brute-force result: the lower bound is computed with the
 *     same rounded operations as d2 on the box edge, and fp32 subtraction,
 *     multiplication and addition round monotonically, so no point of a
 *     pruned box can reach the k-th key.
 *
 * Every function returns 0 on success or a negative code:
 *   -1 invalid argument, -2 coordinate not finite or outside [0,1),
 *   -5 out of memory.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ERANGE (-2)
#define OR_ENOMEM (-5)

#define CODE_LEVELS 16 /* Morton codes are taken at level 16: 32-bit codes */

/* ------------------------------------------------------------------------ */
/* Squared distance and the total-order key (Definition 1, ties by id).     */
/* ------------------------------------------------------------------------ */

static float sq_dist(float qx, float qy, float px, float py)
{
    float dx = qx - px;
    float dy = qy - py;
    float ax = dx * dx;
    float ay = dy * dy;
    return ax + ay;
}

/* Squared distances are never negative and never NaN for inputs in [0,1),
 * so their bit patterns order like their values; the key orders by d2 first
 * and by object id second. */
static uint64_t make_key(float d2, int32_t id)
{
    uint32_t bits;
    memcpy(&bits, &d2, sizeof bits);
    return ((uint64_t)bits << 32) | (uint32_t)id;
}

static float key_d2(uint64_t key)
{
    uint32_t bits = (uint32_t)(key >> 32);
    float f;
    memcpy(&f, &bits, sizeof f);
    return f;
}

/* ------------------------------------------------------------------------ */
/* Validation and Morton codes (Sec. 4.1, index creation).                  */
/* ------------------------------------------------------------------------ */

int oracle_validate(const float *x, const float *y, int64_t n)
{
    if (n < 0 || (n > 0 && (!x || !y)))
        return OR_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(x[i]) || !isfinite(y[i]))
            return OR_ERANGE;
        if (!(x[i] >= 0.0f && x[i] < 1.0f && y[i] >= 0.0f && y[i] < 1.0f))
            return OR_ERANGE;
    }
    return OR_OK;
}

/* The cell of the 2^16 x 2^16 uniform grid (the virtual full quadtree at
 * level 16) holding a coordinate in [0,1): scaling by 2^16 is exact in fp32
 * and the conversion truncates, i.e. takes the floor. */
static uint32_t grid_cell(float v)
{
    float s = v * 65536.0f;
    uint32_t c = (uint32_t)s;
    return c;
}

/* Interleave: bit b of the x cell goes to bit 2b, bit b of the y cell to
 * bit 2b+1.  Written as the plain definition, one bit at a time. */
uint32_t oracle_morton(float x, float y)
{
    uint32_t cx = grid_cell(x), cy = grid_cell(y), code = 0;
    for (int b = 0; b < CODE_LEVELS; ++b) {
        code |= ((cx >> b) & 1u) << (2 * b);
        code |= ((cy >> b) & 1u) << (2 * b + 1);
    }
    return code;
}

/* Inverse of the interleave, used to recover a quadrant's box. */
static void morton_cells(uint32_t code, uint32_t *cx, uint32_t *cy)
{
    uint32_t a = 0, b = 0;
    for (int i = 0; i < CODE_LEVELS; ++i) {
        a |= ((code >> (2 * i)) & 1u) << i;
        b |= ((code >> (2 * i + 1)) & 1u) << i;
    }
    *cx = a;
    *cy = b;
}

int oracle_morton_codes(const float *x, const float *y, int64_t n, uint32_t *codes)
{
    int rc = oracle_validate(x, y, n);
    if (rc)
        return rc;
    if (n > 0 && !codes)
        return OR_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        codes[i] = oracle_morton(x[i], y[i]);
    return OR_OK;
}

/* The level-l quadrant that contains a level-16 code: z' = floor(z / 4^(16-l))
 * (Sec. 4.1, ancestor property). */
static uint32_t ancestor(uint32_t code, int level)
{
    if (level <= 0)
        return 0;
    return code >> (2 * (CODE_LEVELS - level));
}

/* ------------------------------------------------------------------------ */
/* Index: sort by (code, id) and split quadrants holding more than th.      */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t code; /* level-16 code */
    uint32_t key;  /* Morton code at the maximum level L: the sort key */
    int32_t id;
} obj_ref;

static int cmp_obj(const void *pa, const void *pb)
{
    const obj_ref *a = (const obj_ref *)pa, *b = (const obj_ref *)pb;
    if (a->key != b->key)
        return a->key < b->key ? -1 : 1;
    if (a->id != b->id)
        return a->id < b->id ? -1 : 1;
    return 0;
}

/* Quadtree node.  Leaves hold the half-open interval [begin,end) of the
 * sorted objects (possibly empty); inner nodes have four children, in
 * Morton order 0..3. */
typedef struct {
    int level;
    uint32_t prefix; /* quadrant id at its level */
    int64_t begin, end;
    int64_t child[4]; /* -1 for leaves */
    float x0, y0, x1, y1;
} qnode;

typedef struct {
    qnode *nodes;
    int64_t count, cap;
} node_vec;

static int64_t push_node(node_vec *v, const qnode *nd)
{
    if (v->count == v->cap) {
        int64_t ncap = v->cap ? 2 * v->cap : 64;
        qnode *p = (qnode *)realloc(v->nodes, (size_t)ncap * sizeof(qnode));
        if (!p)
            return -1;
        v->nodes = p;
        v->cap = ncap;
    }
    v->nodes[v->count] = *nd;
    return v->count++;
}

static void set_box(qnode *nd)
{
    /* Box of quadrant (level, prefix): [cx*2^-l, (cx+1)*2^-l) along x, same
     * for y; every edge is a multiple of 2^-16 below or at 1 and is exact. */
    uint32_t full = nd->level > 0 ? nd->prefix << (2 * (CODE_LEVELS - nd->level)) : 0;
    uint32_t cx, cy;
    morton_cells(full, &cx, &cy);
    uint32_t side = 1u << (CODE_LEVELS - nd->level);
    nd->x0 = (float)cx / 65536.0f;
    nd->y0 = (float)cy / 65536.0f;
    nd->x1 = (float)(cx + side) / 65536.0f;
    nd->y1 = (float)(cy + side) / 65536.0f;
}

/* Split [begin,end) at `level` if it holds more than th objects and
 * level < L; the four children are the runs of equal level+1 ancestors. */
static int64_t build_node(node_vec *v, const obj_ref *objs, int level, uint32_t prefix,
                          int64_t begin, int64_t end, int th, int L)
{
    qnode nd;
    memset(&nd, 0, sizeof nd);
    nd.level = level;
    nd.prefix = prefix;
    nd.begin = begin;
    nd.end = end;
    for (int c = 0; c < 4; ++c)
        nd.child[c] = -1;
    set_box(&nd);
    int64_t self = push_node(v, &nd);
    if (self < 0)
        return -1;
    if (end - begin > th && level < L) {
        int64_t start = begin;
        for (int c = 0; c < 4; ++c) {
            uint32_t want = prefix * 4u + (uint32_t)c;
            int64_t stop = start;
            while (stop < end && ancestor(objs[stop].code, level + 1) == want)
                ++stop;
            int64_t ch = build_node(v, objs, level + 1, want, start, stop, th, L);
            if (ch < 0)
                return -1;
            v->nodes[self].child[c] = ch;
            start = stop;
        }
    }
    return self;
}

typedef struct {
    int64_t n;
    obj_ref *objs; /* sorted by (level-L code, id) */
    float *sx, *sy; /* positions in sorted order */
    node_vec tree;
} qindex;

static void free_index(qindex *ix)
{
    free(ix->objs);
    free(ix->sx);
    free(ix->sy);
    free(ix->tree.nodes);
    memset(ix, 0, sizeof *ix);
}

static int make_index(const float *x, const float *y, int64_t n, int th, int L, qindex *ix)
{
    memset(ix, 0, sizeof *ix);
    int rc = oracle_validate(x, y, n);
    if (rc)
        return rc;
    if (th < 1 || L < 1 || L > CODE_LEVELS)
        return OR_EINVAL;
    ix->n = n;
    size_t m = n > 0 ? (size_t)n : 1;
    ix->objs = (obj_ref *)malloc(m * sizeof(obj_ref));
    ix->sx = (float *)malloc(m * sizeof(float));
    ix->sy = (float *)malloc(m * sizeof(float));
    if (!ix->objs || !ix->sx || !ix->sy) {
        free_index(ix);
        return OR_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        ix->objs[i].code = oracle_morton(x[i], y[i]);
        ix->objs[i].key = ancestor(ix->objs[i].code, L);
        ix->objs[i].id = (int32_t)i;
    }
    qsort(ix->objs, (size_t)n, sizeof(obj_ref), cmp_obj);
    for (int64_t i = 0; i < n; ++i) {
        ix->sx[i] = x[ix->objs[i].id];
        ix->sy[i] = y[ix->objs[i].id];
    }
    if (build_node(&ix->tree, ix->objs, 0, 0, 0, n, th, L) < 0) {
        free_index(ix);
        return OR_ENOMEM;
    }
    return OR_OK;
}

/*
 * oracle_build_index: sorted codes and ids, and the non-empty leaves in
 * Morton order (level, quadrant id, [begin,end)).  *n_leaves receives the
 * number of non-empty leaves even when leaf_cap is too small (then the
 * arrays hold the first leaf_cap and -1 is returned); *n_empty the number
 * of empty leaves produced by splits.
 */
int oracle_build_index(const float *x, const float *y, int64_t n, int32_t th, int32_t L,
                       uint32_t *codes_sorted, int32_t *ids_sorted, int32_t *leaf_level,
                       uint32_t *leaf_prefix, int64_t *leaf_begin, int64_t *leaf_end,
                       int64_t leaf_cap, int64_t *n_leaves, int64_t *n_empty)
{
    qindex ix;
    int rc = make_index(x, y, n, th, L, &ix);
    if (rc)
        return rc;
    for (int64_t i = 0; i < n; ++i) {
        if (codes_sorted)
            codes_sorted[i] = ix.objs[i].code;
        if (ids_sorted)
            ids_sorted[i] = ix.objs[i].id;
    }
    int64_t nl = 0, ne = 0;
    for (int64_t k = 0; k < ix.tree.count; ++k) {
        const qnode *nd = &ix.tree.nodes[k];
        if (nd->child[0] >= 0)
            continue;
        if (nd->end == nd->begin) {
            ++ne;
            continue;
        }
        if (nl < leaf_cap) {
            leaf_level[nl] = nd->level;
            leaf_prefix[nl] = nd->prefix;
            leaf_begin[nl] = nd->begin;
            leaf_end[nl] = nd->end;
        }
        ++nl;
    }
    /* Nodes were created depth-first in child order 0..3, so leaves came out
     * in Morton order. */
    if (n_leaves)
        *n_leaves = nl;
    if (n_empty)
        *n_empty = ne;
    free_index(&ix);
    return nl > leaf_cap ? OR_EINVAL : OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Bounded max-heap of keys: the current best k candidates of one query.    */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t *a;
    int size, cap;
} kheap;

static void heap_sift_down(kheap *h, int i)
{
    for (;;) {
        int l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->size && h->a[l] > h->a[m])
            m = l;
        if (r < h->size && h->a[r] > h->a[m])
            m = r;
        if (m == i)
            return;
        uint64_t t = h->a[i];
        h->a[i] = h->a[m];
        h->a[m] = t;
        i = m;
    }
}

static void heap_offer(kheap *h, uint64_t key)
{
    if (h->cap == 0)
        return;
    if (h->size < h->cap) {
        int i = h->size++;
        h->a[i] = key;
        while (i > 0) {
            int p = (i - 1) / 2;
            if (h->a[p] >= h->a[i])
                break;
            uint64_t t = h->a[p];
            h->a[p] = h->a[i];
            h->a[i] = t;
            i = p;
        }
    } else if (key < h->a[0]) {
        h->a[0] = key;
        heap_sift_down(h, 0);
    }
}

static int cmp_u64(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Write the heap ascending into a result row of capacity k, padding with
 * id -1 and d2 +inf. */
static void emit_row(kheap *h, int k, int32_t *ids, float *d2, int32_t *count)
{
    qsort(h->a, (size_t)h->size, sizeof(uint64_t), cmp_u64);
    for (int j = 0; j < k; ++j) {
        if (j < h->size) {
            ids[j] = (int32_t)(uint32_t)(h->a[j] & 0xffffffffu);
            d2[j] = key_d2(h->a[j]);
        } else {
            ids[j] = -1;
            d2[j] = INFINITY;
        }
    }
    *count = h->size;
}

/* ------------------------------------------------------------------------ */
/* Quadtree k-NN of one query (Sec. 4.2: own leaf first, then neighbouring  */
/* leaves whose borders are nearer than the current farthest result).       */
/* ------------------------------------------------------------------------ */

/* Lower bound of d2 from (qx,qy) to any point of the box, with the same
 * rounded operations as sq_dist applied to the nearest box edge. */
static float box_lower_bound(const qnode *nd, float qx, float qy)
{
    float gx = 0.0f, gy = 0.0f;
    if (qx < nd->x0)
        gx = nd->x0 - qx;
    else if (qx >= nd->x1)
        gx = qx - nd->x1;
    if (qy < nd->y0)
        gy = nd->y0 - qy;
    else if (qy >= nd->y1)
        gy = qy - nd->y1;
    float ax = gx * gx;
    float ay = gy * gy;
    return ax + ay;
}

static void dfs(const qindex *ix, int64_t node, float qx, float qy, int32_t self, kheap *h)
{
    const qnode *nd = &ix->tree.nodes[node];
    if (nd->child[0] < 0) {
        for (int64_t j = nd->begin; j < nd->end; ++j) {
            if (ix->objs[j].id == self)
                continue;
            heap_offer(h, make_key(sq_dist(qx, qy, ix->sx[j], ix->sy[j]), ix->objs[j].id));
        }
        return;
    }
    float lb[4];
    int order[4];
    for (int c = 0; c < 4; ++c) {
        lb[c] = box_lower_bound(&ix->tree.nodes[nd->child[c]], qx, qy);
        order[c] = c;
    }
    /* Enter the children in ascending lower bound (ties by child index). */
    for (int a = 1; a < 4; ++a)
        for (int b = a; b > 0 && lb[order[b]] < lb[order[b - 1]]; --b) {
            int t = order[b];
            order[b] = order[b - 1];
            order[b - 1] = t;
        }
    for (int a = 0; a < 4; ++a) {
        int c = order[a];
        const qnode *ch = &ix->tree.nodes[nd->child[c]];
        if (ch->end == ch->begin)
            continue;
        /* Prune only when the box is strictly farther than the k-th key's
         * distance; at equality a tie with a smaller id may still enter. */
        if (h->size == h->cap && lb[c] > key_d2(h->a[0]))
            continue;
        dfs(ix, nd->child[c], qx, qy, self, h);
    }
}

/* ------------------------------------------------------------------------ */
/* Query batches: issuers[i] (NULL = all objects 0..n-1 in order) and       */
/* ks[i] (NULL = k_uniform).  Row i of the output starts at offsets[i]      */
/* (NULL = i*k_uniform) and holds ks[i] slots.                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    const qindex *ix;     /* quadtree search when set */
    const float *x, *y;   /* brute force when ix is NULL */
    int64_t n;
    /* Free query centres (Definition 1's q = (x, y, k)): when qx is set,
     * query i is centred on (qx[i], qy[i]) and excludes object exclude[i]
     * (NULL or -1: nothing excluded); issuers is then unused. */
    const float *qx, *qy;
    const int32_t *exclude;
    const int32_t *issuers;
    const int32_t *ks;
    int32_t k_uniform;
    const int64_t *offsets;
    int32_t *out_ids;
    float *out_d2;
    int32_t *out_count;
    int64_t q_begin, q_end;
    int status;
} batch_job;

static void run_one(const batch_job *jb, int64_t q, kheap *h)
{
    int32_t s;
    float qx, qy;
    if (jb->qx) {
        s = jb->exclude ? jb->exclude[q] : -1;
        qx = jb->qx[q];
        qy = jb->qy[q];
    } else {
        s = jb->issuers ? jb->issuers[q] : (int32_t)q;
        qx = jb->x[s];
        qy = jb->y[s];
    }
    int32_t k = jb->ks ? jb->ks[q] : jb->k_uniform;
    int64_t off = jb->offsets ? jb->offsets[q] : q * (int64_t)jb->k_uniform;
    /* Candidates: every object but the excluded one (if any). */
    int64_t others = jb->n - (s >= 0 ? 1 : 0);
    h->size = 0;
    h->cap = (int)((int64_t)k < others ? k : (others > 0 ? others : 0));
    if (jb->ix) {
        if (jb->n > 0 && h->cap > 0)
            dfs(jb->ix, 0, qx, qy, s, h);
    } else {
        for (int64_t j = 0; j < jb->n; ++j) {
            if (j == s)
                continue;
            heap_offer(h, make_key(sq_dist(qx, qy, jb->x[j], jb->y[j]), (int32_t)j));
        }
    }
    emit_row(h, k, jb->out_ids + off, jb->out_d2 + off, jb->out_count + q);
}

static void *job_main(void *arg)
{
    batch_job *jb = (batch_job *)arg;
    int32_t kmax = jb->k_uniform;
    if (jb->ks)
        for (int64_t q = jb->q_begin; q < jb->q_end; ++q)
            if (jb->ks[q] > kmax)
                kmax = jb->ks[q];
    kheap h;
    h.a = (uint64_t *)malloc((size_t)(kmax > 0 ? kmax : 1) * sizeof(uint64_t));
    if (!h.a) {
        jb->status = OR_ENOMEM;
        return NULL;
    }
    for (int64_t q = jb->q_begin; q < jb->q_end; ++q)
        run_one(jb, q, &h);
    free(h.a);
    jb->status = OR_OK;
    return NULL;
}

static int check_queries(int64_t n, const int32_t *issuers, const int32_t *ks, int64_t nq,
                         int32_t k_uniform, const int64_t *offsets)
{
    if (nq < 0 || (!issuers && nq != n))
        return OR_EINVAL;
    if (!ks && k_uniform < 1)
        return OR_EINVAL;
    if (ks && !offsets)
        return OR_EINVAL;
    for (int64_t q = 0; q < nq; ++q) {
        if (issuers && (issuers[q] < 0 || issuers[q] >= n))
            return OR_EINVAL;
        if (ks && ks[q] < 1)
            return OR_EINVAL;
    }
    return OR_OK;
}

/* Free centres: finite, inside [0,1)^2 like the objects; exclude[i] is -1
 * or an object id. */
static int check_points(int64_t n, const float *qx, const float *qy, const int32_t *exclude,
                        const int32_t *ks, int64_t nq, int32_t k_uniform, const int64_t *offsets)
{
    if (nq < 0 || !qx || !qy)
        return OR_EINVAL;
    if (!ks && k_uniform < 1)
        return OR_EINVAL;
    if (ks && !offsets)
        return OR_EINVAL;
    for (int64_t q = 0; q < nq; ++q) {
        if (!(qx[q] >= 0.0f && qx[q] < 1.0f && qy[q] >= 0.0f && qy[q] < 1.0f))
            return OR_ERANGE;
        if (exclude && (exclude[q] < -1 || exclude[q] >= n))
            return OR_EINVAL;
        if (ks && ks[q] < 1)
            return OR_EINVAL;
    }
    return OR_OK;
}

static int run_batch(batch_job *proto, int64_t nq, int threads)
{
    if (threads < 1)
        threads = 1;
    if (threads > 256)
        threads = 256;
    if ((int64_t)threads > nq)
        threads = nq > 0 ? (int)nq : 1;
    batch_job jobs[256];
    pthread_t tids[256];
    int started[256];
    for (int t = 0; t < threads; ++t) {
        jobs[t] = *proto;
        jobs[t].q_begin = nq * t / threads;
        jobs[t].q_end = nq * (t + 1) / threads;
        jobs[t].status = OR_OK;
        started[t] = 0;
    }
    for (int t = 1; t < threads; ++t)
        started[t] = pthread_create(&tids[t], NULL, job_main, &jobs[t]) == 0;
    job_main(&jobs[0]);
    for (int t = 1; t < threads; ++t) {
        if (started[t])
            pthread_join(tids[t], NULL);
        else
            job_main(&jobs[t]);
    }
    for (int t = 0; t < threads; ++t)
        if (jobs[t].status)
            return jobs[t].status;
    return OR_OK;
}

/* Definition 1 written out: every other object is a candidate. */
int oracle_brute_knn(const float *x, const float *y, int64_t n, const int32_t *issuers,
                     const int32_t *ks, int64_t nq, int32_t k_uniform, const int64_t *offsets,
                     int32_t *out_ids, float *out_d2, int32_t *out_count, int32_t threads)
{
    int rc = oracle_validate(x, y, n);
    if (rc)
        return rc;
    rc = check_queries(n, issuers, ks, nq, k_uniform, offsets);
    if (rc)
        return rc;
    batch_job proto;
    memset(&proto, 0, sizeof proto);
    proto.x = x;
    proto.y = y;
    proto.n = n;
    proto.issuers = issuers;
    proto.ks = ks;
    proto.k_uniform = k_uniform;
    proto.offsets = offsets;
    proto.out_ids = out_ids;
    proto.out_d2 = out_d2;
    proto.out_count = out_count;
    return run_batch(&proto, nq, threads);
}

/* Sequential quadtree k-NN: build the index (Sec. 4.1) then answer every
 * query with the pruned depth-first visit.  Same output contract as
 * oracle_brute_knn. */
int oracle_knn(const float *x, const float *y, int64_t n, const int32_t *issuers,
               const int32_t *ks, int64_t nq, int32_t k_uniform, const int64_t *offsets,
               int32_t th, int32_t L, int32_t *out_ids, float *out_d2, int32_t *out_count,
               int32_t threads)
{
    int rc = check_queries(n, issuers, ks, nq, k_uniform, offsets);
    if (rc)
        return rc;
    qindex ix;
    rc = make_index(x, y, n, th, L, &ix);
    if (rc)
        return rc;
    batch_job proto;
    memset(&proto, 0, sizeof proto);
    proto.ix = &ix;
    proto.x = x;
    proto.y = y;
    proto.n = n;
    proto.issuers = issuers;
    proto.ks = ks;
    proto.k_uniform = k_uniform;
    proto.offsets = offsets;
    proto.out_ids = out_ids;
    proto.out_d2 = out_d2;
    proto.out_count = out_count;
    rc = run_batch(&proto, nq, threads);
    free_index(&ix);
    return rc;
}

/* Definition 1 with a free centre: query i is q = (qx[i], qy[i], k_i), and
 * object exclude[i] (if not NULL and not -1) is left out.  Every other
 * object is a candidate; ties by id.  Rows hold min(k_i, candidates). */
int oracle_brute_knn_points(const float *x, const float *y, int64_t n, const float *qx,
                            const float *qy, const int32_t *exclude, const int32_t *ks,
                            int64_t nq, int32_t k_uniform, const int64_t *offsets,
                            int32_t *out_ids, float *out_d2, int32_t *out_count, int32_t threads)
{
    int rc = oracle_validate(x, y, n);
    if (rc)
        return rc;
    rc = check_points(n, qx, qy, exclude, ks, nq, k_uniform, offsets);
    if (rc)
        return rc;
    batch_job proto;
    memset(&proto, 0, sizeof proto);
    proto.x = x;
    proto.y = y;
    proto.n = n;
    proto.qx = qx;
    proto.qy = qy;
    proto.exclude = exclude;
    proto.ks = ks;
    proto.k_uniform = k_uniform;
    proto.offsets = offsets;
    proto.out_ids = out_ids;
    proto.out_d2 = out_d2;
    proto.out_count = out_count;
    return run_batch(&proto, nq, threads);
}

/* The quadtree search of oracle_knn with free centres (same contract as
 * oracle_brute_knn_points). */
int oracle_knn_points(const float *x, const float *y, int64_t n, const float *qx,
                      const float *qy, const int32_t *exclude, const int32_t *ks, int64_t nq,
                      int32_t k_uniform, const int64_t *offsets, int32_t th, int32_t L,
                      int32_t *out_ids, float *out_d2, int32_t *out_count, int32_t threads)
{
    int rc = check_points(n, qx, qy, exclude, ks, nq, k_uniform, offsets);
    if (rc)
        return rc;
    qindex ix;
    rc = make_index(x, y, n, th, L, &ix);
    if (rc)
        return rc;
    batch_job proto;
    memset(&proto, 0, sizeof proto);
    proto.ix = &ix;
    proto.x = x;
    proto.y = y;
    proto.n = n;
    proto.qx = qx;
    proto.qy = qy;
    proto.exclude = exclude;
    proto.ks = ks;
    proto.k_uniform = k_uniform;
    proto.offsets = offsets;
    proto.out_ids = out_ids;
    proto.out_d2 = out_d2;
    proto.out_count = out_count;
    rc = run_batch(&proto, nq, threads);
    free_index(&ix);
    return rc;
}

/* The squared distance exactly as the oracle rounds it; lets tests probe
 * the arithmetic (no contraction, denormals kept) on chosen operands. */
float oracle_sq_dist(float qx, float qy, float px, float py)
{
    return sq_dist(qx, qy, px, py);
}
