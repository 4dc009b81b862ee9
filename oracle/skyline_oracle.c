/*
 * CPU oracle for the SkyCell exact-skyline path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: it exists so that tests, the smoke check and the CPU
 * baseline in the benchmark can compare the GPU result with a plain, slow,
 * obviously correct computation.  It shares no code with the HIP library.
 *
 * What is computed (SkyCell paper, Section III):
 *   Definition 1 (point domination):  p dominates q  iff  p[k] <= q[k] for
 *       every dimension k and p[l] < q[l] for at least one dimension l
 *       (smaller is better, Section I).
 *   Definition 2 (skyline):  the points not dominated by any other point.
 *   The skyline set is unique; the oracle returns it as ascending indices.
 *   Exact copies never dominate each other, so every copy of a skyline point
 *   is reported.
 *
 * Arithmetic: inputs (binary32 or uint16) are widened to binary64, which is
 * exact, and only compared.  The one place floating point decides an integer
 * is the cell quantiser (Equation 1); it multiplies in binary32 with
 * round-to-nearest, the precision the GPU kernel uses, then floors.
 *
 * Algorithms:
 *   O1  brute force, O(n^2 d): the definition written out.
 *   O2  sort-first skyline (SFS, Section II-A; also the per-cell refine the
 *       paper names in Section V): points sorted by an exact linear extension
 *       of the dominance order, a window of accepted points, blocked so that
 *       host threads can share the work.
 *   Per-index check: is one point dominated by any point (brute force), for
 *       sampled parity at sizes where O1/O2 are too slow.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_NAN (-6)
#define ORC_E_NOMEM (-3)

/* ------------------------------------------------------------------ */
/* Definition 1: a dominates b (rows of length d).                      */
/* ------------------------------------------------------------------ */
static int dominates(const double *a, const double *b, int d)
{
    int strictly_better = 0;
    for (int k = 0; k < d; ++k) {
        if (a[k] > b[k]) return 0;
        if (a[k] < b[k]) strictly_better = 1;
    }
    return strictly_better;
}

int orc_dominates_f32(const float *a, const float *b, int d)
{
    double x[64], y[64];
    if (d < 1 || d > 64) return ORC_E_INVAL;
    for (int k = 0; k < d; ++k) { x[k] = a[k]; y[k] = b[k]; }
    return dominates(x, y, d);
}

/* ------------------------------------------------------------------ */
/* Widening to binary64 (exact for both input types).                   */
/* ------------------------------------------------------------------ */
static double *widen_f32(const float *p, int64_t n, int d, int *has_nan)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)d);
    if (!w) return NULL;
    *has_nan = 0;
    for (int64_t i = 0; i < n * d; ++i) {
        if (isnan(p[i])) *has_nan = 1;
        w[i] = (double)p[i];
    }
    return w;
}

static double *widen_u16(const uint16_t *p, int64_t n, int d)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)d);
    if (!w) return NULL;
    for (int64_t i = 0; i < n * d; ++i) w[i] = (double)p[i];
    return w;
}

/* ------------------------------------------------------------------ */
/* A minimal parallel-for over [0, count) with host threads.            */
/* ------------------------------------------------------------------ */
typedef void (*range_fn)(void *ctx, int64_t lo, int64_t hi);

typedef struct {
    range_fn fn;
    void *ctx;
    int64_t count;
    int64_t chunk;
    int64_t next;
    pthread_mutex_t lock;
} pfor_t;

static void *pfor_worker(void *arg)
{
    pfor_t *pf = (pfor_t *)arg;
    for (;;) {
        pthread_mutex_lock(&pf->lock);
        int64_t lo = pf->next;
        pf->next += pf->chunk;
        pthread_mutex_unlock(&pf->lock);
        if (lo >= pf->count) break;
        int64_t hi = lo + pf->chunk < pf->count ? lo + pf->chunk : pf->count;
        pf->fn(pf->ctx, lo, hi);
    }
    return NULL;
}

static void parallel_for(int nthreads, int64_t count, int64_t chunk, range_fn fn, void *ctx)
{
    if (count <= 0) return;
    if (nthreads <= 1 || count <= chunk) {
        fn(ctx, 0, count);
        return;
    }
    pfor_t pf = {fn, ctx, count, chunk, 0, PTHREAD_MUTEX_INITIALIZER};
    pthread_t th[256];
    if (nthreads > 256) nthreads = 256;
    int started = 0;
    for (int t = 0; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, pfor_worker, &pf) == 0) ++started;
    if (started == 0) pfor_worker(&pf);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&pf.lock);
}

/* ------------------------------------------------------------------ */
/* O1: brute force.  flag[i] = 1 iff no j dominates i.                  */
/* ------------------------------------------------------------------ */
typedef struct {
    const double *w;
    int64_t n;
    int d;
    uint8_t *flag;
} brute_ctx;

static void brute_range(void *vctx, int64_t lo, int64_t hi)
{
    brute_ctx *c = (brute_ctx *)vctx;
    for (int64_t i = lo; i < hi; ++i) {
        const double *pi = c->w + (size_t)i * c->d;
        uint8_t sky = 1;
        for (int64_t j = 0; j < c->n; ++j) {
            if (j != i && dominates(c->w + (size_t)j * c->d, pi, c->d)) { sky = 0; break; }
        }
        c->flag[i] = sky;
    }
}

static int64_t flags_to_indices(const uint8_t *flag, int64_t n, int32_t *out)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (flag[i]) out[m++] = (int32_t)i;
    return m;
}

static int64_t brute_core(const double *w, int64_t n, int d, int32_t *out, int nthreads)
{
    uint8_t *flag = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    if (!flag) return ORC_E_NOMEM;
    brute_ctx c = {w, n, d, flag};
    parallel_for(nthreads, n, 64, brute_range, &c);
    int64_t m = flags_to_indices(flag, n, out);
    free(flag);
    return m;
}

/* ------------------------------------------------------------------ */
/* O2: sort-first skyline with an exact sort key.                      */
/*                                                                    */
/* Key(i) = (s_i, p_i[0], ..., p_i[d-1], i) where s_i is the binary64 sum */
/* of the coordinates taken in dimension order.  Rounded addition is    */
/* monotone, so q dominating p gives s_q <= s_p; when the sums tie, the */
/* first differing coordinate has q < p.  Hence every dominator of p    */
/* sorts strictly before p, and a window of accepted points suffices.   */
/* ------------------------------------------------------------------ */
typedef struct {
    const double *w;
    const double *sum;
    int d;
} sort_ctx_t;

static sort_ctx_t g_sort_ctx; /* qsort has no context argument */
static pthread_mutex_t g_sort_lock = PTHREAD_MUTEX_INITIALIZER;

static int key_cmp(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    const sort_ctx_t *c = &g_sort_ctx;
    if (c->sum[i] < c->sum[j]) return -1;
    if (c->sum[i] > c->sum[j]) return 1;
    for (int k = 0; k < c->d; ++k) {
        double x = c->w[(size_t)i * c->d + k], y = c->w[(size_t)j * c->d + k];
        if (x < y) return -1;
        if (x > y) return 1;
    }
    return (i > j) - (i < j);
}

typedef struct {
    const double *w;
    int d;
    const int64_t *order;   /* sorted point ids */
    const int64_t *window;  /* accepted point ids, in sorted order */
    int64_t wlen;
    int64_t blk_lo;         /* block = order[blk_lo .. blk_hi) */
    uint8_t *alive;         /* per block slot */
} sfs_ctx;

/* Phase 1: each block point against the window of earlier accepted points. */
static void sfs_window_range(void *vctx, int64_t lo, int64_t hi)
{
    sfs_ctx *c = (sfs_ctx *)vctx;
    for (int64_t s = lo; s < hi; ++s) {
        const double *p = c->w + (size_t)c->order[c->blk_lo + s] * c->d;
        uint8_t ok = 1;
        for (int64_t t = 0; t < c->wlen; ++t) {
            if (dominates(c->w + (size_t)c->window[t] * c->d, p, c->d)) { ok = 0; break; }
        }
        c->alive[s] = ok;
    }
}

/* Phase 2: each phase-1 survivor against earlier phase-1 survivors of the
 * same block.  A block point rejected in phase 1 has a window dominator that
 * would also have rejected every point it dominates, so it can be ignored. */
typedef struct {
    sfs_ctx *base;
    const uint8_t *alive1;
    uint8_t *alive2;
} sfs2_ctx;

static void sfs_block_range(void *vctx, int64_t lo, int64_t hi)
{
    sfs2_ctx *c2 = (sfs2_ctx *)vctx;
    sfs_ctx *c = c2->base;
    for (int64_t s = lo; s < hi; ++s) {
        if (!c2->alive1[s]) { c2->alive2[s] = 0; continue; }
        const double *p = c->w + (size_t)c->order[c->blk_lo + s] * c->d;
        uint8_t ok = 1;
        for (int64_t t = 0; t < s; ++t) {
            if (!c2->alive1[t]) continue;
            if (dominates(c->w + (size_t)c->order[c->blk_lo + t] * c->d, p, c->d)) { ok = 0; break; }
        }
        c2->alive2[s] = ok;
    }
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int64_t sfs_core(const double *w, int64_t n, int d, int32_t *out, int nthreads)
{
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double *sum = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t *window = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    const int64_t B = 4096;
    uint8_t *alive1 = (uint8_t *)malloc((size_t)B), *alive2 = (uint8_t *)malloc((size_t)B);
    if (!order || !sum || !window || !alive1 || !alive2) {
        free(order); free(sum); free(window); free(alive1); free(alive2);
        return ORC_E_NOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        /* Infinities are clamped to +-2^129 (beyond every finite binary32)
         * before summing, so that a point holding both +inf and -inf gets a
         * finite sum instead of NaN.  The clamp is non-decreasing, so the sum
         * stays a monotone function of the coordinates and the key remains a
         * linear extension of the dominance order; ties still fall back to
         * the unclamped coordinates. */
        double s = 0.0;
        for (int k = 0; k < d; ++k) {
            double v = w[(size_t)i * d + k];
            if (v > 0x1p129) v = 0x1p129;
            if (v < -0x1p129) v = -0x1p129;
            s += v;
        }
        sum[i] = s;
        order[i] = i;
    }
    pthread_mutex_lock(&g_sort_lock);
    g_sort_ctx.w = w; g_sort_ctx.sum = sum; g_sort_ctx.d = d;
    qsort(order, (size_t)n, sizeof(int64_t), key_cmp);
    pthread_mutex_unlock(&g_sort_lock);

    int64_t wlen = 0;
    for (int64_t lo = 0; lo < n; lo += B) {
        int64_t len = (n - lo) < B ? (n - lo) : B;
        sfs_ctx c = {w, d, order, window, wlen, lo, alive1};
        parallel_for(nthreads, len, 16, sfs_window_range, &c);
        sfs2_ctx c2 = {&c, alive1, alive2};
        parallel_for(nthreads, len, 16, sfs_block_range, &c2);
        for (int64_t s = 0; s < len; ++s)
            if (alive2[s]) window[wlen++] = order[lo + s];
    }
    for (int64_t t = 0; t < wlen; ++t) out[t] = (int32_t)window[t];
    qsort(out, (size_t)wlen, sizeof(int32_t), cmp_i32);
    free(order); free(sum); free(window); free(alive1); free(alive2);
    return wlen;
}

/* ------------------------------------------------------------------ */
/* Per-index check: is point i a skyline point of the whole set?        */
/* ------------------------------------------------------------------ */
typedef struct {
    const double *w;
    int64_t n;
    int d;
    const int64_t *idx;
    uint8_t *res;
} check_ctx;

static void check_range(void *vctx, int64_t lo, int64_t hi)
{
    check_ctx *c = (check_ctx *)vctx;
    for (int64_t s = lo; s < hi; ++s) {
        int64_t i = c->idx[s];
        const double *pi = c->w + (size_t)i * c->d;
        uint8_t sky = 1;
        for (int64_t j = 0; j < c->n; ++j) {
            if (j != i && dominates(c->w + (size_t)j * c->d, pi, c->d)) { sky = 0; break; }
        }
        c->res[s] = sky;
    }
}

/* ------------------------------------------------------------------ */
/* Exported entry points.  Points are row-major [n][d] on the host.     */
/* Return: number of skyline indices written to out (ascending), or a  */
/* negative error code.                                                 */
/* ------------------------------------------------------------------ */
static int args_ok(const void *p, int64_t n, int d, const void *out)
{
    if (n < 0 || d < 1 || d > 64) return 0;
    if (n > 0 && (!p || !out)) return 0;
    if (n >= ((int64_t)1 << 31)) return 0;
    return 1;
}

int64_t orc_skyline_brute_f32(const float *pts, int64_t n, int d, int32_t *out, int nthreads)
{
    if (!args_ok(pts, n, d, out)) return ORC_E_INVAL;
    int nan = 0;
    double *w = widen_f32(pts, n, d, &nan);
    if (!w) return ORC_E_NOMEM;
    if (nan) { free(w); return ORC_E_NAN; }
    int64_t m = brute_core(w, n, d, out, nthreads);
    free(w);
    return m;
}

int64_t orc_skyline_sfs_f32(const float *pts, int64_t n, int d, int32_t *out, int nthreads)
{
    if (!args_ok(pts, n, d, out)) return ORC_E_INVAL;
    int nan = 0;
    double *w = widen_f32(pts, n, d, &nan);
    if (!w) return ORC_E_NOMEM;
    if (nan) { free(w); return ORC_E_NAN; }
    int64_t m = sfs_core(w, n, d, out, nthreads);
    free(w);
    return m;
}

int64_t orc_skyline_brute_u16(const uint16_t *pts, int64_t n, int d, int32_t *out, int nthreads)
{
    if (!args_ok(pts, n, d, out)) return ORC_E_INVAL;
    double *w = widen_u16(pts, n, d);
    if (!w) return ORC_E_NOMEM;
    int64_t m = brute_core(w, n, d, out, nthreads);
    free(w);
    return m;
}

int64_t orc_skyline_sfs_u16(const uint16_t *pts, int64_t n, int d, int32_t *out, int nthreads)
{
    if (!args_ok(pts, n, d, out)) return ORC_E_INVAL;
    double *w = widen_u16(pts, n, d);
    if (!w) return ORC_E_NOMEM;
    int64_t m = sfs_core(w, n, d, out, nthreads);
    free(w);
    return m;
}

/* res[s] = 1 iff pts[idx[s]] is a skyline point of all n points. */
int orc_is_skyline_f32(const float *pts, int64_t n, int d, const int64_t *idx, int64_t m,
                       uint8_t *res, int nthreads)
{
    if (!args_ok(pts, n, d, res) || m < 0 || (m > 0 && !idx)) return ORC_E_INVAL;
    for (int64_t s = 0; s < m; ++s)
        if (idx[s] < 0 || idx[s] >= n) return ORC_E_INVAL;
    int nan = 0;
    double *w = widen_f32(pts, n, d, &nan);
    if (!w) return ORC_E_NOMEM;
    if (nan) { free(w); return ORC_E_NAN; }
    check_ctx c = {w, n, d, idx, res};
    parallel_for(nthreads, m, 1, check_range, &c);
    free(w);
    return ORC_OK;
}

int orc_is_skyline_u16(const uint16_t *pts, int64_t n, int d, const int64_t *idx, int64_t m,
                       uint8_t *res, int nthreads)
{
    if (!args_ok(pts, n, d, res) || m < 0 || (m > 0 && !idx)) return ORC_E_INVAL;
    for (int64_t s = 0; s < m; ++s)
        if (idx[s] < 0 || idx[s] >= n) return ORC_E_INVAL;
    double *w = widen_u16(pts, n, d);
    if (!w) return ORC_E_NOMEM;
    check_ctx c = {w, n, d, idx, res};
    parallel_for(nthreads, m, 1, check_range, &c);
    free(w);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O3: orthant-emptiness test on a k-d tree.                           */
/*                                                                    */
/* By Definitions 1-2, p is a skyline point iff no point q satisfies   */
/* q <= p in every dimension with q != p as a vector (q <= p and       */
/* q != p is exactly "q dominates p").  So the oracle asks, for each   */
/* p, whether the closed lower orthant {q : q <= p} holds a point that */
/* differs from p.  A k-d tree over all points answers this with       */
/* bounding boxes of the actual points in each node:                  */
/*   - a node whose box minimum exceeds p in some dimension holds no   */
/*     point of the orthant and is skipped;                           */
/*   - a node whose box maximum is <= p everywhere lies inside the     */
/*     orthant; it holds a point != p iff its box minimum is below p   */
/*     in some dimension (otherwise min = max = p: only copies of p);  */
/*   - a leaf is scanned point by point with Definition 1.             */
/* The search stops at the first dominator.  Only comparisons are used */
/* (binary64 widened inputs), so the result is exact.                  */
/* ------------------------------------------------------------------ */
#define KD_LEAF 24

typedef struct {
    int64_t lo, hi;       /* points tp[lo .. hi) in tree order */
    int32_t left, right;  /* child nodes, -1 for a leaf */
} kd_node;

typedef struct {
    int d;
    const double *w;      /* original points, row-major */
    double *tp;           /* points copied in tree order */
    int64_t *perm;        /* tree position -> original index */
    kd_node *nodes;
    double *bmin, *bmax;  /* per node, d values each */
    int64_t nnodes, cap;
} kd_tree;

static double kd_val(const kd_tree *t, int64_t pos, int k) { return t->w[(size_t)t->perm[pos] * t->d + k]; }

static void kd_swap(int64_t *a, int64_t i, int64_t j) { int64_t x = a[i]; a[i] = a[j]; a[j] = x; }

/* Rearrange perm[lo..hi) so that position m holds the element of rank m - lo
 * in dimension k, smaller-or-equal values before it and larger-or-equal after
 * (quickselect with a three-way partition, so heavy ties stay linear). */
static void kd_select(kd_tree *t, int64_t lo, int64_t hi, int64_t m, int k)
{
    int64_t *a = t->perm;
    while (hi - lo > 1) {
        const double x0 = kd_val(t, lo, k), x1 = kd_val(t, lo + (hi - lo) / 2, k), x2 = kd_val(t, hi - 1, k);
        double pv = x0 < x1 ? (x1 < x2 ? x1 : (x0 < x2 ? x2 : x0)) : (x0 < x2 ? x0 : (x1 < x2 ? x2 : x1));
        int64_t lt = lo, i = lo, gt = hi;  /* [lo,lt) < pv, [lt,i) == pv, [gt,hi) > pv */
        while (i < gt) {
            const double v = kd_val(t, i, k);
            if (v < pv) kd_swap(a, lt++, i++);
            else if (v > pv) kd_swap(a, i, --gt);
            else ++i;
        }
        if (m < lt) hi = lt;
        else if (m >= gt) lo = gt;
        else return;
    }
}

static int32_t kd_new_node(kd_tree *t, int64_t lo, int64_t hi)
{
    if (t->nnodes == t->cap) return -1;
    const int32_t id = (int32_t)t->nnodes++;
    t->nodes[id].lo = lo;
    t->nodes[id].hi = hi;
    t->nodes[id].left = t->nodes[id].right = -1;
    double *mn = t->bmin + (size_t)id * t->d, *mx = t->bmax + (size_t)id * t->d;
    for (int k = 0; k < t->d; ++k) { mn[k] = INFINITY; mx[k] = -INFINITY; }
    for (int64_t i = lo; i < hi; ++i)
        for (int k = 0; k < t->d; ++k) {
            const double v = kd_val(t, i, k);
            if (v < mn[k]) mn[k] = v;
            if (v > mx[k]) mx[k] = v;
        }
    return id;
}

/* Split on the dimension of widest extent, at the median. */
static int kd_build(kd_tree *t, int32_t id)
{
    const int64_t lo = t->nodes[id].lo, hi = t->nodes[id].hi;
    if (hi - lo <= KD_LEAF) return ORC_OK;
    const double *mn = t->bmin + (size_t)id * t->d, *mx = t->bmax + (size_t)id * t->d;
    int k = 0;
    double best = 0.0;
    for (int j = 0; j < t->d; ++j) {
        const double ext = mx[j] > mn[j] ? mx[j] - mn[j] : 0.0;  /* +inf for infinite ranges */
        if (ext > best) { best = ext; k = j; }
    }
    if (best == 0.0) return ORC_OK;  /* all points of the node are copies: keep a leaf */
    const int64_t mid = lo + (hi - lo) / 2;
    kd_select(t, lo, hi, mid, k);
    const int32_t l = kd_new_node(t, lo, mid), r = kd_new_node(t, mid, hi);
    if (l < 0 || r < 0) return ORC_E_NOMEM;
    t->nodes[id].left = l;
    t->nodes[id].right = r;
    int rc = kd_build(t, l);
    if (rc == ORC_OK) rc = kd_build(t, r);
    return rc;
}

typedef struct {
    const kd_tree *t;
    uint8_t *flag;   /* by original index: 1 = skyline */
} kd_query_ctx;

static int kd_has_dominator(const kd_tree *t, const double *p)
{
    const int d = t->d;
    int32_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const int32_t id = stack[--sp];
        const double *mn = t->bmin + (size_t)id * d, *mx = t->bmax + (size_t)id * d;
        int outside = 0, inside = 1, below = 0;
        for (int k = 0; k < d; ++k) {
            if (mn[k] > p[k]) { outside = 1; break; }
            if (mx[k] > p[k]) inside = 0;
            if (mn[k] < p[k]) below = 1;
        }
        if (outside) continue;
        if (inside) {
            if (below) return 1;  /* some point of the node is <= p and != p */
            continue;             /* the node holds only copies of p */
        }
        const kd_node *nd = &t->nodes[id];
        if (nd->left < 0) {
            for (int64_t i = nd->lo; i < nd->hi; ++i)
                if (dominates(t->tp + (size_t)i * d, p, d)) return 1;
            continue;
        }
        /* the left child holds the smaller values of the split dimension:
         * search it first, where dominators are more likely */
        if (sp + 2 > 256) return -1;
        stack[sp++] = nd->right;
        stack[sp++] = nd->left;
    }
    return 0;
}

static int g_kd_overflow = 0;

static void kd_query_range(void *vctx, int64_t lo, int64_t hi)
{
    kd_query_ctx *c = (kd_query_ctx *)vctx;
    const kd_tree *t = c->t;
    for (int64_t i = lo; i < hi; ++i) {
        const int r = kd_has_dominator(t, t->w + (size_t)i * t->d);
        if (r < 0) __atomic_store_n(&g_kd_overflow, 1, __ATOMIC_RELAXED);
        c->flag[i] = r == 0;
    }
}

static int64_t kdtree_core(const double *w, int64_t n, int d, int32_t *out, int nthreads)
{
    if (n == 0) return 0;
    kd_tree t;
    memset(&t, 0, sizeof(t));
    t.d = d;
    t.w = w;
    t.cap = n / 4 + 16;  /* median splits of nodes above KD_LEAF: fewer than n/6 + 2 nodes */
    t.perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    t.tp = (double *)malloc(sizeof(double) * (size_t)n * (size_t)d);
    t.nodes = (kd_node *)malloc(sizeof(kd_node) * (size_t)t.cap);
    t.bmin = (double *)malloc(sizeof(double) * (size_t)t.cap * (size_t)d);
    t.bmax = (double *)malloc(sizeof(double) * (size_t)t.cap * (size_t)d);
    uint8_t *flag = (uint8_t *)malloc((size_t)n);
    int64_t m = ORC_E_NOMEM;
    if (!t.perm || !t.tp || !t.nodes || !t.bmin || !t.bmax || !flag) goto done;
    for (int64_t i = 0; i < n; ++i) t.perm[i] = i;
    if (kd_new_node(&t, 0, n) != 0 || kd_build(&t, 0) != ORC_OK) goto done;
    for (int64_t i = 0; i < n; ++i)
        memcpy(t.tp + (size_t)i * d, w + (size_t)t.perm[i] * d, sizeof(double) * (size_t)d);
    g_kd_overflow = 0;
    kd_query_ctx c = {&t, flag};
    parallel_for(nthreads, n, 256, kd_query_range, &c);
    if (g_kd_overflow) { m = ORC_E_INVAL; goto done; }
    m = flags_to_indices(flag, n, out);
done:
    free(t.perm); free(t.tp); free(t.nodes); free(t.bmin); free(t.bmax); free(flag);
    return m;
}

int64_t orc_skyline_kdtree_f32(const float *pts, int64_t n, int d, int32_t *out, int nthreads)
{
    if (!args_ok(pts, n, d, out)) return ORC_E_INVAL;
    int nan = 0;
    double *w = widen_f32(pts, n, d, &nan);
    if (!w) return ORC_E_NOMEM;
    if (nan) { free(w); return ORC_E_NAN; }
    int64_t m = kdtree_core(w, n, d, out, nthreads);
    free(w);
    return m;
}

int64_t orc_skyline_kdtree_u16(const uint16_t *pts, int64_t n, int d, int32_t *out, int nthreads)
{
    if (!args_ok(pts, n, d, out)) return ORC_E_INVAL;
    double *w = widen_u16(pts, n, d);
    if (!w) return ORC_E_NOMEM;
    int64_t m = kdtree_core(w, n, d, out, nthreads);
    free(w);
    return m;
}

/* ------------------------------------------------------------------ */
/* Equation 1, generalised to g cells per dimension: the column of a    */
/* point in dimension k is floor(p[k] * g), computed as a binary32      */
/* product rounded to nearest and then floored, clamped to [0, g-1] so */
/* that values outside [0, 1) still land in a cell (any non-decreasing  */
/* map keeps cell domination sound).  uint16 data with values below     */
/* 2^bits use the exact integer form floor(v * g / 2^bits).             */
/* coords is row-major [n][d].                                          */
/* ------------------------------------------------------------------ */
int orc_cell_coords_f32(const float *pts, int64_t n, int d, int g, int32_t *coords)
{
    if (!args_ok(pts, n, d, coords) || g < 1) return ORC_E_INVAL;
    const float gf = (float)g;
    for (int64_t i = 0; i < n * d; ++i) {
        float x = pts[i];
        if (isnan(x)) return ORC_E_NAN;
        volatile float prod = x * gf; /* one binary32 multiply, round to nearest */
        float f = floorf(prod);
        int32_t c;
        if (!(f >= 0.0f)) c = 0;
        else if (f >= gf) c = g - 1;
        else c = (int32_t)f;
        coords[i] = c;
    }
    return ORC_OK;
}

int orc_cell_coords_u16(const uint16_t *pts, int64_t n, int d, int g, int bits, int32_t *coords)
{
    if (!args_ok(pts, n, d, coords) || g < 1 || bits < 1 || bits > 16) return ORC_E_INVAL;
    for (int64_t i = 0; i < n * d; ++i) {
        int64_t c = ((int64_t)pts[i] * g) >> bits;
        coords[i] = (int32_t)(c > g - 1 ? g - 1 : c);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Definition 3, cell domination, brute force over the non-empty cells. */
/* cells: row-major [m][d] coordinates of the distinct non-empty cells. */
/* dominated[a] = 1 iff some other listed cell b has b[k] < a[k] in     */
/* every dimension (a dominated cell cannot hold a skyline point).      */
/* ------------------------------------------------------------------ */
int orc_cells_dominated(const int32_t *cells, int64_t m, int d, uint8_t *dominated)
{
    if (m < 0 || d < 1 || (m > 0 && (!cells || !dominated))) return ORC_E_INVAL;
    for (int64_t a = 0; a < m; ++a) {
        uint8_t dom = 0;
        for (int64_t b = 0; b < m && !dom; ++b) {
            int all_less = 1;
            for (int k = 0; k < d; ++k)
                if (!(cells[b * d + k] < cells[a * d + k])) { all_less = 0; break; }
            dom = (uint8_t)all_less;
        }
        dominated[a] = dom;
    }
    return ORC_OK;
}
