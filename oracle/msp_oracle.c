/*
 * msp_oracle.c -- plain, single-threaded reference solver (test
 * infrastructure only; see msp_oracle.h).  Written for clarity, not speed:
 * every routine follows the definition or the algorithm it names, with
 * library qsort/bsearch-style steps and nothing fused or reordered.
 *
 * Integer only.  Counts of 1-D hits use unsigned __int128.
 */
#include "msp_oracle.h"

#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define ORC_EINVAL   (-1)
#define ORC_ERANGE   (-2)
#define ORC_EKEY     (-3)
#define ORC_ESIZE    (-4)
#define ORC_ENOMEM   (-5)

#define ORC_MAXN     128   /* variables per instance */

/* ------------------------------------------------------------------------ */
/* Validation and the surrogate key (Section 1, eq. surrogate).              */
/* ------------------------------------------------------------------------ */

static int validate(const int32_t *A, const int32_t *d, int m, int n, int key_rows)
{
    if (!A || !d || m < 1 || n < 1 || n > ORC_MAXN || key_rows < 1 || key_rows > m)
        return ORC_EINVAL;
    for (int i = 0; i < m; ++i) {
        int64_t s = 0;
        if (d[i] < 0) return ORC_EINVAL;
        for (int j = 0; j < n; ++j) {
            if (A[(size_t)i * n + j] < 0) return ORC_EINVAL;
            s += A[(size_t)i * n + j];
        }
        if (s > 65534) return ORC_ERANGE;
    }
    return 0;
}

/* The key's place values, K_d and the column weights w_j.  With wide != NULL
 * a key past int64 is allowed: every value is then kept modulo 2^64 (the
 * bit pattern in an int64), which is exact for residues modulo 2^k, and
 * *wide = 1; equality of two such keys is decided on the key rows' sums
 * instead (see orc_mitm_residues).  wide == NULL: overflow is ORC_EKEY. */
static int key_setup_impl(const int32_t *A, const int32_t *d, int m, int n, int key_rows,
                          int key_base, int64_t *base, int64_t *kd, int64_t *w, int *infeasible,
                          int *wide)
{
    int rc = validate(A, d, m, n, key_rows);
    if (rc) return rc;
    if (key_base != 0 && key_base != 1) return ORC_EINVAL;
    int32_t amax = 0;
    for (size_t k = 0; k < (size_t)m * n; ++k)
        if (A[k] > amax) amax = A[k];
    /* D > a_ij for every coefficient; D = 100 for the paper's [0,99] family. */
    int64_t D = amax + 1 > 100 ? (int64_t)amax + 1 : 100;
    int64_t B = (int64_t)n * D;
    /* Digit i (the row sum a_i.x, 0..rowsum_i) has radix B (key_base 0) or
     * rowsum_i + 1 (key_base 1, mixed radix); radix[i] > every digit value
     * is what makes the key exact.  Place values: the product of the radices
     * of the rows below.  The largest key, sum_i place_i rowsum_i, must
     * stay below 2^63. */
    int64_t rowsum[ORC_MAXN];
    uint64_t place[ORC_MAXN];                  /* modulo 2^64 */
    unsigned __int128 kmax = 0, p = 1;
    int over = 0;                               /* the key does not fit int64 */
    *infeasible = 0;
    for (int i = 0; i < key_rows; ++i) {
        rowsum[i] = 0;
        for (int j = 0; j < n; ++j) rowsum[i] += A[(size_t)i * n + j];
        if (d[i] > rowsum[i]) *infeasible = 1;     /* row i can never hold */
        place[i] = (uint64_t)p;
        if (!over) {
            kmax += p * (unsigned __int128)rowsum[i];
            if (kmax >= ((unsigned __int128)1 << 63)) over = 1;
        }
        if (!over) {
            p *= (unsigned __int128)(key_base ? rowsum[i] + 1 : B);
            if (i + 1 < key_rows && p >= ((unsigned __int128)1 << 63)) over = 1;
        } else {
            p = (uint64_t)p * (uint64_t)(key_base ? rowsum[i] + 1 : B);
        }
    }
    if (over && !wide) return ORC_EKEY;
    if (wide) *wide = over;
    uint64_t k = 0;
    for (int i = 0; i < key_rows; ++i)
        if (!*infeasible) k += place[i] * (uint64_t)d[i];
    for (int j = 0; j < n; ++j) {
        uint64_t s = 0;
        for (int i = 0; i < key_rows; ++i) s += place[i] * (uint64_t)A[(size_t)i * n + j];
        w[j] = (int64_t)s;
    }
    *base = key_base ? rowsum[0] + 1 : B;
    *kd = *infeasible ? -1 : (int64_t)k;
    return 0;
}

int orc_key_setup(const int32_t *A, const int32_t *d, int m, int n, int key_rows,
                  int key_base, int64_t *base, int64_t *kd, int64_t *w, int *infeasible)
{
    return key_setup_impl(A, d, m, n, key_rows, key_base, base, kd, w, infeasible, NULL);
}

int orc_key_setup_wide(const int32_t *A, const int32_t *d, int m, int n, int key_rows,
                       int key_base, int64_t *base, int64_t *kd, int64_t *w, int *infeasible,
                       int *wide)
{
    return key_setup_impl(A, d, m, n, key_rows, key_base, base, kd, w, infeasible, wide);
}

static int64_t pos_mod(int64_t x, int64_t mod)
{
    int64_t r = x % mod;
    return r < 0 ? r + mod : r;
}

/* Left half = columns [0, hL). */
static int half_left(int n) { return (n + 1) / 2; }

static void put_solution(uint8_t *sol, uint64_t capacity, orc_result *res, int n,
                         const int *cols, const uint64_t *masks, const int *widths)
{
    /* cols[q]: first column of quarter q; masks[q]: its subset; widths[q]. */
    if (sol && res->stored < capacity) {
        uint8_t *x = sol + res->stored * (uint64_t)n;
        memset(x, 0, (size_t)n);
        for (int q = 0; q < 4; ++q)
            for (int b = 0; b < widths[q]; ++b)
                x[cols[q] + b] = (uint8_t)((masks[q] >> b) & 1u);
        res->stored++;
    }
    res->nsol++;
}

static void add_h(orc_result *res, u128 v)
{
    u128 h = ((u128)res->h_hi << 64) | res->h_lo;
    h += v;
    res->h_lo = (uint64_t)h;
    res->h_hi = (uint64_t)(h >> 64);
}

/* ------------------------------------------------------------------------ */
/* O1: brute force -- the definition of S and H written out.                 */
/* ------------------------------------------------------------------------ */

int orc_brute(const int32_t *A, const int32_t *d, int m, int n, int key_rows, int key_base,
              int64_t slice_mod, int64_t slice_res, uint64_t *hr,
              uint8_t *sol, uint64_t capacity, orc_result *res)
{
    int64_t base, kd, w[ORC_MAXN];
    int infeasible, wide;
    int rc = key_setup_impl(A, d, m, n, key_rows, key_base, &base, &kd, w, &infeasible, &wide);
    if (rc) return rc;
    if (n > 30) return ORC_ESIZE;
    if (slice_mod < 0 || (slice_mod > 0 && (slice_res < 0 || slice_res >= slice_mod)))
        return ORC_EINVAL;
    /* A key past int64 is known modulo 2^64 only: slices by powers of two. */
    if (wide && slice_mod > 0 && (slice_mod & (slice_mod - 1))) return ORC_EINVAL;
    memset(res, 0, sizeof *res);
    for (int i = 0; i < m; ++i) hr[i] = 0;
    const int hL = half_left(n);
    int64_t sums[16] = {0};
    uint64_t kleft = 0;                   /* key of x restricted to the left half, mod 2^64 */
    uint8_t x[ORC_MAXN] = {0};
    const uint64_t total = (uint64_t)1 << n;
    /* Gray-code walk: step g flips bit ctz(g), so every x is visited once. */
    for (uint64_t g = 0; g < total; ++g) {
        if (g) {
            int j = __builtin_ctzll(g);
            int sgn = x[j] ? -1 : 1;
            x[j] ^= 1u;
            for (int i = 0; i < m; ++i) sums[i] += sgn * (int64_t)A[(size_t)i * n + j];
            if (j < hL) kleft += sgn > 0 ? (uint64_t)w[j] : -(uint64_t)w[j];
        }
        if (slice_mod > 0 && !wide && pos_mod((int64_t)kleft, slice_mod) != slice_res) continue;
        if (slice_mod > 0 && wide && (int64_t)(kleft & (uint64_t)(slice_mod - 1)) != slice_res)
            continue;
        int k = 0;
        while (k < m && sums[k] == d[k]) ++k;     /* rows 1..k hold */
        for (int i = 0; i < k; ++i) hr[i]++;
        if (k >= key_rows) add_h(res, 1);
        if (k == m) {
            if (sol && res->stored < capacity) {
                memcpy(sol + res->stored * (uint64_t)n, x, (size_t)n);
                res->stored++;
            }
            res->nsol++;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Counting dynamic programmes (exact reference counts for H).               */
/* ------------------------------------------------------------------------ */

int orc_dp_count_row(const int32_t *a, int n, int64_t target, uint64_t *lo, uint64_t *hi)
{
    if (!a || n < 0 || !lo || !hi) return ORC_EINVAL;
    int64_t total = 0;
    for (int j = 0; j < n; ++j) {
        if (a[j] < 0) return ORC_EINVAL;
        total += a[j];
    }
    *lo = *hi = 0;
    if (target < 0 || target > total) return 0;
    u128 *c = calloc((size_t)total + 1, sizeof *c);
    if (!c) return ORC_ENOMEM;
    c[0] = 1;
    int64_t reach = 0;
    for (int j = 0; j < n; ++j) {
        /* c[s] = #subsets of a[0..j) with sum s; include a[j] or not. */
        for (int64_t s = reach; s >= 0; --s)
            if (c[s]) c[s + a[j]] += c[s];
        reach += a[j];
    }
    *lo = (uint64_t)c[target];
    *hi = (uint64_t)(c[target] >> 64);
    free(c);
    return 0;
}

int orc_dp_count_2rows(const int32_t *a1, const int32_t *a2, int n,
                       int64_t t1, int64_t t2, uint64_t *count)
{
    if (!a1 || !a2 || n < 0 || n > 63 || !count) return ORC_EINVAL;
    int64_t s1 = 0, s2 = 0;
    for (int j = 0; j < n; ++j) {
        if (a1[j] < 0 || a2[j] < 0) return ORC_EINVAL;
        s1 += a1[j];
        s2 += a2[j];
    }
    *count = 0;
    if (t1 < 0 || t2 < 0 || t1 > s1 || t2 > s2) return 0;
    const int64_t W = s2 + 1;
    uint64_t *c = calloc((size_t)(s1 + 1) * (size_t)W, sizeof *c);
    if (!c) return ORC_ENOMEM;
    c[0] = 1;
    int64_t r1 = 0, r2 = 0;
    for (int j = 0; j < n; ++j) {
        for (int64_t u = r1; u >= 0; --u)
            for (int64_t v = r2; v >= 0; --v) {
                uint64_t cv = c[u * W + v];
                if (cv) c[(u + a1[j]) * W + (v + a2[j])] += cv;
            }
        r1 += a1[j];
        r2 += a2[j];
    }
    *count = c[t1 * W + t2];
    free(c);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Quarter lists shared by the two meet-in-the-middle oracles below.         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int col0, width;     /* columns [col0, col0+width) */
    uint64_t size;       /* 2^width subsets            */
    int64_t *key;        /* 1-D key weight of each subset (index = subset mask) */
    int32_t *vec;        /* size x m partial row sums */
} quarter;

static void quarter_free(quarter *q)
{
    free(q->key);
    free(q->vec);
    q->key = NULL;
    q->vec = NULL;
}

/* Power set of one quarter: weight and partial row-sum vector of every
 * subset, indexed by its bit mask (Algorithm 1 lists 2^A, 2^B, 2^C, 2^D). */
static int quarter_build(quarter *q, const int32_t *A, int m, int n, const int64_t *w,
                         int col0, int width)
{
    q->col0 = col0;
    q->width = width;
    q->size = (uint64_t)1 << width;
    q->key = malloc(q->size * sizeof *q->key);
    q->vec = malloc(q->size * (size_t)m * sizeof *q->vec);
    if (!q->key || !q->vec) {
        quarter_free(q);
        return ORC_ENOMEM;
    }
    for (uint64_t u = 0; u < q->size; ++u) {
        uint64_t k = 0;                          /* modulo 2^64 (exact below 2^63) */
        for (int i = 0; i < m; ++i) q->vec[u * m + i] = 0;
        for (int b = 0; b < width; ++b) {
            if (!((u >> b) & 1u)) continue;
            int j = col0 + b;
            k += (uint64_t)w[j];
            for (int i = 0; i < m; ++i) q->vec[u * m + i] += A[(size_t)i * n + j];
        }
        q->key[u] = (int64_t)k;
    }
    return 0;
}

static int quarters_build(quarter Q[4], const int32_t *A, int m, int n, const int64_t *w)
{
    const int hL = half_left(n);
    const int qa = (hL + 1) / 2, qb = hL / 2;
    const int qc = (n - hL + 1) / 2, qd = (n - hL) / 2;
    if (qa > 26 || qc > 26) return ORC_ESIZE;
    memset(Q, 0, 4 * sizeof *Q);
    int rc = quarter_build(&Q[0], A, m, n, w, 0, qa);
    if (!rc) rc = quarter_build(&Q[1], A, m, n, w, qa, qb);
    if (!rc) rc = quarter_build(&Q[2], A, m, n, w, hL, qc);
    if (!rc) rc = quarter_build(&Q[3], A, m, n, w, hL + qc, qd);
    if (rc)
        for (int i = 0; i < 4; ++i) quarter_free(&Q[i]);
    return rc;
}

/* A half-vector record used by the exact verify joins. */
typedef struct {
    int64_t key;
    uint64_t m1, m2;      /* subset masks of the two quarters of the half */
    int32_t v[16];        /* partial row sums (left) or d minus them (right) */
} half_rec;

static int g_cmp_m;       /* number of rows compared by cmp_vec (single-threaded) */

static int cmp_vec(const void *pa, const void *pb)
{
    const half_rec *a = pa, *b = pb;
    for (int i = 0; i < g_cmp_m; ++i)
        if (a->v[i] != b->v[i]) return a->v[i] < b->v[i] ? -1 : 1;
    return 0;
}

static int cmp_key(const void *pa, const void *pb)
{
    const half_rec *a = pa, *b = pb;
    return a->key < b->key ? -1 : (a->key > b->key ? 1 : 0);
}

/* Exact join of Algorithm 3: Q = left vectors (sorted), R = d - right
 * vectors; every right entry is searched in Q and each equal pair is a
 * solution.  Entries of R with a negative component can match nothing. */
static void join_vectors(half_rec *L, uint64_t nl, half_rec *R, uint64_t nr, int m,
                         const quarter Q[4], uint8_t *sol, uint64_t capacity,
                         orc_result *res, int n)
{
    g_cmp_m = m;
    qsort(L, nl, sizeof *L, cmp_vec);
    for (uint64_t k = 0; k < nr; ++k) {
        int neg = 0;
        for (int i = 0; i < m; ++i) neg |= R[k].v[i] < 0;
        if (neg) continue;
        /* lower bound of R[k] in L */
        uint64_t lo = 0, hi = nl;
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (cmp_vec(&L[mid], &R[k]) < 0) lo = mid + 1; else hi = mid;
        }
        for (uint64_t t = lo; t < nl && cmp_vec(&L[t], &R[k]) == 0; ++t) {
            int cols[4] = {Q[0].col0, Q[1].col0, Q[2].col0, Q[3].col0};
            int widths[4] = {Q[0].width, Q[1].width, Q[2].width, Q[3].width};
            uint64_t masks[4] = {L[t].m1, L[t].m2, R[k].m1, R[k].m2};
            put_solution(sol, capacity, res, n, cols, masks, widths);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* O3: Schroeppel-Shamir with heaps (Algorithm 1) + verify (Algs. 2-3).      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t key;
    uint64_t i;          /* position in the sorted list of 2^A (or 2^C) */
    uint64_t b;          /* subset of B (or D) this chain is bound to    */
} heap_ent;

typedef struct {
    heap_ent *e;
    uint64_t n;
    int max_heap;        /* 0: min-heap (H1), 1: max-heap (H2) */
} heap;

static int heap_before(const heap *h, const heap_ent *x, const heap_ent *y)
{
    return h->max_heap ? x->key > y->key : x->key < y->key;
}

static void heap_push(heap *h, heap_ent v)
{
    uint64_t k = h->n++;
    h->e[k] = v;
    while (k > 0) {
        uint64_t p = (k - 1) / 2;
        if (!heap_before(h, &h->e[k], &h->e[p])) break;
        heap_ent t = h->e[p]; h->e[p] = h->e[k]; h->e[k] = t;
        k = p;
    }
}

static heap_ent heap_pop(heap *h)
{
    heap_ent top = h->e[0];
    h->e[0] = h->e[--h->n];
    uint64_t k = 0;
    for (;;) {
        uint64_t l = 2 * k + 1, r = l + 1, best = k;
        if (l < h->n && heap_before(h, &h->e[l], &h->e[best])) best = l;
        if (r < h->n && heap_before(h, &h->e[r], &h->e[best])) best = r;
        if (best == k) break;
        heap_ent t = h->e[best]; h->e[best] = h->e[k]; h->e[k] = t;
        k = best;
    }
    return top;
}

/* 2^A ordered by weight: permutation of subset masks. */
static const quarter *g_sort_q;
static int g_sort_desc;
static int cmp_subset(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    int64_t ka = g_sort_q->key[a], kb = g_sort_q->key[b];
    if (ka != kb) return g_sort_desc ? (ka > kb ? -1 : 1) : (ka < kb ? -1 : 1);
    return a < b ? -1 : (a > b ? 1 : 0);
}

static uint64_t *sorted_subsets(const quarter *q, int descending)
{
    uint64_t *p = malloc(q->size * sizeof *p);
    if (!p) return NULL;
    for (uint64_t u = 0; u < q->size; ++u) p[u] = u;
    g_sort_q = q;
    g_sort_desc = descending;
    qsort(p, q->size, sizeof *p, cmp_subset);
    return p;
}

static int grow(half_rec **buf, uint64_t *cap, uint64_t need)
{
    if (need <= *cap) return 0;
    uint64_t nc = *cap ? *cap : 1024;
    while (nc < need) nc *= 2;
    half_rec *nb = realloc(*buf, nc * sizeof *nb);
    if (!nb) return ORC_ENOMEM;
    *buf = nb;
    *cap = nc;
    return 0;
}

int orc_ss_heap(const int32_t *A, const int32_t *d, int m, int n, int key_rows, int key_base,
                int64_t slice_mod, int64_t slice_res,
                uint8_t *sol, uint64_t capacity, orc_result *res)
{
    int64_t base, kd, w[ORC_MAXN];
    int infeasible;
    int rc = orc_key_setup(A, d, m, n, key_rows, key_base, &base, &kd, w, &infeasible);
    if (rc) return rc;
    if (m > 16) return ORC_ESIZE;
    if (slice_mod < 0 || (slice_mod > 0 && (slice_res < 0 || slice_res >= slice_mod)))
        return ORC_EINVAL;
    memset(res, 0, sizeof *res);
    if (infeasible) return 0;   /* some key row can never hold: H = 0, S = {} */

    quarter Q[4];
    rc = quarters_build(Q, A, m, n, w);
    if (rc) return rc;
    const quarter *qA = &Q[0], *qB = &Q[1], *qC = &Q[2], *qD = &Q[3];

    /* Line 3-4: 2^A ascending, 2^C descending by weight. */
    uint64_t *sa = sorted_subsets(qA, 0);
    uint64_t *sc = sorted_subsets(qC, 1);
    heap H1 = {malloc(qB->size * sizeof(heap_ent)), 0, 0};
    heap H2 = {malloc(qD->size * sizeof(heap_ent)), 0, 1};
    half_rec *G1 = NULL, *G2 = NULL;
    uint64_t c1 = 0, c2 = 0;
    if (!sa || !sc || !H1.e || !H2.e) { rc = ORC_ENOMEM; goto done; }

    /* Lines 5-6: one chain per subset of B (resp. D), starting at s^A_1 (s^C_1). */
    for (uint64_t b = 0; b < qB->size; ++b)
        heap_push(&H1, (heap_ent){qA->key[sa[0]] + qB->key[b], 0, b});
    for (uint64_t b = 0; b < qD->size; ++b)
        heap_push(&H2, (heap_ent){qC->key[sc[0]] + qD->key[b], 0, b});

    while (H1.n > 0 && H2.n > 0) {
        const int64_t alpha = H1.e[0].key, beta = H2.e[0].key;
        if (alpha + beta < kd) {
            /* Advance the smallest left sum.  An exhausted chain is dropped
             * (it can never reach the target), never matched. */
            heap_ent t = heap_pop(&H1);
            if (t.i + 1 < qA->size)
                heap_push(&H1, (heap_ent){qA->key[sa[t.i + 1]] + qB->key[t.b], t.i + 1, t.b});
        } else if (alpha + beta > kd) {
            heap_ent t = heap_pop(&H2);
            if (t.i + 1 < qC->size)
                heap_push(&H2, (heap_ent){qC->key[sc[t.i + 1]] + qD->key[t.b], t.i + 1, t.b});
        } else {
            /* alpha + beta = K_d.  Take EVERY heap entry with key alpha (beta),
             * not only the two tops, so that cross pairs between different
             * chains with equal sums are not lost.  For each popped chain the
             * run E_A of equal weight starting at position i is found by a
             * linear walk (line 15) and the chain is re-inserted past it. */
            uint64_t n1 = 0, n2 = 0;
            while (H1.n > 0 && H1.e[0].key == alpha) {
                heap_ent t = heap_pop(&H1);
                uint64_t e = t.i;
                while (e < qA->size && qA->key[sa[e]] == qA->key[sa[t.i]]) ++e;
                for (uint64_t k = t.i; k < e; ++k) {
                    if ((rc = grow(&G1, &c1, n1 + 1))) goto done;
                    half_rec *r = &G1[n1++];
                    r->key = alpha;
                    r->m1 = sa[k];
                    r->m2 = t.b;
                    for (int i = 0; i < m; ++i)
                        r->v[i] = qA->vec[sa[k] * m + i] + qB->vec[t.b * m + i];
                }
                if (e < qA->size)
                    heap_push(&H1, (heap_ent){qA->key[sa[e]] + qB->key[t.b], e, t.b});
            }
            while (H2.n > 0 && H2.e[0].key == beta) {
                heap_ent t = heap_pop(&H2);
                uint64_t e = t.i;
                while (e < qC->size && qC->key[sc[e]] == qC->key[sc[t.i]]) ++e;
                for (uint64_t k = t.i; k < e; ++k) {
                    if ((rc = grow(&G2, &c2, n2 + 1))) goto done;
                    half_rec *r = &G2[n2++];
                    r->key = beta;
                    r->m1 = sc[k];
                    r->m2 = t.b;
                    for (int i = 0; i < m; ++i)
                        r->v[i] = d[i] - (qC->vec[sc[k] * m + i] + qD->vec[t.b * m + i]);
                }
                if (e < qC->size)
                    heap_push(&H2, (heap_ent){qC->key[sc[e]] + qD->key[t.b], e, t.b});
            }
            /* The slice keeps only x whose left key is in the residue class;
             * all of G1 shares the left key alpha. */
            if (slice_mod > 0 && pos_mod(alpha, slice_mod) != slice_res) continue;
            add_h(res, (u128)n1 * n2);
            join_vectors(G1, n1, G2, n2, m, Q, sol, capacity, res, n);
        }
    }
    rc = 0;
done:
    free(sa);
    free(sc);
    free(H1.e);
    free(H2.e);
    free(G1);
    free(G2);
    for (int i = 0; i < 4; ++i) quarter_free(&Q[i]);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* O2: meet in the middle one residue class at a time.                        */
/* ------------------------------------------------------------------------ */

static int64_t g_res_mod;
static const quarter *g_res_q;
static int cmp_residue(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    int64_t ra = pos_mod(g_res_q->key[a], g_res_mod), rb = pos_mod(g_res_q->key[b], g_res_mod);
    if (ra != rb) return ra < rb ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Subsets of q sorted by key mod M, and the residue of each position. */
static uint64_t *sort_by_residue(const quarter *q, int64_t M, int64_t **res_out)
{
    uint64_t *p = malloc(q->size * sizeof *p);
    int64_t *r = malloc(q->size * sizeof *r);
    if (!p || !r) { free(p); free(r); return NULL; }
    for (uint64_t u = 0; u < q->size; ++u) p[u] = u;
    g_res_mod = M;
    g_res_q = q;
    qsort(p, q->size, sizeof *p, cmp_residue);
    for (uint64_t u = 0; u < q->size; ++u) r[u] = pos_mod(q->key[p[u]], M);
    *res_out = r;
    return p;
}

/* First position with residue >= t in a residue-sorted list. */
static uint64_t lower_res(const int64_t *r, uint64_t n, int64_t t)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (r[mid] < t) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Pairs (l, r) whose first k row entries agree (left sums against d minus
 * right sums): both lists sorted on those entries, equal runs multiplied. */
static u128 count_row_matches(half_rec *L, uint64_t nl, half_rec *R, uint64_t nr, int k)
{
    g_cmp_m = k;
    qsort(L, nl, sizeof *L, cmp_vec);
    qsort(R, nr, sizeof *R, cmp_vec);
    u128 h = 0;
    uint64_t i = 0, j = 0;
    while (i < nl && j < nr) {
        const int c = cmp_vec(&L[i], &R[j]);
        if (c < 0) { ++i; continue; }
        if (c > 0) { ++j; continue; }
        uint64_t i2 = i, j2 = j;
        while (i2 < nl && cmp_vec(&L[i2], &L[i]) == 0) ++i2;
        while (j2 < nr && cmp_vec(&R[j2], &R[j]) == 0) ++j2;
        h += (u128)(i2 - i) * (j2 - j);
        i = i2;
        j = j2;
    }
    return h;
}

int orc_mitm_residues(const int32_t *A, const int32_t *d, int m, int n,
                      int key_rows, int key_base, int log2_m, int64_t rho_lo, int64_t rho_hi,
                      int64_t slice_mod, int64_t slice_res,
                      uint8_t *sol, uint64_t capacity, orc_result *res)
{
    int64_t base, kd, w[ORC_MAXN];
    int infeasible, wide;
    int rc = key_setup_impl(A, d, m, n, key_rows, key_base, &base, &kd, w, &infeasible, &wide);
    if (rc) return rc;
    if (m > 16 || log2_m < 0 || log2_m > 40) return ORC_EINVAL;
    const int64_t M = (int64_t)1 << log2_m;
    if (rho_lo < 0 || rho_hi > M || rho_lo > rho_hi) return ORC_EINVAL;
    if (slice_mod < 0 || (slice_mod > 0 && (slice_res < 0 || slice_res >= slice_mod ||
                                            M % slice_mod != 0)))
        return ORC_EINVAL;
    memset(res, 0, sizeof *res);
    if (infeasible) return 0;

    quarter Q[4];
    rc = quarters_build(Q, A, m, n, w);
    if (rc) return rc;
    const quarter *qA = &Q[0], *qB = &Q[1], *qC = &Q[2], *qD = &Q[3];
    int64_t *rB = NULL, *rD = NULL;
    uint64_t *pB = sort_by_residue(qB, M, &rB);
    uint64_t *pD = sort_by_residue(qD, M, &rD);
    half_rec *L = NULL, *R = NULL;
    uint64_t cl = 0, cr = 0;
    if (!pB || !pD) { rc = ORC_ENOMEM; goto done; }

    for (int64_t rho = rho_lo; rho < rho_hi; ++rho) {
        if (slice_mod > 0 && rho % slice_mod != slice_res) continue;
        uint64_t nl = 0, nr = 0;
        /* L(rho): every (a, b) with k_a + k_b = rho (mod M). */
        for (uint64_t a = 0; a < qA->size; ++a) {
            int64_t t = (int64_t)(((uint64_t)rho - (uint64_t)qA->key[a]) & (uint64_t)(M - 1));
            for (uint64_t p = lower_res(rB, qB->size, t); p < qB->size && rB[p] == t; ++p) {
                uint64_t b = pB[p];
                if ((rc = grow(&L, &cl, nl + 1))) goto done;
                half_rec *h = &L[nl++];
                h->key = (int64_t)((uint64_t)qA->key[a] + (uint64_t)qB->key[b]);
                h->m1 = a;
                h->m2 = b;
                for (int i = 0; i < m; ++i) h->v[i] = qA->vec[a * m + i] + qB->vec[b * m + i];
            }
        }
        /* R(rho): every (c, e) with K_d - (k_c + k_e) = rho (mod M). */
        for (uint64_t c = 0; c < qC->size; ++c) {
            int64_t t = (int64_t)(((uint64_t)kd - (uint64_t)qC->key[c] - (uint64_t)rho) &
                                  (uint64_t)(M - 1));
            for (uint64_t p = lower_res(rD, qD->size, t); p < qD->size && rD[p] == t; ++p) {
                uint64_t e = pD[p];
                if ((rc = grow(&R, &cr, nr + 1))) goto done;
                half_rec *h = &R[nr++];
                h->key = (int64_t)((uint64_t)qC->key[c] + (uint64_t)qD->key[e]);
                h->m1 = c;
                h->m2 = e;
                for (int i = 0; i < m; ++i)
                    h->v[i] = d[i] - (qC->vec[c * m + i] + qD->vec[e * m + i]);
            }
        }
        /* H: pairs with k_L + k_R = K_d, counted run by run.  A key past
         * int64 (known modulo 2^64 only) is compared through what it encodes:
         * k_L + k_R = K_d exactly when rows 1..r hold (eq. surrogate), i.e.
         * when the left sums of the key rows equal d minus the right sums. */
        if (wide) {
            add_h(res, count_row_matches(L, nl, R, nr, key_rows));
        } else {
        qsort(L, nl, sizeof *L, cmp_key);
        qsort(R, nr, sizeof *R, cmp_key);
        uint64_t i = 0, j = nr;   /* R scanned from the top: k_R descending */
        while (i < nl && j > 0) {
            int64_t s = L[i].key + R[j - 1].key;
            if (s < kd) { ++i; continue; }
            if (s > kd) { --j; continue; }
            uint64_t i2 = i, j2 = j;
            while (i2 < nl && L[i2].key == L[i].key) ++i2;
            while (j2 > 0 && R[j2 - 1].key == R[j - 1].key) --j2;
            add_h(res, (u128)(i2 - i) * (j - j2));
            i = i2;
            j = j2;
        }
        }
        /* S: exact join of full row vectors. */
        join_vectors(L, nl, R, nr, m, Q, sol, capacity, res, n);
    }
    rc = 0;
done:
    free(pB); free(pD); free(rB); free(rD); free(L); free(R);
    for (int i = 0; i < 4; ++i) quarter_free(&Q[i]);
    return rc;
}
