/*
 * fsm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-thread CPU computation of frequent subgraph mining
 * results, written from the problem's definition.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this library; the
 * device path never links or calls it, and this file shares no code with it.
 *
 * What it computes (Section 2.2, the MNI-support definition and the FSM
 * problem statement; edge-induced semantics as used in Section 6.1):
 *   Given a simple undirected graph G with vertex labels, a threshold t and a
 *   maximum size s_max, output every connected vertex-labelled pattern P with
 *   2 <= |V_P| <= s_max whose MNI support
 *       sigma(P) = min over pattern vertices v of |{ f(v) : f in Emb(P,G) }|
 *   is >= t.  Emb(P,G) is the set of all injective, label-preserving maps
 *   f : V_P -> V such that every pattern edge maps onto a graph edge
 *   (non-edges of P are unconstrained: edge-induced subgraphs).
 *
 * How (no embedding enumeration):
 *   - Growth.  Size-1 "patterns" are single labels with at least t vertices.
 *     Size-(k+1) candidates are a frequent size-k pattern plus one new vertex
 *     of a frequent label joined to a non-empty subset of the old vertices.
 *     Every connected graph has a non-cut vertex, so every frequent size-(k+1)
 *     pattern arises this way from a frequent size-k pattern (support is
 *     anti-monotone, Section 2.2).  A candidate is also dropped when deleting
 *     one of its non-cut vertices leaves an infrequent pattern (same reason).
 *   - Canonical form.  The code of a pattern is the lexicographically smallest
 *     (label sequence, adjacency bit sequence) over all n! vertex orders; the
 *     adjacency bits list the pairs (i<j) in row-major upper-triangle order.
 *     Patterns with equal codes are isomorphic (Section 2.1).
 *   - Support.  For each automorphism orbit O (a representative c) and each
 *     graph vertex u with the right label, a backtracking search decides
 *     whether some embedding maps c to u.  Every vertex of one orbit has the
 *     same image set, so sigma is the minimum over orbits of those counts.
 *
 * Vertex-induced mode (oracle_mine_ex with induced = 1): an embedding must
 * also map every non-edge of P onto a non-edge of G, i.e. its image is an
 * induced subgraph (the vertex-induced reading of Section 2.1).  Deleting a
 * non-cut vertex of an induced embedding leaves an induced embedding of the
 * induced sub-pattern, so the growth and the drop-vertex check stay exact.
 *
 * Also: a count of connected edge-induced subgraphs with a given number of
 * vertices (every connected vertex set, enumerated once by Wernicke's ESU
 * scheme, times the number of connected spanning edge subsets of its induced
 * subgraph, counted by brute force).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OMAX 9                     /* largest pattern size handled */
#define OPAIRS (OMAX * (OMAX - 1) / 2)

/* ------------------------------------------------------------------ graph */

typedef struct {
    int64_t n;
    int64_t *off;   /* n+1 */
    int32_t *adj;   /* sorted by (label, id) within each row */
    int32_t *lab;   /* n */
} ograph;

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Simple graph from an edge list: loops dropped, duplicates merged, both
 * directions stored.  Returns 0, or -1 on bad input / allocation failure. */
static int graph_build(ograph *g, int64_t n, int64_t m, const int32_t *src,
                       const int32_t *dst, const int32_t *labels) {
    memset(g, 0, sizeof(*g));
    if (n <= 0 || m < 0) return -1;
    for (int64_t v = 0; v < n; v++)
        if (labels[v] < 0) return -1;
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
    if (!key) return -1;
    int64_t k = 0;
    for (int64_t e = 0; e < m; e++) {
        int64_t a = src[e], b = dst[e];
        if (a < 0 || a >= n || b < 0 || b >= n) { free(key); return -1; }
        if (a == b) continue;
        /* (row, neighbour) keys; rows are re-sorted by label further down */
        key[k++] = (a << 32) | (int64_t)(uint32_t)b;
        key[k++] = (b << 32) | (int64_t)(uint32_t)a;
    }
    qsort(key, (size_t)k, sizeof(int64_t), cmp_i64);
    int64_t u = 0;
    for (int64_t i = 0; i < k; i++)
        if (i == 0 || key[i] != key[i - 1]) key[u++] = key[i];
    g->n = n;
    g->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(u + 1));
    g->lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!g->off || !g->adj || !g->lab) { free(key); return -1; }
    memcpy(g->lab, labels, sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < u; i++) {
        g->off[(key[i] >> 32) + 1]++;
        g->adj[i] = (int32_t)(key[i] & 0xffffffff);
    }
    for (int64_t v = 0; v < n; v++) g->off[v + 1] += g->off[v];
    free(key);
    /* re-sort every row by (label, id) so a label's neighbours are contiguous */
    for (int64_t v = 0; v < n; v++) {
        int64_t b = g->off[v], e = g->off[v + 1];
        for (int64_t i = b + 1; i < e; i++) {          /* insertion sort */
            int32_t x = g->adj[i];
            int64_t j = i - 1;
            while (j >= b && (g->lab[g->adj[j]] > g->lab[x] ||
                              (g->lab[g->adj[j]] == g->lab[x] && g->adj[j] > x))) {
                g->adj[j + 1] = g->adj[j];
                j--;
            }
            g->adj[j + 1] = x;
        }
    }
    return 0;
}

static void graph_free(ograph *g) {
    free(g->off); free(g->adj); free(g->lab);
    memset(g, 0, sizeof(*g));
}

/* first index in row v whose (label, id) is >= (l, id) */
static int64_t row_lower(const ograph *g, int64_t v, int32_t l, int32_t id) {
    int64_t lo = g->off[v], hi = g->off[v + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        int32_t w = g->adj[mid];
        int32_t lw = g->lab[w];
        if (lw < l || (lw == l && w < id)) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int adjacent(const ograph *g, int32_t a, int32_t b) {
    int64_t i = row_lower(g, a, g->lab[b], b);
    return i < g->off[a + 1] && g->adj[i] == b;
}

/* ---------------------------------------------------------------- patterns */

typedef struct {
    int n;
    int32_t lab[OMAX];
    uint8_t e[OMAX][OMAX];   /* symmetric adjacency matrix */
} opat;

/* Position of the unordered pair (i<j) in row-major upper-triangle order. */
static int pair_pos(int i, int j, int n) {
    return i * n - i * (i + 1) / 2 + (j - i - 1);
}

/* Code of the pattern under vertex order `ord` (ord[new] = old vertex):
 * labels in new order, and the adjacency bit sequence packed with its first
 * pair as the most significant bit, so integer order = sequence order. */
static void code_under(const opat *p, const int *ord, int32_t *lab_out,
                       uint64_t *seq_out) {
    int n = p->n;
    uint64_t seq = 0;
    for (int i = 0; i < n; i++) lab_out[i] = p->lab[ord[i]];
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            seq = (seq << 1) | (uint64_t)(p->e[ord[i]][ord[j]] != 0);
    *seq_out = seq;
}

/* -1 / 0 / 1 comparison of two codes of the same size */
static int code_cmp(int n, const int32_t *la, uint64_t sa, const int32_t *lb,
                    uint64_t sb) {
    for (int i = 0; i < n; i++)
        if (la[i] != lb[i]) return la[i] < lb[i] ? -1 : 1;
    if (sa != sb) return sa < sb ? -1 : 1;
    return 0;
}

/* next lexicographic permutation of a[0..n-1]; 0 when wrapped */
static int next_perm(int *a, int n) {
    int i = n - 2;
    while (i >= 0 && a[i] >= a[i + 1]) i--;
    if (i < 0) return 0;
    int j = n - 1;
    while (a[j] <= a[i]) j--;
    int t = a[i]; a[i] = a[j]; a[j] = t;
    for (int l = i + 1, r = n - 1; l < r; l++, r--) { t = a[l]; a[l] = a[r]; a[r] = t; }
    return 1;
}

/* Canonical form: try every vertex order, keep the smallest code. */
static void canonicalize(const opat *p, opat *out) {
    int n = p->n, ord[OMAX], best[OMAX];
    int32_t bl[OMAX], cl[OMAX];
    uint64_t bs = 0, cs;
    for (int i = 0; i < n; i++) ord[i] = i;
    int first = 1;
    do {
        code_under(p, ord, cl, &cs);
        if (first || code_cmp(n, cl, cs, bl, bs) < 0) {
            memcpy(bl, cl, sizeof(cl)); bs = cs;
            memcpy(best, ord, sizeof(ord)); first = 0;
        }
    } while (next_perm(ord, n));
    out->n = n;
    memset(out->e, 0, sizeof(out->e));
    for (int i = 0; i < n; i++) out->lab[i] = p->lab[best[i]];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) out->e[i][j] = p->e[best[i]][best[j]];
}

/* Packed adjacency of a pattern: bit pair_pos(i,j) set when i~j (LSB-first).
 * This is the exported form; the sequence form above orders codes. */
static uint64_t pack_adj(const opat *p) {
    uint64_t a = 0;
    for (int i = 0; i < p->n; i++)
        for (int j = i + 1; j < p->n; j++)
            if (p->e[i][j]) a |= 1ull << pair_pos(i, j, p->n);
    return a;
}

static uint64_t seq_of(const opat *p) {
    int ord[OMAX];
    int32_t l[OMAX];
    uint64_t s;
    for (int i = 0; i < p->n; i++) ord[i] = i;
    code_under(p, ord, l, &s);
    return s;
}

/* orbit[v] = smallest vertex in v's automorphism orbit */
static void orbits(const opat *p, int *orbit) {
    int n = p->n, ord[OMAX];
    for (int i = 0; i < n; i++) { ord[i] = i; orbit[i] = i; }
    do {
        int ok = 1;
        for (int i = 0; i < n && ok; i++) {
            if (p->lab[ord[i]] != p->lab[i]) ok = 0;
            for (int j = 0; j < n && ok; j++)
                if (p->e[ord[i]][ord[j]] != p->e[i][j]) ok = 0;
        }
        if (!ok) continue;
        /* ord is an automorphism: i and ord[i] share an orbit */
        for (int i = 0; i < n; i++) {
            int a = orbit[i], b = orbit[ord[i]];
            int lo = a < b ? a : b, hi = a < b ? b : a;
            if (lo == hi) continue;
            for (int v = 0; v < n; v++)
                if (orbit[v] == hi) orbit[v] = lo;
        }
    } while (next_perm(ord, n));
}

static int connected_mask(const opat *p, unsigned mask) {
    if (!mask) return 0;
    unsigned seen = mask & (~mask + 1u), grow = seen;
    while (grow) {
        unsigned next = 0;
        for (int v = 0; v < p->n; v++)
            if (grow & (1u << v))
                for (int w = 0; w < p->n; w++)
                    if (p->e[v][w] && (mask & (1u << w)) && !(seen & (1u << w)))
                        next |= 1u << w;
        seen |= next;
        grow = next;
    }
    return seen == mask;
}

/* ----------------------------------------------------- pattern collections */

typedef struct {
    opat p;          /* canonical */
    uint64_t seq;    /* adjacency sequence of the canonical form */
    int64_t support; /* -1 while unknown, or infrequent */
} oentry;

typedef struct {
    oentry *v;
    int64_t len, cap;
} olist;

static int olist_push(olist *l, const oentry *e) {
    if (l->len == l->cap) {
        int64_t c = l->cap ? l->cap * 2 : 64;
        oentry *nv = (oentry *)realloc(l->v, sizeof(oentry) * (size_t)c);
        if (!nv) return -1;
        l->v = nv; l->cap = c;
    }
    l->v[l->len++] = *e;
    return 0;
}

static int entry_cmp(const void *a, const void *b) {
    const oentry *x = (const oentry *)a, *y = (const oentry *)b;
    if (x->p.n != y->p.n) return x->p.n < y->p.n ? -1 : 1;
    return code_cmp(x->p.n, x->p.lab, x->seq, y->p.lab, y->seq);
}

static void olist_sort_unique(olist *l) {
    if (!l->len) return;
    qsort(l->v, (size_t)l->len, sizeof(oentry), entry_cmp);
    int64_t u = 1;
    for (int64_t i = 1; i < l->len; i++)
        if (entry_cmp(&l->v[i], &l->v[u - 1]) != 0) l->v[u++] = l->v[i];
    l->len = u;
}

static int olist_contains(const olist *l, const opat *p) {
    oentry key;
    key.p = *p;
    key.seq = seq_of(p);
    int64_t lo = 0, hi = l->len;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        int c = entry_cmp(&l->v[mid], &key);
        if (c == 0) return 1;
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* -------------------------------------------------------- existence search */

typedef struct {
    const ograph *g;
    const opat *p;
    int induced;        /* 1: pattern non-edges must map onto non-edges */
    int order[OMAX];    /* matching order, order[0] = start vertex */
    int anchor[OMAX];   /* an earlier-matched pattern neighbour of order[d] */
    int32_t map[OMAX];  /* map[pattern vertex] = graph vertex */
} osearch;

static int search_from(osearch *s, int d) {
    const opat *p = s->p;
    if (d == p->n) return 1;
    int x = s->order[d];
    int32_t base = s->map[s->anchor[d]];
    int32_t want = p->lab[x];
    const ograph *g = s->g;
    int64_t i = row_lower(g, base, want, INT32_MIN);
    for (; i < g->off[base + 1]; i++) {
        int32_t c = g->adj[i];
        if (g->lab[c] != want) break;
        int ok = 1;
        for (int e = 0; e < d && ok; e++)
            if (s->map[s->order[e]] == c) ok = 0;           /* injective */
        for (int e = 0; e < d && ok; e++) {
            int y = s->order[e];
            if (p->e[x][y] && y != s->anchor[d] && !adjacent(g, s->map[y], c)) ok = 0;
            if (s->induced && !p->e[x][y] && adjacent(g, s->map[y], c)) ok = 0;
        }
        if (!ok) continue;
        s->map[x] = c;
        if (search_from(s, d + 1)) return 1;
    }
    return 0;
}

/* breadth-first matching order rooted at `start` (pattern is connected) */
static void plan_order(osearch *s, int start) {
    const opat *p = s->p;
    int seen[OMAX] = {0}, head = 0, tail = 0;
    s->order[tail++] = start;
    s->anchor[0] = -1;
    seen[start] = 1;
    while (head < tail) {
        int v = s->order[head++];
        for (int w = 0; w < p->n; w++)
            if (p->e[v][w] && !seen[w]) {
                seen[w] = 1;
                s->anchor[tail] = v;
                s->order[tail++] = w;
            }
    }
}

typedef struct {
    int32_t *verts;   /* vertices grouped by label */
    int64_t *start;   /* start[l] .. start[l+1] for label l */
    int32_t nlab;     /* labels are 0..nlab-1 after this table is built */
} obylabel;

static int bylabel_build(const ograph *g, obylabel *b) {
    int32_t maxl = 0;
    for (int64_t v = 0; v < g->n; v++) if (g->lab[v] > maxl) maxl = g->lab[v];
    b->nlab = maxl + 1;
    b->start = (int64_t *)calloc((size_t)b->nlab + 1, sizeof(int64_t));
    b->verts = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->n);
    if (!b->start || !b->verts) return -1;
    for (int64_t v = 0; v < g->n; v++) b->start[g->lab[v] + 1]++;
    for (int32_t l = 0; l < b->nlab; l++) b->start[l + 1] += b->start[l];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)b->nlab);
    if (!fill) return -1;
    memcpy(fill, b->start, sizeof(int64_t) * (size_t)b->nlab);
    for (int64_t v = 0; v < g->n; v++) b->verts[fill[g->lab[v]]++] = (int32_t)v;
    free(fill);
    return 0;
}

static void bylabel_free(obylabel *b) { free(b->verts); free(b->start); }

/* Exact MNI support of pattern p, or -1 once it is certainly below t.
 * When `t` <= 0 the exact support is always returned. */
static int64_t support_of(const ograph *g, const obylabel *bl, const opat *p,
                          int64_t t, int induced) {
    int orbit[OMAX];
    orbits(p, orbit);
    int64_t best = INT64_MAX;
    for (int c = 0; c < p->n; c++) {
        if (orbit[c] != c) continue;
        int32_t l = p->lab[c];
        if (l >= bl->nlab) return t > 0 ? -1 : 0;
        int64_t b = bl->start[l], e = bl->start[l + 1];
        int64_t found = 0, remaining = e - b;
        osearch s;
        s.g = g; s.p = p; s.induced = induced;
        plan_order(&s, c);
        for (int64_t i = b; i < e; i++) {
            s.map[c] = bl->verts[i];
            remaining--;
            if (search_from(&s, 1)) found++;
            if (t > 0 && found + remaining < t) return -1;
            if (found >= best) break;       /* cannot lower the minimum */
        }
        if (found < best) best = found;
    }
    if (t > 0 && best < t) return -1;
    return best;
}

/* ------------------------------------------------------------------ mining */

typedef struct oracle_result {
    int64_t count;
    int32_t *size;
    int32_t *labels;     /* count x 7, unused slots -1 */
    uint64_t *adj;       /* LSB-first pair bits of the canonical form */
    int64_t *support;
    int64_t level_candidates[OMAX + 1];
    int64_t level_frequent[OMAX + 1];
} oracle_result;

/* drop-vertex check: every connected one-vertex-smaller sub-pattern frequent */
static int subpatterns_frequent(const opat *q, const olist *prev) {
    if (q->n <= 2) return 1;
    unsigned all = (1u << q->n) - 1u;
    for (int x = 0; x < q->n; x++) {
        unsigned rest = all & ~(1u << x);
        if (!connected_mask(q, rest)) continue;
        opat sub, canon;
        sub.n = q->n - 1;
        memset(sub.e, 0, sizeof(sub.e));
        int map[OMAX], k = 0;
        for (int v = 0; v < q->n; v++) if (v != x) map[k++] = v;
        for (int i = 0; i < sub.n; i++) {
            sub.lab[i] = q->lab[map[i]];
            for (int j = 0; j < sub.n; j++) sub.e[i][j] = q->e[map[i]][map[j]];
        }
        canonicalize(&sub, &canon);
        if (!olist_contains(prev, &canon)) return 0;
    }
    return 1;
}

int oracle_mine_ex(int64_t n_vertices, int64_t n_edges, const int32_t *src,
                   const int32_t *dst, const int32_t *labels, int64_t support,
                   int32_t max_size, int32_t induced, oracle_result **out) {
    if (!out) return -1;
    *out = NULL;
    if (support < 1 || max_size < 2 || max_size > OMAX) return -1;
    ograph g;
    if (graph_build(&g, n_vertices, n_edges, src, dst, labels)) {
        graph_free(&g);
        return -1;
    }
    obylabel bl;
    if (bylabel_build(&g, &bl)) { graph_free(&g); return -1; }
    oracle_result *r = (oracle_result *)calloc(1, sizeof(oracle_result));
    olist all = {0}, cur = {0};
    /* size 1: frequent labels */
    for (int32_t l = 0; l < bl.nlab; l++)
        if (bl.start[l + 1] - bl.start[l] >= support) {
            oentry e;
            memset(&e, 0, sizeof(e));
            e.p.n = 1; e.p.lab[0] = l; e.seq = 0;
            e.support = bl.start[l + 1] - bl.start[l];
            olist_push(&cur, &e);
        }
    olist freq_labels = cur;      /* size-1 list doubles as the label menu */
    cur.v = NULL; cur.len = cur.cap = 0;
    for (int64_t i = 0; i < freq_labels.len; i++) olist_push(&cur, &freq_labels.v[i]);
    for (int k = 1; k < max_size; k++) {
        olist cand = {0};
        for (int64_t pi = 0; pi < cur.len; pi++) {
            const opat *p = &cur.v[pi].p;
            for (int64_t li = 0; li < freq_labels.len; li++) {
                for (unsigned s = 1; s < (1u << p->n); s++) {
                    oentry e;
                    memset(&e, 0, sizeof(e));
                    opat q = *p;
                    q.n = p->n + 1;
                    q.lab[p->n] = freq_labels.v[li].p.lab[0];
                    for (int v = 0; v < q.n; v++) { q.e[p->n][v] = 0; q.e[v][p->n] = 0; }
                    for (int v = 0; v < p->n; v++)
                        if (s & (1u << v)) q.e[v][p->n] = q.e[p->n][v] = 1;
                    canonicalize(&q, &e.p);
                    e.seq = seq_of(&e.p);
                    e.support = -1;
                    olist_push(&cand, &e);
                }
            }
        }
        olist_sort_unique(&cand);
        r->level_candidates[k + 1] = cand.len;
        olist next = {0};
        for (int64_t ci = 0; ci < cand.len; ci++) {
            oentry *e = &cand.v[ci];
            if (k + 1 >= 3 && !subpatterns_frequent(&e->p, &cur)) continue;
            e->support = support_of(&g, &bl, &e->p, support, induced);
            if (e->support >= support) {
                olist_push(&next, e);
                olist_push(&all, e);
            }
        }
        r->level_frequent[k + 1] = next.len;
        free(cand.v);
        free(cur.v);
        cur = next;
        if (!cur.len) break;
    }
    free(cur.v);
    free(freq_labels.v);
    olist_sort_unique(&all);
    r->count = all.len;
    r->size = (int32_t *)malloc(sizeof(int32_t) * (size_t)(all.len + 1));
    r->labels = (int32_t *)malloc(sizeof(int32_t) * OMAX * (size_t)(all.len + 1));
    r->adj = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(all.len + 1));
    r->support = (int64_t *)malloc(sizeof(int64_t) * (size_t)(all.len + 1));
    for (int64_t i = 0; i < all.len; i++) {
        const oentry *e = &all.v[i];
        r->size[i] = e->p.n;
        for (int j = 0; j < OMAX; j++) r->labels[i * OMAX + j] = j < e->p.n ? e->p.lab[j] : -1;
        r->adj[i] = pack_adj(&e->p);
        r->support[i] = e->support;
    }
    free(all.v);
    bylabel_free(&bl);
    graph_free(&g);
    *out = r;
    return 0;
}

int oracle_mine(int64_t n_vertices, int64_t n_edges, const int32_t *src,
                const int32_t *dst, const int32_t *labels, int64_t support,
                int32_t max_size, oracle_result **out) {
    return oracle_mine_ex(n_vertices, n_edges, src, dst, labels, support, max_size, 0, out);
}

int64_t oracle_result_count(const oracle_result *r) { return r ? r->count : -1; }

int oracle_result_get(const oracle_result *r, int32_t *sizes, int32_t *labels,
                      uint64_t *adj, int64_t *supports) {
    if (!r) return -1;
    memcpy(sizes, r->size, sizeof(int32_t) * (size_t)r->count);
    memcpy(labels, r->labels, sizeof(int32_t) * OMAX * (size_t)r->count);
    memcpy(adj, r->adj, sizeof(uint64_t) * (size_t)r->count);
    memcpy(supports, r->support, sizeof(int64_t) * (size_t)r->count);
    return 0;
}

/* candidates / frequent patterns seen per size, for diagnostics */
int oracle_result_levels(const oracle_result *r, int64_t *cand, int64_t *freq) {
    if (!r) return -1;
    for (int i = 0; i <= OMAX; i++) { cand[i] = r->level_candidates[i]; freq[i] = r->level_frequent[i]; }
    return 0;
}

void oracle_result_free(oracle_result *r) {
    if (!r) return;
    free(r->size); free(r->labels); free(r->adj); free(r->support);
    free(r);
}

/* Canonical form of one pattern given as labels + LSB-first pair bits. */
int oracle_canonical(int32_t n, const int32_t *labels, uint64_t adj,
                     int32_t *out_labels, uint64_t *out_adj) {
    if (n < 1 || n > OMAX) return -1;
    opat p, c;
    p.n = n;
    memset(p.e, 0, sizeof(p.e));
    for (int i = 0; i < n; i++) p.lab[i] = labels[i];
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            if (adj & (1ull << pair_pos(i, j, n))) p.e[i][j] = p.e[j][i] = 1;
    canonicalize(&p, &c);
    for (int i = 0; i < n; i++) out_labels[i] = c.lab[i];
    *out_adj = pack_adj(&c);
    return 0;
}

/* Exact MNI support of one pattern (labels + LSB-first pair bits); the
 * pattern must be connected.  Returns -1 on bad input. */
int64_t oracle_pattern_support_ex(int64_t n_vertices, int64_t n_edges,
                                  const int32_t *src, const int32_t *dst,
                                  const int32_t *labels, int32_t n,
                                  const int32_t *plabels, uint64_t padj, int32_t induced) {
    if (n < 1 || n > OMAX) return -1;
    opat p;
    p.n = n;
    memset(p.e, 0, sizeof(p.e));
    for (int i = 0; i < n; i++) p.lab[i] = plabels[i];
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            if (padj & (1ull << pair_pos(i, j, n))) p.e[i][j] = p.e[j][i] = 1;
    if (!connected_mask(&p, (1u << n) - 1u)) return -1;
    ograph g;
    if (graph_build(&g, n_vertices, n_edges, src, dst, labels)) { graph_free(&g); return -1; }
    obylabel bl;
    if (bylabel_build(&g, &bl)) { graph_free(&g); return -1; }
    int64_t s = support_of(&g, &bl, &p, 0, induced);
    bylabel_free(&bl);
    graph_free(&g);
    return s;
}

/* A normalised input graph kept for many support queries (same graph
 * normalisation and support search as above). */
typedef struct oracle_graph {
    ograph g;
    obylabel bl;
} oracle_graph;

oracle_graph *oracle_graph_new(int64_t n_vertices, int64_t n_edges, const int32_t *src,
                               const int32_t *dst, const int32_t *labels) {
    oracle_graph *h = (oracle_graph *)calloc(1, sizeof(oracle_graph));
    if (!h) return NULL;
    if (graph_build(&h->g, n_vertices, n_edges, src, dst, labels) ||
        bylabel_build(&h->g, &h->bl)) {
        graph_free(&h->g);
        free(h);
        return NULL;
    }
    return h;
}

/* MNI support of one connected pattern on a kept graph; with t > 0 the
 * search stops once the support is certainly below t and returns -1 (the
 * exact support otherwise).  -2 on a bad pattern. */
int64_t oracle_graph_support(const oracle_graph *h, int32_t n, const int32_t *plabels,
                             uint64_t padj, int64_t t, int32_t induced) {
    if (!h || n < 1 || n > OMAX) return -2;
    opat p;
    p.n = n;
    memset(p.e, 0, sizeof(p.e));
    for (int i = 0; i < n; i++) p.lab[i] = plabels[i];
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            if (padj & (1ull << pair_pos(i, j, n))) p.e[i][j] = p.e[j][i] = 1;
    if (!connected_mask(&p, (1u << n) - 1u)) return -2;
    return support_of(&h->g, &h->bl, &p, t, induced);
}

void oracle_graph_free(oracle_graph *h) {
    if (!h) return;
    bylabel_free(&h->bl);
    graph_free(&h->g);
    free(h);
}

int64_t oracle_pattern_support(int64_t n_vertices, int64_t n_edges,
                               const int32_t *src, const int32_t *dst,
                               const int32_t *labels, int32_t n,
                               const int32_t *plabels, uint64_t padj) {
    return oracle_pattern_support_ex(n_vertices, n_edges, src, dst, labels, n, plabels, padj, 0);
}

/* ------------------------------------------- connected subgraph counting */

typedef struct {
    const ograph *g;
    int size;
    int32_t sub[OMAX];
    int64_t total;
    int32_t *ext;        /* extension stack storage */
    int64_t ext_cap;
    uint8_t *mark;       /* per-vertex: in sub or in its neighbourhood */
} oesu;

/* connected spanning edge subsets of the subgraph induced by sub[0..k-1] */
static int64_t spanning_connected(const ograph *g, const int32_t *sub, int k) {
    int ei[OPAIRS], ej[OPAIRS], m = 0;
    for (int i = 0; i < k; i++)
        for (int j = i + 1; j < k; j++)
            if (adjacent(g, sub[i], sub[j])) { ei[m] = i; ej[m] = j; m++; }
    int64_t count = 0;
    opat p;
    p.n = k;
    for (uint64_t s = 0; s < (1ull << m); s++) {
        memset(p.e, 0, sizeof(p.e));
        for (int b = 0; b < m; b++)
            if (s & (1ull << b)) p.e[ei[b]][ej[b]] = p.e[ej[b]][ei[b]] = 1;
        if (connected_mask(&p, (1u << k) - 1u)) count++;
    }
    return count;
}

static int in_sub(const oesu *s, int k, int32_t v) {
    for (int i = 0; i < k; i++) if (s->sub[i] == v) return 1;
    return 0;
}

static int near_sub(const oesu *s, int k, int32_t v) {
    for (int i = 0; i < k; i++) if (adjacent(s->g, s->sub[i], v)) return 1;
    return 0;
}

/* Wernicke's ESU: every connected vertex set of the target size, once. */
static void esu_extend(oesu *s, int k, int32_t *ext, int64_t next_len, int32_t root) {
    if (k == s->size) {
        s->total += spanning_connected(s->g, s->sub, k);
        return;
    }
    int64_t len = next_len;
    while (len > 0) {
        int32_t w = ext[--len];
        /* new extension = remaining ext + exclusive neighbours of w above root */
        int32_t *nx = ext + next_len;
        int64_t nl = 0;
        for (int64_t i = 0; i < len; i++) nx[nl++] = ext[i];
        const ograph *g = s->g;
        for (int64_t i = g->off[w]; i < g->off[w + 1]; i++) {
            int32_t u = g->adj[i];
            if (u <= root || in_sub(s, k, u) || near_sub(s, k, u)) continue;
            int dup = 0;
            for (int64_t j = 0; j < nl; j++) if (nx[j] == u) { dup = 1; break; }
            if (!dup) nx[nl++] = u;
        }
        s->sub[k] = w;
        esu_extend(s, k + 1, nx, nl, root);
    }
}

/* Number of connected edge-induced subgraphs of G with exactly `size`
 * vertices (every (V', E') with E' a connected spanning edge set of V'). */
int64_t oracle_count_connected(int64_t n_vertices, int64_t n_edges,
                               const int32_t *src, const int32_t *dst,
                               const int32_t *labels, int32_t size) {
    if (size < 1 || size > OMAX) return -1;
    ograph g;
    if (graph_build(&g, n_vertices, n_edges, src, dst, labels)) { graph_free(&g); return -1; }
    int64_t maxdeg = 0;
    for (int64_t v = 0; v < g.n; v++)
        if (g.off[v + 1] - g.off[v] > maxdeg) maxdeg = g.off[v + 1] - g.off[v];
    oesu s;
    memset(&s, 0, sizeof(s));
    s.g = &g;
    s.size = size;
    s.ext_cap = (maxdeg + 1) * (OMAX + 1) * (OMAX + 1) + 16;
    s.ext = (int32_t *)malloc(sizeof(int32_t) * (size_t)s.ext_cap);
    if (!s.ext) { graph_free(&g); return -1; }
    for (int64_t v = 0; v < g.n; v++) {
        s.sub[0] = (int32_t)v;
        int64_t nl = 0;
        for (int64_t i = g.off[v]; i < g.off[v + 1]; i++)
            if (g.adj[i] > v) s.ext[nl++] = g.adj[i];
        if (size == 1) { s.total += 1; continue; }
        esu_extend(&s, 1, s.ext, nl, (int32_t)v);
    }
    free(s.ext);
    graph_free(&g);
    return s.total;
}
