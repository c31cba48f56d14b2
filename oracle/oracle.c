/*
 * CPU oracle for Motifs-k (arXiv 1804.09741).  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the package smoke check and the benchmark's CPU
 * baseline leg may load this file's library.  The product path (the HIP
 * library under paper_1804_09741_amd/) never calls it and shares no code,
 * header, table or constant with it.
 *
 * What it computes (Problem Motifs-k, Section 1): for a directed graph G and
 * k in 3..6, the histogram H_k(G) that counts the connected induced k-vertex
 * subgraphs of G grouped by isomorphism class.  "Connected" is weak
 * connectivity: delta(v) ignores arc direction (Section 2, definition of
 * delta and adj).  Each vertex set is counted once.
 *
 * How, plainly and single-threaded:
 *   1. every connected k-vertex set is listed exactly once by Wernicke's ESU
 *      enumeration (the exact enumeration FanMod is built on): root v, the
 *      extension set holds neighbours with larger ids, and a child only adds
 *      exclusive neighbours of the new vertex;
 *   2. the induced subgraph G[S] of the listed set S = (s_0..s_{k-1}) is
 *      written as a k(k-1)-bit adjacency code, bit i(k-1)+j-[j>i] set iff
 *      the arc s_i -> s_j exists (the key "is an adjacency matrix" of
 *      Section 3.2; row = source, diagonal skipped);
 *   3. the class of the code is its canonical form: the minimum code over
 *      all k! relabelings of the vertices, found by trying every one;
 *   4. the count of that canonical code is incremented (exact 64-bit).
 *
 * k = 7 (oracle_count7) follows the same steps with 42-bit codes and reports
 * the histogram by canonical code (no table of all 2^42 codes is made).
 *
 * Arc tests use an n x n bit matrix; neighbour lists delta(v) are built by
 * testing every pair.  Canonical forms are tabulated for every code when
 * k <= 5 and memoised per labeled code when k = 6 (a cache only: each entry
 * is the same brute-force minimum).
 *
 * Section 3 also counts H_k from the connected (k-2)-sets X instead of the
 * k-sets: every unordered pair {y, z} of vertices adjacent to X closes the
 * connected k-set X + {y, z}.  A k-set S is then reached once per "core" X
 * of S: a (k-2)-subset that induces a weakly connected subgraph and that
 * both remaining vertices of S touch.  That number depends only on the
 * class of G[S]; oracle_core_mult() computes it from this definition, by
 * trying every (k-2)-subset of a k-vertex code.  (The paper does not state
 * this divisor; see the readings of the paper in the design notes.)
 *
 * Error codes: 0 ok, -1 bad argument, -2 k out of range, -3 graph not a
 * simple digraph CSR, -4 out of memory, -5 output buffer too small.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ERANGE (-2)
#define OR_EGRAPH (-3)
#define OR_ENOMEM (-4)
#define OR_ESMALL (-5)

/* position of arc i -> j in a k-vertex adjacency code */
static int bit_of(int k, int i, int j) { return i * (k - 1) + j - (j > i ? 1 : 0); }

static void code_to_matrix(int k, uint32_t code, unsigned char a[6][6])
{
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
            a[i][j] = (i != j) && ((code >> bit_of(k, i, j)) & 1u);
}

/* weak connectivity of the k-vertex digraph given by code (graph search) */
int oracle_connected(int k, uint32_t code)
{
    unsigned char a[6][6];
    if (k < 1 || k > 6) return 0;
    code_to_matrix(k, code, a);
    int seen[6] = {0}, stack[6], top = 0, reached = 1;
    seen[0] = 1;
    stack[top++] = 0;
    while (top > 0) {
        int u = stack[--top];
        for (int w = 0; w < k; ++w)
            if (!seen[w] && (a[u][w] || a[w][u])) {
                seen[w] = 1;
                ++reached;
                stack[top++] = w;
            }
    }
    return reached == k;
}

/* number of cores of the k-vertex digraph given by code: subsets X of
 * k-2 vertices with G[X] weakly connected such that each of the two
 * vertices outside X has an arc to or from some vertex of X */
int oracle_core_mult(int k, uint32_t code)
{
    unsigned char a[6][6];
    if (k < 3 || k > 6) return OR_ERANGE;
    code_to_matrix(k, code, a);
    int cores = 0;
    for (int y = 0; y < k; ++y)
        for (int z = y + 1; z < k; ++z) {
            /* X = all vertices but y and z */
            int x[6], nx = 0;
            for (int v = 0; v < k; ++v)
                if (v != y && v != z) x[nx++] = v;
            int y_touches = 0, z_touches = 0;
            for (int i = 0; i < nx; ++i) {
                if (a[y][x[i]] || a[x[i]][y]) y_touches = 1;
                if (a[z][x[i]] || a[x[i]][z]) z_touches = 1;
            }
            if (!y_touches || !z_touches) continue;
            /* weak connectivity of G[X] by graph search from x[0] */
            int seen[6] = {0}, stack[6], top = 0, reached = 1;
            seen[0] = 1;
            stack[top++] = 0;
            while (top > 0) {
                int i = stack[--top];
                for (int j = 0; j < nx; ++j)
                    if (!seen[j] && (a[x[i]][x[j]] || a[x[j]][x[i]])) {
                        seen[j] = 1;
                        ++reached;
                        stack[top++] = j;
                    }
            }
            if (reached == nx) ++cores;
        }
    return cores;
}

/* next permutation in lexicographic order; 0 when p was the last one */
static int next_perm(int *p, int k)
{
    int i = k - 2;
    while (i >= 0 && p[i] > p[i + 1]) --i;
    if (i < 0) return 0;
    int j = k - 1;
    while (p[j] < p[i]) --j;
    int t = p[i]; p[i] = p[j]; p[j] = t;
    for (int l = i + 1, r = k - 1; l < r; ++l, --r) { t = p[l]; p[l] = p[r]; p[r] = t; }
    return 1;
}

/* canonical form: min over all relabelings pi of the code with arc
   pi(i) -> pi(j) for every arc i -> j of the input */
uint32_t oracle_canon(int k, uint32_t code)
{
    unsigned char a[6][6];
    int p[6];
    code_to_matrix(k, code, a);
    for (int i = 0; i < k; ++i) p[i] = i;
    uint32_t best = 0xFFFFFFFFu;
    do {
        uint32_t c = 0;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j)
                if (a[i][j]) c |= 1u << bit_of(k, p[i], p[j]);
        if (c < best) best = c;
    } while (next_perm(p, k));
    return best;
}

/* canon[c] and conn[c] for every code c of a k-vertex digraph, k <= 5 */
int oracle_canon_table(int k, uint32_t *canon, uint8_t *conn)
{
    if (k < 1 || k > 5) return OR_ERANGE;
    if (!canon || !conn) return OR_EINVAL;
    uint32_t ncodes = 1u << (k * (k - 1));
    for (uint32_t c = 0; c < ncodes; ++c) {
        canon[c] = oracle_canon(k, c);
        conn[c] = (uint8_t)oracle_connected(k, c);
    }
    return OR_OK;
}

/* ---------------- a small open-addressing map uint32 -> uint64 ---------- */

typedef struct {
    uint32_t *keys;
    uint64_t *vals;
    uint8_t *used;
    size_t cap, size;
} u32map;

static int map_init(u32map *m, size_t cap)
{
    m->cap = cap;
    m->size = 0;
    m->keys = (uint32_t *)malloc(cap * sizeof(uint32_t));
    m->vals = (uint64_t *)malloc(cap * sizeof(uint64_t));
    m->used = (uint8_t *)calloc(cap, 1);
    return (m->keys && m->vals && m->used) ? OR_OK : OR_ENOMEM;
}

static void map_free(u32map *m)
{
    free(m->keys);
    free(m->vals);
    free(m->used);
    m->keys = NULL; m->vals = NULL; m->used = NULL;
}

static size_t map_slot(const u32map *m, uint32_t key)
{
    size_t h = (size_t)(key * 2654435761u) & (m->cap - 1);
    while (m->used[h] && m->keys[h] != key) h = (h + 1) & (m->cap - 1);
    return h;
}

/* returns a pointer to the value of key, inserting 0 if absent (NULL: OOM) */
static uint64_t *map_get(u32map *m, uint32_t key, int *inserted)
{
    if (2 * (m->size + 1) > m->cap) {
        u32map bigger;
        if (map_init(&bigger, m->cap * 2) != OR_OK) { map_free(&bigger); return NULL; }
        for (size_t i = 0; i < m->cap; ++i)
            if (m->used[i]) {
                size_t s = map_slot(&bigger, m->keys[i]);
                bigger.used[s] = 1;
                bigger.keys[s] = m->keys[i];
                bigger.vals[s] = m->vals[i];
                bigger.size++;
            }
        map_free(m);
        *m = bigger;
    }
    size_t s = map_slot(m, key);
    *inserted = !m->used[s];
    if (!m->used[s]) {
        m->used[s] = 1;
        m->keys[s] = key;
        m->vals[s] = 0;
        m->size++;
    }
    return &m->vals[s];
}

/* ---------------- the enumeration --------------------------------------- */

typedef struct {
    int n, k;
    const uint64_t *arcbits; /* n*n bits, bit u*n+v set iff arc u -> v */
    size_t words_per_row;
    const int32_t *nb_ptr;   /* delta(v) = nb[nb_ptr[v] .. nb_ptr[v+1]) */
    const int32_t *nb;
    const uint32_t *canon_small; /* k <= 5: canonical form of every code */
    u32map *memo;                /* k == 6: labeled code -> canonical code */
    uint64_t *hist_small;        /* k <= 5: count per canonical code */
    u32map *hist_map;            /* k == 6: canonical code -> count */
    int *buf[6];                 /* extension set storage, one per depth */
    int sub[6];
    int failed;
} esu_ctx;

static int arc(const esu_ctx *e, int u, int v)
{
    size_t bit = (size_t)u * e->n + v;
    return (int)((e->arcbits[bit >> 6] >> (bit & 63)) & 1u);
}

static void record(esu_ctx *e)
{
    int k = e->k;
    uint32_t code = 0;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
            if (i != j && arc(e, e->sub[i], e->sub[j])) code |= 1u << bit_of(k, i, j);
    if (k <= 5) {
        e->hist_small[e->canon_small[code]] += 1;
        return;
    }
    int ins = 0;
    uint64_t *cv = map_get(e->memo, code, &ins);
    if (!cv) { e->failed = 1; return; }
    if (ins) *cv = oracle_canon(k, code);
    uint64_t *hv = map_get(e->hist_map, (uint32_t)*cv, &ins);
    if (!hv) { e->failed = 1; return; }
    *hv += 1;
}

/* is u in V_sub or adjacent (either direction) to a vertex of V_sub? */
static int in_closed_nbhd(const esu_ctx *e, int depth, int u)
{
    for (int i = 0; i < depth; ++i) {
        int s = e->sub[i];
        if (s == u || arc(e, s, u) || arc(e, u, s)) return 1;
    }
    return 0;
}

/* ESU extension step: V_sub = sub[0..depth), ext[0..next) is V_ext */
static void extend(esu_ctx *e, int depth, const int *ext, int next, int root)
{
    if (e->failed) return;
    if (depth == e->k) {
        record(e);
        return;
    }
    int *child = e->buf[depth];
    for (int i = 0; i < next; ++i) {
        int w = ext[i];
        /* V_ext' = (V_ext without w and without the ones taken before it)
                    + exclusive neighbours of w that exceed the root */
        int cn = 0;
        for (int j = i + 1; j < next; ++j) child[cn++] = ext[j];
        for (int t = e->nb_ptr[w]; t < e->nb_ptr[w + 1]; ++t) {
            int u = e->nb[t];
            if (u > root && !in_closed_nbhd(e, depth, u)) child[cn++] = u;
        }
        e->sub[depth] = w;
        extend(e, depth + 1, child, cn, root);
    }
}

typedef struct { uint32_t code; uint64_t count; } pair_t;

static int pair_cmp(const void *a, const void *b)
{
    uint32_t x = ((const pair_t *)a)->code, y = ((const pair_t *)b)->code;
    return (x > y) - (x < y);
}

static int check_graph(int n, const int32_t *row_ptr, const int32_t *col)
{
    if (n < 0 || !row_ptr) return OR_EINVAL;
    if (row_ptr[0] != 0) return OR_EGRAPH;
    for (int v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return OR_EGRAPH;
    if (row_ptr[n] > 0 && !col) return OR_EINVAL;
    for (int64_t e = 0; e < row_ptr[n]; ++e)
        if (col[e] < 0 || col[e] >= n) return OR_EGRAPH;
    return OR_OK;
}

/*
 * H_k of the digraph (n, row_ptr, col) given as out-adjacency CSR.
 * k <= 5 needs canon_small = the canonical form of every code (from
 * oracle_canon_table); k == 6 passes NULL.  On success writes the distinct
 * canonical codes that occur, ascending, to out_codes and their counts to
 * out_counts, returns how many there are, and stores the number of listed
 * subgraphs in *total.
 */
int64_t oracle_count(int n, const int32_t *row_ptr, const int32_t *col, int k,
                     const uint32_t *canon_small, uint32_t *out_codes,
                     uint64_t *out_counts, int64_t capacity, uint64_t *total)
{
    if (k < 3 || k > 6) return OR_ERANGE;
    int rc = check_graph(n, row_ptr, col);
    if (rc != OR_OK) return rc;
    if (k <= 5 && !canon_small) return OR_EINVAL;
    if (total) *total = 0;

    size_t wpr = ((size_t)n * n + 63) / 64;
    uint64_t *bits = (uint64_t *)calloc(wpr, sizeof(uint64_t));
    if (!bits) return OR_ENOMEM;
    int64_t result = 0;
    for (int u = 0; u < n && result == 0; ++u)
        for (int32_t t = row_ptr[u]; t < row_ptr[u + 1]; ++t) {
            int v = col[t];
            size_t bit = (size_t)u * n + v;
            if (u == v || ((bits[bit >> 6] >> (bit & 63)) & 1u)) { result = OR_EGRAPH; break; }
            bits[bit >> 6] |= 1ull << (bit & 63);
        }
    if (result != 0 || n < k) { free(bits); return result; }

    esu_ctx e;
    memset(&e, 0, sizeof(e));
    e.n = n;
    e.k = k;
    e.arcbits = bits;
    e.words_per_row = wpr;

    /* delta(v): every u with an arc either way, ascending */
    int32_t *nb_ptr = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * (2 * (size_t)row_ptr[n] + 1));
    if (!nb_ptr || !nb) { free(bits); free(nb_ptr); free(nb); return OR_ENOMEM; }
    e.nb_ptr = nb_ptr;
    e.nb = nb;
    int32_t cnt = 0;
    for (int v = 0; v < n; ++v) {
        nb_ptr[v] = cnt;
        for (int u = 0; u < n; ++u)
            if (u != v && (arc(&e, v, u) || arc(&e, u, v))) nb[cnt++] = u;
    }
    nb_ptr[n] = cnt;

    u32map memo, hmap;
    memset(&memo, 0, sizeof(memo));
    memset(&hmap, 0, sizeof(hmap));
    uint32_t ncodes = 1u << (k * (k - 1));
    if (k <= 5) {
        e.canon_small = canon_small;
        e.hist_small = (uint64_t *)calloc(ncodes, sizeof(uint64_t));
        if (!e.hist_small) result = OR_ENOMEM;
    } else {
        if (map_init(&memo, 1 << 16) != OR_OK || map_init(&hmap, 1 << 16) != OR_OK)
            result = OR_ENOMEM;
        e.memo = &memo;
        e.hist_map = &hmap;
    }

    int *ext = (int *)malloc(sizeof(int) * ((size_t)n + 1) * (size_t)(k + 1));
    if (!ext) result = OR_ENOMEM;
    for (int d = 0; d < k && ext; ++d) e.buf[d] = ext + (size_t)(d + 1) * ((size_t)n + 1);
    for (int v = 0; v < n && result == 0 && !e.failed; ++v) {
        int en = 0;
        for (int t = nb_ptr[v]; t < nb_ptr[v + 1]; ++t)
            if (nb[t] > v) ext[en++] = nb[t];
        e.sub[0] = v;
        extend(&e, 1, ext, en, v);
    }
    if (e.failed && result == 0) result = OR_ENOMEM;

    if (result == 0) {
        int64_t nout = 0;
        uint64_t sum = 0;
        if (k <= 5) {
            for (uint32_t c = 0; c < ncodes; ++c)
                if (e.hist_small[c]) {
                    if (nout < capacity) {
                        out_codes[nout] = c;
                        out_counts[nout] = e.hist_small[c];
                    }
                    sum += e.hist_small[c];
                    ++nout;
                }
        } else {
            /* ascending canonical codes */
            pair_t *pairs = (pair_t *)malloc(sizeof(pair_t) * (hmap.size + 1));
            if (!pairs) { result = OR_ENOMEM; goto done; }
            for (size_t s = 0; s < hmap.cap; ++s)
                if (hmap.used[s]) {
                    pairs[nout].code = hmap.keys[s];
                    pairs[nout].count = hmap.vals[s];
                    sum += hmap.vals[s];
                    ++nout;
                }
            qsort(pairs, (size_t)nout, sizeof(pair_t), pair_cmp);
            for (int64_t i = 0; i < nout && i < capacity; ++i) {
                out_codes[i] = pairs[i].code;
                out_counts[i] = pairs[i].count;
            }
            free(pairs);
        }
        if (total) *total = sum;
        result = nout > capacity ? OR_ESMALL : nout;
    }
done:
    free(ext);
    free(e.hist_small);
    map_free(&memo);
    map_free(&hmap);
    free(nb_ptr);
    free(nb);
    free(bits);
    return result;
}

/* ------------------------------------------------------------------------
 * Ensemble of random graphs (Section 1, step (a); the paper does not fix the
 * null model).  Reading: degree-preserving directed switches.  Graph r of an
 * ensemble with seed s draws from the SplitMix64 stream whose seed is output
 * r of SplitMix64(s); each attempt t takes outputs 2t and 2t+1 of that
 * stream, maps each to an arc index in [0, m) by the high 32 bits times m,
 * and with arcs a -> b and c -> d:
 *   rejects it when a = c or b = d (nothing would change), when a = d or
 *   c = b (a loop), or when a -> d or c -> b already exists (a duplicate);
 *   otherwise replaces the two arcs by a -> d and c -> b (each arc keeps its
 *   position in the CSR, so every out- and in-degree is kept).
 * Attempts go on until `target` switches are accepted or `max_attempts`
 * attempts are made.
 * ------------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output i (i = 0, 1, ...)
 * of seed s is the mixing function applied to s + (i + 1) * 0x9E3779B97F4A7C15. */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint32_t arc_index(uint64_t r, int64_t m)
{
    return (uint32_t)(((r >> 32) * (uint64_t)m) >> 32);
}

/* Graph r of the ensemble of (n, row_ptr, col) with seed `seed`: its arc
 * heads into out_col (m entries, same row_ptr).  Returns the number of
 * accepted switches, or a negative error code. */
int64_t oracle_switch_chain(int n, const int32_t *row_ptr, const int32_t *col, uint64_t seed,
                            uint64_t r, uint64_t target, uint64_t max_attempts, int32_t *out_col)
{
    int rc = check_graph(n, row_ptr, col);
    if (rc != OR_OK) return rc;
    const int64_t m = row_ptr[n];
    if (m > 0 && !out_col) return OR_EINVAL;
    int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
    size_t nbits = (size_t)n * (size_t)n;
    unsigned char *arc = (unsigned char *)calloc(nbits + 1, 1);
    if (!src || !arc) { free(src); free(arc); return OR_ENOMEM; }
    for (int u = 0; u < n; ++u)
        for (int32_t t = row_ptr[u]; t < row_ptr[u + 1]; ++t) {
            src[t] = u;
            out_col[t] = col[t];
            arc[(size_t)u * n + col[t]] = 1;
        }
    const uint64_t stream = oracle_splitmix64(seed, r);
    uint64_t accepted = 0;
    for (uint64_t t = 0; m > 0 && accepted < target && t < max_attempts; ++t) {
        uint32_t i = arc_index(oracle_splitmix64(stream, 2 * t), m);
        uint32_t j = arc_index(oracle_splitmix64(stream, 2 * t + 1), m);
        int a = src[i], b = out_col[i], c = src[j], d = out_col[j];
        if (a == c || b == d) continue;
        if (a == d || c == b) continue;
        if (arc[(size_t)a * n + d] || arc[(size_t)c * n + b]) continue;
        arc[(size_t)a * n + b] = 0;
        arc[(size_t)c * n + d] = 0;
        arc[(size_t)a * n + d] = 1;
        arc[(size_t)c * n + b] = 1;
        out_col[i] = d;
        out_col[j] = b;
        ++accepted;
    }
    free(src);
    free(arc);
    return (int64_t)accepted;
}

/* ------------------------------------------------------------------------
 * k = 7.  Section 1 gives the number of 7-vertex classes (880,471,142); a
 * table over all 2^42 codes is out of reach, so the histogram is keyed by
 * canonical code.  Same definition as above with 42-bit codes: ESU lists
 * every connected 7-set once, its code has bit i*6 + j - [j > i] set iff
 * arc s_i -> s_j, and its class is the minimum code over all 5040
 * relabelings, found by trying every one (memoised per labeled code).
 */

typedef struct {
    uint64_t *keys;
    uint64_t *vals;
    uint8_t *used;
    size_t cap, size;
} u64map;

static int map64_init(u64map *m, size_t cap)
{
    m->cap = cap;
    m->size = 0;
    m->keys = (uint64_t *)malloc(cap * sizeof(uint64_t));
    m->vals = (uint64_t *)malloc(cap * sizeof(uint64_t));
    m->used = (uint8_t *)calloc(cap, 1);
    return (m->keys && m->vals && m->used) ? OR_OK : OR_ENOMEM;
}

static void map64_free(u64map *m)
{
    free(m->keys);
    free(m->vals);
    free(m->used);
    m->keys = NULL; m->vals = NULL; m->used = NULL;
}

static size_t map64_slot(const u64map *m, uint64_t key)
{
    size_t h = (size_t)((key * 0x9E3779B97F4A7C15ull) >> 20) & (m->cap - 1);
    while (m->used[h] && m->keys[h] != key) h = (h + 1) & (m->cap - 1);
    return h;
}

/* pointer to the value of key, inserting 0 if absent (NULL: out of memory) */
static uint64_t *map64_get(u64map *m, uint64_t key, int *inserted)
{
    if (2 * (m->size + 1) > m->cap) {
        u64map bigger;
        if (map64_init(&bigger, m->cap * 2) != OR_OK) { map64_free(&bigger); return NULL; }
        for (size_t i = 0; i < m->cap; ++i)
            if (m->used[i]) {
                size_t s = map64_slot(&bigger, m->keys[i]);
                bigger.used[s] = 1;
                bigger.keys[s] = m->keys[i];
                bigger.vals[s] = m->vals[i];
                bigger.size++;
            }
        map64_free(m);
        *m = bigger;
    }
    size_t s = map64_slot(m, key);
    *inserted = !m->used[s];
    if (!m->used[s]) {
        m->used[s] = 1;
        m->keys[s] = key;
        m->vals[s] = 0;
        m->size++;
    }
    return &m->vals[s];
}

/* canonical form of a 7-vertex code: min over all relabelings pi of the
   code with arc pi(i) -> pi(j) for every arc i -> j */
uint64_t oracle_canon7(uint64_t code)
{
    int ai[42], aj[42], na = 0;  /* the arcs i -> j of the code */
    for (int i = 0; i < 7; ++i)
        for (int j = 0; j < 7; ++j)
            if (i != j && ((code >> bit_of(7, i, j)) & 1u)) {
                ai[na] = i;
                aj[na] = j;
                ++na;
            }
    int p[7];
    for (int i = 0; i < 7; ++i) p[i] = i;
    uint64_t best = ~0ull;
    do {
        uint64_t c = 0;
        for (int t = 0; t < na; ++t) c |= 1ull << bit_of(7, p[ai[t]], p[aj[t]]);
        best = c < best ? c : best;
    } while (next_perm(p, 7));
    return best;
}

typedef struct {
    int n;
    const uint64_t *arcbits; /* n*n bits, bit u*n+v set iff arc u -> v */
    const int32_t *nb_ptr;   /* delta(v) = nb[nb_ptr[v] .. nb_ptr[v+1]) */
    const int32_t *nb;
    u64map *memo;            /* labeled code -> canonical code */
    u64map *hist;            /* canonical code -> count */
    int *buf[7];
    int sub[7];
    int failed;
} esu7_ctx;

static int arc7(const esu7_ctx *e, int u, int v)
{
    size_t bit = (size_t)u * e->n + v;
    return (int)((e->arcbits[bit >> 6] >> (bit & 63)) & 1u);
}

static void record7(esu7_ctx *e)
{
    uint64_t code = 0;
    for (int i = 0; i < 7; ++i)
        for (int j = 0; j < 7; ++j)
            if (i != j && arc7(e, e->sub[i], e->sub[j])) code |= 1ull << bit_of(7, i, j);
    int ins = 0;
    uint64_t *cv = map64_get(e->memo, code, &ins);
    if (!cv) { e->failed = 1; return; }
    if (ins) *cv = oracle_canon7(code);
    const uint64_t canon = *cv;
    uint64_t *hv = map64_get(e->hist, canon, &ins);
    if (!hv) { e->failed = 1; return; }
    *hv += 1;
}

static int in_closed_nbhd7(const esu7_ctx *e, int depth, int u)
{
    for (int i = 0; i < depth; ++i) {
        int s = e->sub[i];
        if (s == u || arc7(e, s, u) || arc7(e, u, s)) return 1;
    }
    return 0;
}

/* ESU extension step: V_sub = sub[0..depth), ext[0..next) is V_ext */
static void extend7(esu7_ctx *e, int depth, const int *ext, int next, int root)
{
    if (e->failed) return;
    if (depth == 7) {
        record7(e);
        return;
    }
    int *child = e->buf[depth];
    for (int i = 0; i < next; ++i) {
        int w = ext[i];
        int cn = 0;
        for (int j = i + 1; j < next; ++j) child[cn++] = ext[j];
        for (int t = e->nb_ptr[w]; t < e->nb_ptr[w + 1]; ++t) {
            int u = e->nb[t];
            if (u > root && !in_closed_nbhd7(e, depth, u)) child[cn++] = u;
        }
        e->sub[depth] = w;
        extend7(e, depth + 1, child, cn, root);
    }
}

typedef struct { uint64_t code; uint64_t count; } pair64_t;

static int pair64_cmp(const void *a, const void *b)
{
    uint64_t x = ((const pair64_t *)a)->code, y = ((const pair64_t *)b)->code;
    return (x > y) - (x < y);
}

/*
 * H_7 of the digraph (n, row_ptr, col) given as out-adjacency CSR: the
 * distinct canonical codes that occur, ascending, in out_codes, their counts
 * in out_counts; returns how many there are (OR_ESMALL when more than
 * capacity) and stores the number of listed subgraphs in *total.
 */
int64_t oracle_count7(int n, const int32_t *row_ptr, const int32_t *col, uint64_t *out_codes,
                      uint64_t *out_counts, int64_t capacity, uint64_t *total)
{
    int rc = check_graph(n, row_ptr, col);
    if (rc != OR_OK) return rc;
    if (total) *total = 0;
    size_t words = ((size_t)n * n + 63) / 64;
    uint64_t *bits = (uint64_t *)calloc(words + 1, sizeof(uint64_t));
    if (!bits) return OR_ENOMEM;
    for (int u = 0; u < n; ++u)
        for (int32_t t = row_ptr[u]; t < row_ptr[u + 1]; ++t) {
            int v = col[t];
            size_t bit = (size_t)u * n + v;
            if (u == v || ((bits[bit >> 6] >> (bit & 63)) & 1u)) { free(bits); return OR_EGRAPH; }
            bits[bit >> 6] |= 1ull << (bit & 63);
        }
    if (n < 7) { free(bits); return 0; }

    esu7_ctx e;
    memset(&e, 0, sizeof(e));
    e.n = n;
    e.arcbits = bits;
    int32_t *nb_ptr = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * (2 * (size_t)row_ptr[n] + 1));
    int *ext = (int *)malloc(sizeof(int) * ((size_t)n + 1) * 8);
    u64map memo, hist;
    memset(&memo, 0, sizeof(memo));
    memset(&hist, 0, sizeof(hist));
    int64_t result = 0;
    if (!nb_ptr || !nb || !ext || map64_init(&memo, 1 << 16) != OR_OK ||
        map64_init(&hist, 1 << 16) != OR_OK) {
        result = OR_ENOMEM;
        goto done;
    }
    e.nb_ptr = nb_ptr;
    e.nb = nb;
    e.memo = &memo;
    e.hist = &hist;
    /* delta(v): every u with an arc either way, ascending */
    int32_t cnt = 0;
    for (int v = 0; v < n; ++v) {
        nb_ptr[v] = cnt;
        for (int u = 0; u < n; ++u)
            if (u != v && (arc7(&e, v, u) || arc7(&e, u, v))) nb[cnt++] = u;
    }
    nb_ptr[n] = cnt;
    for (int d = 0; d < 7; ++d) e.buf[d] = ext + (size_t)(d + 1) * ((size_t)n + 1);
    for (int v = 0; v < n && !e.failed; ++v) {
        int en = 0;
        for (int t = nb_ptr[v]; t < nb_ptr[v + 1]; ++t)
            if (nb[t] > v) ext[en++] = nb[t];
        e.sub[0] = v;
        extend7(&e, 1, ext, en, v);
    }
    if (e.failed) {
        result = OR_ENOMEM;
        goto done;
    }
    {
        pair64_t *pairs = (pair64_t *)malloc(sizeof(pair64_t) * (hist.size + 1));
        if (!pairs) {
            result = OR_ENOMEM;
            goto done;
        }
        int64_t nout = 0;
        uint64_t sum = 0;
        for (size_t s = 0; s < hist.cap; ++s)
            if (hist.used[s]) {
                pairs[nout].code = hist.keys[s];
                pairs[nout].count = hist.vals[s];
                sum += hist.vals[s];
                ++nout;
            }
        qsort(pairs, (size_t)nout, sizeof(pair64_t), pair64_cmp);
        for (int64_t i = 0; i < nout && i < capacity; ++i) {
            out_codes[i] = pairs[i].code;
            out_counts[i] = pairs[i].count;
        }
        free(pairs);
        if (total) *total = sum;
        result = nout > capacity ? OR_ESMALL : nout;
    }
done:
    map64_free(&memo);
    map64_free(&hist);
    free(ext);
    free(nb_ptr);
    free(nb);
    free(bits);
    return result;
}
