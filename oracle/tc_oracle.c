/*
 * CPU ORACLE for the cover-edge + forward + hashing triangle count.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU library: no headers, kernels, helpers or tables.
 *
 * Plain, serial, obviously-correct C (one routine, orc_count_emd_entries,
 * shares its edges among OpenMP threads to time the definition on every host
 * core).
 * Every routine names the passage of
 * Bader, "Fast Triangle Counting" (arXiv 2309.09064) that it follows.  Row
 * pointers are int64 here; the Python wrapper converts.
 *
 * Definitions (paper, Introduction and Section II):
 *   G = (V, E) simple undirected, CSR with sorted rows, both directions stored.
 *   A triangle is a set {a, b, c} of distinct vertices with ab, bc, ca in E.
 *   L(v): BFS level, each component searched from its smallest unvisited id
 *   (Algorithm 4, first loop), L(root) = 0.
 *   E0 = {uv : L(u) = L(v)} (horizontal), E1 = E \ E0 (Algorithm 4, partition).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ CSR */

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/*
 * Simple undirected graph in CSR from raw tuples (paper, Introduction: the
 * input is CSR; experimental rules: sorted rows read-only).  Self-loops are
 * dropped, each tuple is stored in both directions, duplicates are removed,
 * rows are sorted ascending.  Returns nnz, -1 if an id is outside [0, n),
 * -2 if nnz > cap, -3 on allocation failure.
 */
int64_t orc_build_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                      int64_t *row_ptr, int32_t *col, int64_t cap)
{
    uint64_t *key = (uint64_t *)malloc((size_t)(2 * m + 1) * sizeof(uint64_t));
    if (!key) return -3;
    int64_t k = 0;
    for (int64_t e = 0; e < m; ++e) {
        int64_t u = src[e], v = dst[e];
        if (u < 0 || u >= n || v < 0 || v >= n) { free(key); return -1; }
        if (u == v) continue;
        key[k++] = ((uint64_t)u << 32) | (uint64_t)v;
        key[k++] = ((uint64_t)v << 32) | (uint64_t)u;
    }
    qsort(key, (size_t)k, sizeof(uint64_t), cmp_u64);
    for (int64_t v = 0; v <= n; ++v) row_ptr[v] = 0;
    int64_t nnz = 0;
    for (int64_t i = 0; i < k; ++i) {
        if (i > 0 && key[i] == key[i - 1]) continue;
        if (nnz >= cap) { free(key); return -2; }
        col[nnz++] = (int32_t)(key[i] & 0xffffffffu);
        row_ptr[(key[i] >> 32) + 1]++;
    }
    for (int64_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
    free(key);
    return nnz;
}

/* ------------------------------------------------------------------ BFS */

/*
 * Algorithm 4, first loop (same as Algorithm 3): for v = 0..n-1 in id order,
 * if v is unvisited, BFS(G, v).  L(v) is the hop distance from the root of
 * v's search; the root gets level 0.  FIFO queue, textbook BFS.
 * Returns the number of components (roots), or -3 on allocation failure.
 */
int64_t orc_bfs_levels(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t *level)
{
    int32_t *queue = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!queue) return -3;
    for (int64_t v = 0; v < n; ++v) level[v] = -1;
    int64_t roots = 0;
    for (int64_t r = 0; r < n; ++r) {
        if (level[r] >= 0) continue;
        ++roots;
        int64_t head = 0, tail = 0;
        level[r] = 0;
        queue[tail++] = (int32_t)r;
        while (head < tail) {
            int32_t u = queue[head++];
            for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
                int32_t w = col[j];
                if (level[w] < 0) {
                    level[w] = level[u] + 1;
                    queue[tail++] = w;
                }
            }
        }
    }
    free(queue);
    return roots;
}

/* --------------------------------------------------------- partition (E0/E1) */

/*
 * Algorithm 4, partition loop: E0 = horizontal edges (equal levels), E1 = the
 * rest.  Output CSRs keep each row in input (ascending) order:
 *   N1(x)  = neighbours y with L(y) != L(x)                       (rp1, c1)
 *   N0(x)  = neighbours y with L(y) == L(x), stored as the part with
 *            rank(y) > rank(x) first, then the part with rank(y) < rank(x);
 *            each part ascending by id.                            (rp0, c0)
 *   up0[x] = |{y in N0(x) : rank(y) > rank(x)}|
 * With by_id == 0, rank(x) = (deg(x), x) compared lexicographically, deg =
 * full degree in G: the forward algorithm's vertex order (paper, Related
 * work: forward with degree ordering; the paper leaves the tie-break open,
 * ids break ties here).  With by_id != 0, rank(x) = x: the u < v of
 * Algorithms 2 and 4 as printed.
 */
static int rank_above(const int64_t *rp, int64_t y, int64_t x, int by_id)
{
    if (by_id) return y > x;
    int64_t dy = rp[y + 1] - rp[y], dx = rp[x + 1] - rp[x];
    return dy > dx || (dy == dx && y > x);
}

void orc_partition(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *level, int32_t by_id,
                   int64_t *rp0, int32_t *c0, int32_t *up0, int64_t *rp1, int32_t *c1)
{
    rp0[0] = 0;
    rp1[0] = 0;
    for (int64_t x = 0; x < n; ++x) {
        int64_t p0 = rp0[x], p1 = rp1[x];
        int32_t up = 0;
        for (int64_t j = row_ptr[x]; j < row_ptr[x + 1]; ++j) {      /* upper part of N0 */
            int32_t y = col[j];
            if (level[y] == level[x] && rank_above(row_ptr, y, x, by_id)) { c0[p0++] = y; ++up; }
        }
        for (int64_t j = row_ptr[x]; j < row_ptr[x + 1]; ++j) {      /* lower part of N0 */
            int32_t y = col[j];
            if (level[y] == level[x] && !rank_above(row_ptr, y, x, by_id)) c0[p0++] = y;
        }
        for (int64_t j = row_ptr[x]; j < row_ptr[x + 1]; ++j) {      /* N1 */
            int32_t y = col[j];
            if (level[y] != level[x]) c1[p1++] = y;
        }
        up0[x] = up;
        rp0[x + 1] = p0;
        rp1[x + 1] = p1;
    }
}

/* ------------------------------------------------ T0 and T1 of Algorithm 4 */

/*
 * The two counts Algorithm 4 adds up, for levels L, each computed from what
 * it counts rather than by the algorithm's loops:
 *   G0 = (V, E0) with E0 = {uv : L(u) = L(v)} (the partition loop), and
 *   G1 = (V, E \ E0), each as a CSR;
 *   T0 = triangles with all three edges in E0 (Algorithm 4 hands G0 to the
 *        forward algorithm, Algorithm 2, which counts exactly these): every
 *        triangle u < v < w of G0 once, from its two smaller vertices;
 *   T1 = for every horizontal edge uv with u < v, the common members of
 *        N1(u) and N1(v) (the hashed loop's intersection): the triangles whose
 *        third vertex lies on another level, each counted from its one
 *        horizontal edge.
 * A common member is found by marking the set N(u) in a vertex-indexed
 * Boolean array and testing each member of the other list against it.
 * With |L(u) - L(v)| <= 1 on every edge, a triangle with two horizontal
 * edges has all three on one level, and one with none would need three
 * distinct levels each within one of the others, which integers do not
 * allow; so T0 + T1 = T (the cover-edge argument of Section II).
 * Outputs T0, T1 and |E0| (undirected).  Returns 0, or -3 on allocation
 * failure.
 */
int orc_alg4(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *level,
             uint64_t *t0_out, uint64_t *t1_out, int64_t *e0_out)
{
    const int64_t nnz = row_ptr[n];
    int64_t *rp0 = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int64_t *rp1 = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *g0 = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    int32_t *g1 = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    unsigned char *in_u = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!rp0 || !rp1 || !g0 || !g1 || !in_u) {
        free(rp0); free(rp1); free(g0); free(g1); free(in_u);
        return -3;
    }
    /* partition: each stored (directed) CSR entry goes to G0 or G1 */
    rp0[0] = rp1[0] = 0;
    for (int64_t u = 0; u < n; ++u) {
        int64_t p0 = rp0[u], p1 = rp1[u];
        for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
            int32_t v = col[j];
            if (level[u] == level[v]) g0[p0++] = v; else g1[p1++] = v;
        }
        rp0[u + 1] = p0;
        rp1[u + 1] = p1;
    }
    uint64_t T0 = 0, T1 = 0;
    for (int64_t u = 0; u < n; ++u) {
        /* T0: w in N0(u) and in N0(v), u < v < w */
        for (int64_t j = rp0[u]; j < rp0[u + 1]; ++j) in_u[g0[j]] = 1;
        for (int64_t j = rp0[u]; j < rp0[u + 1]; ++j) {
            int64_t v = g0[j];
            if (v <= u) continue;
            for (int64_t i = rp0[v]; i < rp0[v + 1]; ++i)
                if (g0[i] > v && in_u[g0[i]]) ++T0;
        }
        for (int64_t j = rp0[u]; j < rp0[u + 1]; ++j) in_u[g0[j]] = 0;
        /* T1: w in N1(u) and in N1(v) for the horizontal edge uv, u < v */
        for (int64_t j = rp1[u]; j < rp1[u + 1]; ++j) in_u[g1[j]] = 1;
        for (int64_t j = rp0[u]; j < rp0[u + 1]; ++j) {
            int64_t v = g0[j];
            if (v <= u) continue;
            for (int64_t i = rp1[v]; i < rp1[v + 1]; ++i)
                if (in_u[g1[i]]) ++T1;
        }
        for (int64_t j = rp1[u]; j < rp1[u + 1]; ++j) in_u[g1[j]] = 0;
    }
    *t0_out = T0;
    *t1_out = T1;
    *e0_out = rp0[n] / 2;
    free(rp0); free(rp1); free(g0); free(g1); free(in_u);
    return 0;
}

/* ----------------------------------------------------- plain-definition count */

/*
 * Direction-oriented edge iterator with a sorted merge ("EMD" in the paper's
 * list of algorithms): for every u and every neighbour v > u, count common
 * neighbours w > v by a two-pointer merge of the sorted rows.  Counts each
 * triangle u < v < w exactly once: the plain definition of T.
 */
uint64_t orc_count_emd(int64_t n, const int64_t *row_ptr, const int32_t *col)
{
    uint64_t T = 0;
    for (int64_t u = 0; u < n; ++u) {
        for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
            int64_t v = col[j];
            if (v <= u) continue;
            int64_t a = row_ptr[u], ae = row_ptr[u + 1], b = row_ptr[v], be = row_ptr[v + 1];
            while (a < ae && b < be) {
                if (col[a] < col[b]) ++a;
                else if (col[a] > col[b]) ++b;
                else { if (col[a] > v) ++T; ++a; ++b; }
            }
        }
    }
    return T;
}

/*
 * The same count restricted to the CSR entries listed in es[0..k): an entry
 * e = (u, v) with u < v adds the common neighbours w > v of u and v, so each
 * triangle u < v < w is counted at the entry of its edge uv.  Entries with
 * v < u add nothing (each undirected edge does its work at one of its two
 * entries).  The entries are shared among `threads` OpenMP threads (1 =
 * serial), so a sample of edges times the definition on every host core;
 * the whole range of entries gives T.  The row u of an entry is found by
 * binary search in row_ptr.
 */
uint64_t orc_count_emd_entries(int64_t n, const int64_t *row_ptr, const int32_t *col, int64_t k, const int64_t *es,
                               int threads)
{
    uint64_t T = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : T) num_threads(threads)
    for (int64_t i = 0; i < k; ++i) {
        int64_t e = es[i];
        int64_t lo = 0, hi = n - 1;           /* last row u with row_ptr[u] <= e */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo + 1) / 2;
            if (row_ptr[mid] <= e) lo = mid; else hi = mid - 1;
        }
        int64_t u = lo, v = col[e];
        if (v <= u) continue;
        int64_t a = row_ptr[u], ae = row_ptr[u + 1], b = row_ptr[v], be = row_ptr[v + 1];
        while (a < ae && b < be) {
            if (col[a] < col[b]) ++a;
            else if (col[a] > col[b]) ++b;
            else { if (col[a] > v) ++T; ++a; ++b; }
        }
    }
    return T;
}

/* -------------------------------------------------------------- Algorithm 3 */

/*
 * Cover-edge triangle count (Algorithm 3) given levels: for each horizontal
 * edge (u, v) with u < v, each common neighbour w counts if L(w) != L(u), or
 * if L(w) == L(u) and v < w.  Intersection by sorted merge.
 */
uint64_t orc_alg3(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *level)
{
    uint64_t T = 0;
    for (int64_t u = 0; u < n; ++u) {
        for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
            int64_t v = col[j];
            if (!(level[u] == level[v] && u < v)) continue;
            int64_t a = row_ptr[u], ae = row_ptr[u + 1], b = row_ptr[v], be = row_ptr[v + 1];
            while (a < ae && b < be) {
                if (col[a] < col[b]) ++a;
                else if (col[a] > col[b]) ++b;
                else {
                    int64_t w = col[a];
                    if (level[w] != level[u] || v < w) ++T;
                    ++a; ++b;
                }
            }
        }
    }
    return T;
}

/* ------------------------------------------------ per-vertex triangle counts */

/*
 * t(v) = number of triangles containing v (the clustering-coefficient input
 * the paper's introduction motivates).  Plain definition by sorted merge:
 * each triangle u < v < w adds 1 to t(u), t(v) and t(w).
 */
void orc_vertex_triangles(int64_t n, const int64_t *row_ptr, const int32_t *col, uint64_t *tv)
{
    for (int64_t v = 0; v < n; ++v) tv[v] = 0;
    for (int64_t u = 0; u < n; ++u) {
        for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
            int64_t v = col[j];
            if (v <= u) continue;
            int64_t a = row_ptr[u], ae = row_ptr[u + 1], b = row_ptr[v], be = row_ptr[v + 1];
            while (a < ae && b < be) {
                if (col[a] < col[b]) ++a;
                else if (col[a] > col[b]) ++b;
                else {
                    if (col[a] > v) { tv[u]++; tv[v]++; tv[col[a]]++; }
                    ++a; ++b;
                }
            }
        }
    }
}

/*
 * t(v) for a sample of vertices, one at a time, from the other plain
 * definition: the edges among the neighbours of v, i.e. half the sum over
 * u in N(v) of |N(u) and N(v) in common| (every such edge is seen from both
 * ends).  Each common count binary-searches the members of N(v) in N(u), so
 * a vertex of degree d costs about d^2 log(d_max): meant for samples of
 * modest degree on graphs too large for the whole-graph routine.
 */
static int64_t in_row(const int32_t *a, int64_t len, int32_t key)
{
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo < len && a[lo] == key;
}

void orc_vertex_triangles_at(int64_t n, const int64_t *row_ptr, const int32_t *col, int64_t k,
                             const int64_t *vs, uint64_t *out)
{
    (void)n;
    for (int64_t i = 0; i < k; ++i) {
        int64_t v = vs[i];
        const int32_t *nv = col + row_ptr[v];
        int64_t dv = row_ptr[v + 1] - row_ptr[v];
        uint64_t twice = 0;
        for (int64_t j = 0; j < dv; ++j) {
            int64_t u = nv[j];
            const int32_t *nu = col + row_ptr[u];
            int64_t du = row_ptr[u + 1] - row_ptr[u];
            for (int64_t t = 0; t < dv; ++t) twice += (uint64_t)in_row(nu, du, nv[t]);
        }
        out[i] = twice / 2;
    }
}

/* ------------------------------------------------ per-edge triangle counts */

/*
 * Support of every edge (the k-truss input the paper's introduction
 * motivates): for each input entry e = (u, v), sup[e] = the number of
 * triangles containing {u, v}, i.e. the common neighbours of u and v,
 * counted by a sorted merge of the two rows.
 */
void orc_edge_support(int64_t n, const int64_t *row_ptr, const int32_t *col, uint32_t *sup)
{
    for (int64_t u = 0; u < n; ++u) {
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t v = col[e];
            int64_t a = row_ptr[u], ae = row_ptr[u + 1], b = row_ptr[v], be = row_ptr[v + 1];
            uint32_t c = 0;
            while (a < ae && b < be) {
                if (col[a] < col[b]) ++a;
                else if (col[a] > col[b]) ++b;
                else { ++c; ++a; ++b; }
            }
            sup[e] = c;
        }
    }
}

/*
 * The same for a sample of entries, one at a time: the row u of each entry is
 * found by binary search in row_ptr, and every member of N(u) is looked up in
 * N(v) by binary search (cost about deg(u) log deg(v) per entry).
 */
void orc_edge_support_at(int64_t n, const int64_t *row_ptr, const int32_t *col, int64_t k,
                         const int64_t *entries, uint32_t *out)
{
    for (int64_t i = 0; i < k; ++i) {
        int64_t e = entries[i];
        int64_t lo = 0, hi = n - 1;           /* last row u with row_ptr[u] <= e */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo + 1) / 2;
            if (row_ptr[mid] <= e) lo = mid; else hi = mid - 1;
        }
        int64_t u = lo, v = col[e];
        const int32_t *nv = col + row_ptr[v];
        int64_t dv = row_ptr[v + 1] - row_ptr[v];
        uint32_t c = 0;
        for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) c += (uint32_t)in_row(nv, dv, col[j]);
        out[i] = c;
    }
}

/* ------------------------------------------------ degree relabel */

static const int64_t *g_rl_deg;

static int cmp_deg_desc(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_rl_deg[x] != g_rl_deg[y]) return g_rl_deg[x] > g_rl_deg[y] ? -1 : 1;
    return (x > y) - (x < y);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Degree ordering (Section III, last paragraph; BaderD / CED): vertices
 * sorted by decreasing degree, ties by increasing id; perm[new] = old.  The
 * relabelled rows are sorted.  Returns 0, or -3 on allocation failure.
 */
int orc_relabel_degree(int64_t n, const int64_t *row_ptr, const int32_t *col, int64_t *out_rp, int32_t *out_col,
                       int32_t *perm)
{
    int64_t *deg = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *inv = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!deg || !inv) { free(deg); free(inv); return -3; }
    for (int64_t v = 0; v < n; ++v) { deg[v] = row_ptr[v + 1] - row_ptr[v]; perm[v] = (int32_t)v; }
    g_rl_deg = deg;
    qsort(perm, (size_t)n, sizeof(int32_t), cmp_deg_desc);
    for (int64_t i = 0; i < n; ++i) inv[perm[i]] = (int32_t)i;
    out_rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = perm[i], o = out_rp[i];
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) out_col[o + e - row_ptr[v]] = inv[col[e]];
        qsort(out_col + o, (size_t)deg[v], sizeof(int32_t), cmp_i32);
        out_rp[i + 1] = o + deg[v];
    }
    free(deg);
    free(inv);
    return 0;
}
