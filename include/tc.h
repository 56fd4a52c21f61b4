/*
 * tc.h -- C ABI of the MI355X (gfx950) triangle-counting library.
 *
 * The library computes the cover-edge + forward + hashing triangle count of
 * Bader, "Fast Triangle Counting" (arXiv 2309.09064, Algorithm 4):
 *   1. BFS levels L(v), each component searched from its smallest vertex id
 *      (Algorithm 4, first loop);
 *   2. the partition of E into horizontal edges E0 (L(u) = L(v)) and the
 *      level-spanning rest E1 (Algorithm 4, partition loop);
 *   3. T0 = triangles inside G0 = (V, E0), counted forward-style over the
 *      rank-oriented lists N0+ (Algorithm 2);
 *   4. T1 = for each horizontal edge {u, v}, |N1(u) & N1(v)| (Algorithm 4,
 *      hashed loop), each intersection hashing the larger list and streaming
 *      the smaller one (Section II, cost min(d(u), d(v)));
 *   T = T0 + T1.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Graph: simple undirected graph in CSR, both directions stored, rows
 *    sorted ascending, no self-loops or duplicates.  row_ptr is int32[n+1]
 *    with row_ptr[0] = 0 and row_ptr[n] = nnz; col_idx is int32[nnz].
 *    nnz < 2^31.  The input is read-only (Section III, experimental rules).
 *  - Pointers named d_* are DEVICE pointers (HIP device memory of the
 *    current device); pointers named h_* or of struct type are HOST pointers.
 *    The caller owns every buffer.
 *  - Scratch memory comes only from the caller's workspace (ws, ws_bytes);
 *    query its size with the matching *_ws function.  Entry points allocate
 *    no device memory, so every auxiliary structure is released when the
 *    caller frees the workspace.  ws must be 256-byte aligned.  The one
 *    library-held buffer is a 4 KB pinned host mailbox per calling thread,
 *    created on the thread's first call, reused by all its later calls (no
 *    allocation per call) and released by tc_thread_release().
 *  - stream: a hipStream_t passed as void*; NULL means the default stream.
 *    Work is enqueued on that stream.  Entry points that return a host value
 *    (nnz, a count) synchronise that stream before returning.
 *  - Errors: functions returning int return TC_OK (0) or a negative tc_err
 *    code.  tc_count returns TC_COUNT_ERROR (UINT64_MAX) on failure; this is
 *    unambiguous because a graph with nnz < 2^31 has fewer than 2^47
 *    triangles.  tc_last_error() returns the calling thread's last code and
 *    tc_strerror() its text.  Arguments are validated on the host before any
 *    device work; with TC_VALIDATE the CSR itself is checked on the device.
 */
#ifndef TC_H
#define TC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
enum tc_err {
    TC_OK = 0,
    TC_ERR_ARG = -1,        /* NULL pointer, negative size, bad option      */
    TC_ERR_RANGE = -2,      /* a vertex id outside [0, n)                    */
    TC_ERR_OVERFLOW = -3,   /* nnz or a size does not fit int32 CSR          */
    TC_ERR_CAPACITY = -4,   /* output buffer too small                       */
    TC_ERR_WORKSPACE = -5,  /* workspace missing, too small or misaligned    */
    TC_ERR_HIP = -6,        /* a HIP runtime call failed                     */
    TC_ERR_NO_DEVICE = -7,  /* no gfx950 device visible                      */
    TC_ERR_INVALID_CSR = -8, /* TC_VALIDATE found a malformed CSR / levels   */
    TC_ERR_TOO_LARGE = -9   /* graph beyond tc_count_noalloc's fixed scratch */
};

#define TC_COUNT_ERROR UINT64_MAX

/* ------------------------------------------------------------ options */

/* Intersection strategies a bucket of work can be given (all exact). */
enum tc_strategy {
    TC_STRAT_AUTO = -1,       /* use the schedule (heuristic or network)     */
    TC_STRAT_WAVE_HASH = 0,   /* owner list in a wavefront-private LDS hash   */
    TC_STRAT_WG_HASH = 1,     /* owner list in a workgroup-shared LDS hash    */
    TC_STRAT_BSEARCH = 2,     /* binary search in the owner's global list     */
    TC_STRAT_MERGE = 3,       /* two-pointer merge of the two sorted lists:
                                 one lane per item for owner lists below
                                 32, else the wavefront per partner          */
    TC_NUM_STRATEGIES = 4
};

/* Orientation of the horizontal edges for the forward count inside G0
 * (Algorithm 2 as Algorithm 4 applies it): which endpoint's N0+ list holds
 * an edge.  T, T0 and T1 do not depend on it; the lengths of the N0+ lists,
 * and so the kind-0 work, do. */
enum tc_orientation {
    TC_ORIENT_RANK = 0,       /* y in N0+(x) when rank(y) > rank(x),
                                 rank(v) = (deg(v), v) lexicographic: the
                                 degree-ordered forward algorithm (default)  */
    TC_ORIENT_ID = 1          /* y in N0+(x) when y > x, ids as stored: the
                                 u < v form of Algorithms 2 and 4            */
};

enum tc_schedule {
    TC_SCHED_HEURISTIC = 0,   /* owner-list-size thresholds                  */
    TC_SCHED_TABLE = 1        /* one strategy per bucket from
                                 opt->sched_table, e.g. the choice of the
                                 learned cost network (tc_mlp_schedule)      */
};

/*
 * Buckets.  The counting work is split into units (owner x, kind): kind 0
 * intersects N0+ lists (T0), kind 1 intersects N1 lists (T1); the owner of a
 * horizontal edge is the endpoint with the larger list.  A unit falls in
 * bucket  b = (kind * 32 + ob) * 32 + pb  where ob = floor(log2 |owner list|)
 * and pb = floor(log2 (mean size of the partner lists streamed against it)),
 * both capped at 31.  Schedules assign one strategy per bucket.
 */
#define TC_NUM_BUCKETS 2048

enum tc_flags {
    TC_VALIDATE = 1,          /* check CSR (sorted, symmetric-free checks,
                                 ranges) and levels on the device            */
    TC_TIMING = 2             /* fill the phase times of tc_stats            */
};

typedef struct tc_options {
    int32_t schedule;         /* tc_schedule                                 */
    int32_t force_strategy;   /* tc_strategy; >= 0 forces it on every bucket.
                                 A wavefront hash whose table cannot hold a
                                 bucket's owner lists becomes the workgroup
                                 hash, which cuts an owner list longer than
                                 half its table into value-range slices
                                 (one work item each)                        */
    int32_t flags;            /* tc_flags bits                               */
    int32_t wave_slots;       /* LDS hash slots per wavefront (power of 2,
                                 64..2048); 0 = default 2048                 */
    int32_t wg_slots;         /* LDS hash slots per workgroup (power of 2,
                                 1024..32768); 0 = default 32768             */
    int32_t chunk_work;       /* target probe elements per work item;
                                 0 = by input size: 16384 below 2^23
                                 entries, 32768 below 2^24, else 65536     */
    int32_t grid_blocks;      /* persistent grid size; 0 = as many 1024-thread
                                 blocks as fit in LDS, at most 2 per CU      */
    int32_t wave_max_owner;   /* heuristic: largest owner list for the
                                 wavefront hash; 0 = wave_slots / 2          */
    int32_t merge_max_owner;  /* heuristic: owner lists up to this size (at
                                 most 31) take the lane merge (one lane per
                                 item of at most 32 partners); 0 = default:
                                 31 for plain and batched counts with
                                 2048-slot wavefront tables, else 15;
                                 -1 = never                                  */
    const int32_t *sched_table; /* device int32[TC_NUM_BUCKETS], read when
                                 schedule == TC_SCHED_TABLE (NULL otherwise):
                                 bits 0-1 the bucket's strategy, bit 2 (with
                                 TC_STRAT_WG_HASH) owner slices of half the
                                 usual size; other values mean binary
                                 search.  A hash strategy in a bucket whose
                                 owners exceed that table's capacity is
                                 replaced as with force_strategy, and the
                                 half-slice bit is dropped where it changes
                                 nothing (owners shorter than half a slice). */
    int64_t batch_group_entries; /* batched counts: most vertices and most
                                 CSR entries one internal group of graphs
                                 may hold (a larger graph gets a group of
                                 its own); 0 = 2^31 - 1024, the int32 limit  */
    int32_t wg_slice_max;     /* workgroup hash: longest owner list held whole
                                 in one table (power of 2, 64..wg_slots/2);
                                 longer lists are cut into value-range slices
                                 of at most this many; 0 = wg_slots / 4      */
    int32_t orientation;      /* tc_orientation of the N0+ lists; 0 = rank   */
} tc_options;

/* Per-call statistics (host struct, all optional). */
typedef struct tc_stats {
    uint64_t T0;              /* triangles inside G0                          */
    uint64_t T1;              /* triangles with exactly one horizontal edge   */
    int64_t e0;               /* undirected horizontal edges |E0|             */
    int64_t units;            /* (owner, kind) work units                     */
    int64_t items;            /* work items after chunking                    */
    int64_t probes;           /* probe elements streamed (sum of the smaller
                                 list over all live intersections)           */
    int64_t hashed;           /* owner-list elements hashed or searched       */
    int32_t levels;           /* number of BFS levels (max level + 1)         */
    int32_t bfs_rounds;       /* BFS level steps executed                     */
    float ms_bfs;             /* phase times (TC_TIMING), milliseconds        */
    float ms_partition;
    float ms_bucket;
    float ms_isect;
    int32_t strategy_items[TC_NUM_STRATEGIES]; /* items run per strategy     */
} tc_stats;

/* ------------------------------------------------------------ error query */

int tc_last_error(void);
const char *tc_strerror(int code);

/* Library version (major * 10000 + minor * 100 + patch). */
int tc_version(void);

/* Releases the calling thread's pinned 4 KB result mailbox (see the
 * conventions above); the thread's next call creates it again.  Call it
 * before a worker thread ends, or before process exit to leave nothing
 * allocated.  No call of this thread may be in flight.  Returns TC_OK or
 * TC_ERR_HIP. */
int tc_thread_release(void);

/* ------------------------------------------------------------ CSR build */

/*
 * Workspace bytes for tc_build_csr with n vertices and m_tuples tuples.
 */
int tc_build_csr_ws(int32_t n, int64_t m_tuples, size_t *h_ws_bytes);

/*
 * Simple undirected CSR from raw edge tuples (the paper's input format,
 * Introduction): drops self-loops, stores each tuple in both directions,
 * removes duplicates and sorts every row.
 *   d_src, d_dst  int32[m_tuples] device, ids in [0, n)
 *   d_row_ptr     int32[n+1] device, output
 *   d_col_idx     int32[col_cap] device, output (first nnz entries)
 *   h_nnz         host, receives nnz
 * Errors: TC_ERR_RANGE (an id outside [0, n)), TC_ERR_OVERFLOW (2 * m_tuples
 * >= 2^31), TC_ERR_CAPACITY (nnz > col_cap; *h_nnz still receives nnz).
 * Synchronises the stream.
 */
int tc_build_csr(int32_t n, int64_t m_tuples, const int32_t *d_src, const int32_t *d_dst,
                 int32_t *d_row_ptr, int32_t *d_col_idx, int64_t col_cap, int64_t *h_nnz,
                 void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ BFS levels */

int tc_bfs_levels_ws(int32_t n, int64_t nnz, size_t *h_ws_bytes);

/*
 * BFS levels with the paper's serial semantics (Algorithm 4, first loop):
 * every component is searched from its smallest vertex id, which gets level
 * 0; L(v) is the hop distance from that root.  The result is unique.
 *   d_levels   int32[n] device, output
 *   h_levels_count  host, optional (NULL ok): max level + 1
 * Computed as connected components by minimum-id linking, then a
 * multi-source direction-optimising BFS from all roots.  Synchronises.
 */
int tc_bfs_levels(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                  int32_t *d_levels, int32_t *h_levels_count, void *ws, size_t ws_bytes,
                  void *stream);

/* ------------------------------------------------------------ count */

int tc_count_ws(int32_t n, int64_t nnz, const tc_options *opt, size_t *h_ws_bytes);

/*
 * Triangle count T = T0 + T1 (Algorithm 4).
 *   d_levels   int32[n] device or NULL.  NULL: computed as by tc_bfs_levels
 *              (charged to this call).  Non-NULL: any levels with
 *              |L(u) - L(v)| <= 1 on every edge give the same T (the
 *              cover-edge argument behind Algorithm 3); the paper notes the
 *              method pays off when BFS results already exist.
 *   opt        host, NULL = defaults (heuristic schedule)
 *   stats      host, NULL ok
 * Returns T, or TC_COUNT_ERROR (see tc_last_error).  Synchronises.
 */
uint64_t tc_count(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                  const int32_t *d_levels, const tc_options *opt, tc_stats *stats, void *ws,
                  size_t ws_bytes, void *stream);

/*
 * Many graphs in one call (the batched configuration: many graphs of uneven
 * size, each counted as by tc_count on its own).  Every graph g is its own
 * simple CSR with LOCAL int32 ids, packed one after another:
 *   h_vtx_off   host int64[graphs + 1]: 0 = off[0] <= ... ; graph g has
 *               n_g = h_vtx_off[g+1] - h_vtx_off[g] vertices
 *   h_edge_off  host int64[graphs + 1]: 0 = off[0] <= ... ; graph g has
 *               nnz_g = h_edge_off[g+1] - h_edge_off[g] CSR entries
 *   d_row_ptr   device int32[h_vtx_off[graphs] + graphs]: graph g's n_g + 1
 *               row pointers start at d_row_ptr[h_vtx_off[g] + g], run from
 *               0 to nnz_g, and index its own entries
 *   d_col_idx   device int32[h_edge_off[graphs]]: graph g's entries at
 *               d_col_idx[h_edge_off[g] ...], ids in [0, n_g)
 *   d_levels    device int32 per packed vertex (h_vtx_off[graphs]), or NULL:
 *               computed per graph as by tc_bfs_levels
 *   d_counts    device uint64[graphs], output: triangles of each graph
 * Each graph must fit int32 CSR (n_g and nnz_g below 2^31 - 1024); the batch
 * as a whole need not: it is processed in groups of consecutive graphs whose
 * union fits (opt->batch_group_entries).  Per group, one pass: ids rebased to
 * the group (an id outside its graph is clamped into it; TC_VALIDATE reports
 * it), BFS levels with one workgroup per graph, the partition, and one
 * persistent intersection launch that drains the work of all the group's
 * graphs, each hit added to its graph's count.  A component never spans two
 * graphs, so each graph's levels, T0 and T1 are those it has alone.  The
 * workspace (tc_count_batched_ws, which needs the offsets) holds a rebased
 * copy of the largest group's CSR besides tc_count's buffers.
 * Returns the total over all graphs, or TC_COUNT_ERROR: TC_ERR_ARG for bad
 * offsets, TC_ERR_OVERFLOW for a graph beyond int32, and with TC_VALIDATE
 * TC_ERR_INVALID_CSR for malformed rows or ids.  stats, when given, sums the
 * groups (levels: the largest level count of any graph).  Synchronises.
 */
int tc_count_batched_ws(int32_t graphs, const int64_t *h_vtx_off, const int64_t *h_edge_off, const tc_options *opt,
                        size_t *h_ws_bytes);
uint64_t tc_count_batched(int32_t graphs, const int64_t *h_vtx_off, const int64_t *h_edge_off,
                          const int32_t *d_row_ptr, const int32_t *d_col_idx, const int32_t *d_levels,
                          const tc_options *opt, uint64_t *d_counts, tc_stats *stats, void *ws, size_t ws_bytes,
                          void *stream);

/*
 * BFS levels of every graph of a packed batch (layout and workspace as for
 * tc_count_batched), each graph as by tc_bfs_levels on its own: every
 * component searched from its smallest local id (Algorithm 4, first loop).
 * One workgroup per graph, largest graphs first.
 *   d_levels        device int32[h_vtx_off[graphs]], output (packed like the
 *                   vertices)
 *   h_levels_count  host, optional: the largest level count of any graph
 * Local ids must lie within their graph (not checked here; an id outside is
 * clamped into it).  Synchronises.
 */
int tc_bfs_levels_batched(int32_t graphs, const int64_t *h_vtx_off, const int64_t *h_edge_off,
                          const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t *d_levels,
                          int32_t *h_levels_count, void *ws, size_t ws_bytes, void *stream);

/*
 * The same batch as one captured graph of device work, replayed at will:
 * tc_batch_plan_create enqueues nothing on its own but records the whole
 * pipeline of tc_count_batched (levels computed, no host read anywhere in
 * it) into a HIP graph bound to the given buffers; tc_batch_plan_launch
 * replays it on `stream`, asynchronously, and leaves the per-graph counts in
 * d_counts when the stream reaches that point.  The buffers (row_ptr,
 * col_idx, d_counts, ws) must stay allocated and unchanged in size while the
 * plan lives; their contents may change between launches (same offsets).
 * Launches of one plan must not overlap.  The plan object is host memory
 * owned by the caller through tc_batch_plan_destroy.  Options as for
 * tc_count_batched except TC_TIMING and TC_VALIDATE (TC_ERR_ARG: both read
 * results on the host).  Workspace: tc_count_batched_ws.  create
 * synchronises `stream` (it uploads the offsets); launch must run on the
 * device that was current at create (TC_ERR_ARG otherwise).
 */
typedef struct tc_batch_plan tc_batch_plan;
int tc_batch_plan_create(int32_t graphs, const int64_t *h_vtx_off, const int64_t *h_edge_off,
                         const int32_t *d_row_ptr, const int32_t *d_col_idx, const tc_options *opt,
                         uint64_t *d_counts, void *ws, size_t ws_bytes, void *stream, tc_batch_plan **h_plan);
int tc_batch_plan_launch(tc_batch_plan *plan, void *stream);
int tc_batch_plan_destroy(tc_batch_plan *plan);

/*
 * The strategy every bucket gets from tc_count under opt for a graph of n
 * vertices and nnz CSR entries: force_strategy, the table or the heuristic,
 * after the feasibility rules, with bit 2 set where a table's half-size
 * workgroup slices apply (see tc_options.sched_table).  d_table: device
 * int32[TC_NUM_BUCKETS].
 */
int tc_schedule_table(int32_t n, int64_t nnz, const tc_options *opt, int32_t *d_table, void *stream);

/*
 * tc_count plus a per-bucket cost profile, the training data of the learned
 * schedule (not part of the paper: it only chooses among exact kernels).
 * Uses the same workspace size as tc_count.  ADDS into
 *   d_prof  uint64[TC_NUM_BUCKETS * TC_NUM_STRATEGIES * 3] device; for
 *           bucket b and strategy s, at ((b * 4) + s) * 3:
 *             [0] wavefront-ticks: elapsed ticks of the device's constant
 *                 clock per work item, times the wavefronts the item holds
 *                 (16 for TC_STRAT_WG_HASH, else 1), summed over items;
 *             [1] elements: partner-list elements streamed plus owner-list
 *                 elements, summed over the bucket's units (the same for
 *                 every strategy);
 *             [2] work items run.
 * so several calls (graphs, forced strategies) accumulate into one profile;
 * the caller zeroes it first.  Returns T like tc_count; the instrumented
 * kernel is slower than tc_count's.
 */
uint64_t tc_count_profile(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                          const int32_t *d_levels, const tc_options *opt, tc_stats *stats,
                          uint64_t *d_prof, void *ws, size_t ws_bytes, void *stream);

/*
 * Per-vertex triangle counts t(v): the number of triangles containing v, the
 * input of the local clustering coefficient (the applications named in the
 * paper's Introduction).  Each triangle is found exactly once by Algorithm
 * 4, through its one cover edge xy and common neighbour w, and adds 1 to
 * t(x), t(y) and t(w), so sum_v t(v) = 3T.
 *   d_tv   device uint64[n], output, written in full (zeroed by the call)
 * Other arguments, the workspace size (tc_count_ws) and the return value as
 * for tc_count; opt->schedule, force_strategy and the tile options apply
 * (the hash tables keep a hit counter beside each key, so wave_slots and
 * wg_slots are capped at 1024 and 16384 here).  Hits are gathered in LDS
 * counters and added to global memory with 64-bit atomics.  Synchronises.
 */
uint64_t tc_vertex_triangles(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                             const int32_t *d_levels, const tc_options *opt, uint64_t *d_tv, tc_stats *stats,
                             void *ws, size_t ws_bytes, void *stream);

/*
 * Per-edge triangle counts (support): for every input entry e = (u, v),
 * d_sup[e] = the number of triangles containing the edge {u, v}, the same at
 * both entries of an edge (the k-truss input; applications named in the
 * paper's Introduction).  Each triangle, found once by Algorithm 4, adds 1 to
 * its three edges, so the entries sum to 6T.
 *   d_sup  device uint32[nnz], output, written in full (zeroed by the call);
 *          indexed like d_col_idx
 * The workspace is larger than tc_count's (two int32 maps of nnz entries from
 * the partitioned lists back to input entries): size it with
 * tc_edge_support_ws.  The hash tables keep a hit counter beside each key,
 * so wave_slots and wg_slots are capped at 1024 and 16384 here.
 * The rows must be symmetric (every (u, v) has its (v, u)); TC_VALIDATE
 * checks this.  Returns T or TC_COUNT_ERROR.  Synchronises.
 */
int tc_edge_support_ws(int32_t n, int64_t nnz, const tc_options *opt, size_t *h_ws_bytes);
uint64_t tc_edge_support(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                         const int32_t *d_levels, const tc_options *opt, uint32_t *d_sup, tc_stats *stats,
                         void *ws, size_t ws_bytes, void *stream);

/*
 * Cover-edge count (Algorithm 3, CE; after tc_relabel_degree, CED): for every
 * horizontal edge uv, u < v, every common neighbour w of the full rows N(u)
 * and N(v) counts when L(w) != L(u), or L(w) = L(u) and w > v.  The same
 * kernels as tc_count, run over full rows instead of the N0+ / N1 split: the
 * single-pass form of the method that Algorithm 4 refines.  Arguments,
 * workspace (tc_count_ws) and return value as for tc_count; stats->T0 is 0
 * and stats->T1 = T.  Synchronises.
 */
uint64_t tc_count_cover_edge(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                             const int32_t *d_levels, const tc_options *opt, tc_stats *stats, void *ws,
                             size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ degree relabel */

/*
 * Degree ordering of the vertices (Section III, last paragraph; the BaderD
 * and CED variants of the experiments): new id i is the vertex with the i-th
 * largest degree, ties by increasing old id.  Writes the relabelled CSR
 * (sorted rows) and the permutation.
 *   d_out_row_ptr  int32[n+1] device, output
 *   d_out_col_idx  int32[nnz] device, output (must not alias d_col_idx)
 *   d_perm         int32[n] device, output: d_perm[new id] = old id
 * Needs tc_relabel_degree_ws bytes of workspace.  Asynchronous on `stream`
 * (argument errors are reported before any work is queued).  T is unchanged
 * by a relabel; BFS roots, levels and the horizontal share k are not.
 */
int tc_relabel_degree_ws(int32_t n, int64_t nnz, size_t *h_ws_bytes);
int tc_relabel_degree(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                      int32_t *d_out_row_ptr, int32_t *d_out_col_idx, int32_t *d_perm, void *ws, size_t ws_bytes,
                      void *stream);

/* ------------------------------------------------------------ cost network
 *
 * A small fully connected network predicts, for a bucket, the cost of each
 * strategy (log2 of wavefront-ticks per element); the learned schedule takes
 * the cheapest feasible one.  The network is not in the paper: it only picks
 * which exact kernel counts a bucket, so it never changes a count.
 *
 *   a1 = relu(W1 x + b1),  a2 = relu(W2 a1 + b2),  y = W3 a2 + b3
 *   x = (ob, pb, kind) of a bucket, as floats; y[k] = predicted cost of
 *   strategy k (k < K; the schedule uses K = TC_NUM_STRATEGIES).
 *
 * Parameters: device float32, row-major, in the order W1[H][3], b1[H],
 * W2[H][H], b2[H], W3[K][H], b3[K]; tc_mlp_param_count gives their number.
 * Supported sizes: H in {8, 16, 32, 64}, 1 <= K <= 8.  A training row is
 * (x[3], c, t, w): features, the strategy measured, its measured cost, a
 * weight w >= 0 (all 1 when d_w is NULL); the loss of R rows is
 * sum w * 0.5 * (y[c] - t)^2 / sum w, minimised by Adam.
 */
#define TC_MLP_IN 3

int tc_mlp_param_count(int32_t hidden, int32_t k, int64_t *h_count);

/* He-uniform weights, zero biases: W[i][j] = (2u - 1) * sqrt(6 / fan_in)
 * with u = (SplitMix64(seed + index) >> 40) * 2^-24, index = the weight's
 * position in the flat parameter array.  Deterministic. */
int tc_mlp_init(float *d_params, int32_t hidden, int32_t k, uint64_t seed, void *stream);

/* y[r][k] for rows r < rows; d_x float[rows][3], d_y float[rows][K]. */
int tc_mlp_forward(const float *d_params, int32_t hidden, int32_t k, const float *d_x, int32_t rows,
                   float *d_y, void *stream);

/* Loss and gradient over rows r < rows: d_c int32[rows] in [0, K) (a row
 * with another index contributes nothing but still counts in sum w), d_t
 * float[rows], d_w float[rows] or NULL; the sum of the weights must be
 * positive.  d_grad float[param_count] (same layout as the parameters),
 * d_loss float[1] (NULL ok).  The sums over rows run in a fixed order in
 * float64, so the result is deterministic.  rows >= 1. */
int tc_mlp_grad_ws(int32_t hidden, int32_t k, int32_t rows, size_t *h_ws_bytes);
int tc_mlp_grad(const float *d_params, int32_t hidden, int32_t k, const float *d_x, const int32_t *d_c,
                const float *d_t, const float *d_w, int32_t rows, float *d_grad, float *d_loss, void *ws,
                size_t ws_bytes, void *stream);

/* One Adam step (Kingma and Ba, with bias correction) on count parameters:
 * m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 * p -= lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * step >= 1.  d_m and d_v start at zero. */
int tc_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int64_t count, int32_t step,
                float lr, float beta1, float beta2, float eps, void *stream);

/* steps Adam steps on the full batch (gradient, then update), numbered
 * first_step, first_step + 1, ...; d_loss float[steps] receives each step's
 * loss before its update (NULL ok).  Workspace: tc_mlp_grad_ws plus the
 * gradient, i.e. tc_mlp_train_ws. */
int tc_mlp_train_ws(int32_t hidden, int32_t k, int32_t rows, size_t *h_ws_bytes);
int tc_mlp_train(float *d_params, float *d_m, float *d_v, int32_t hidden, int32_t k, const float *d_x,
                 const int32_t *d_c, const float *d_t, const float *d_w, int32_t rows, int32_t first_step,
                 int32_t steps, float lr, float beta1, float beta2, float eps, float *d_loss, void *ws,
                 size_t ws_bytes, void *stream);

/* The learned schedule: for every bucket b, the strategy with the smallest
 * predicted cost among those feasible under opt (the wavefront hash is
 * feasible when ob <= log2(wave_slots) - 2, i.e. the owner list fills at most
 * half its table; the workgroup hash, binary search and merge always are).
 * Ties go to the lower strategy number.  K must be TC_NUM_STRATEGIES.
 *   d_table  int32[TC_NUM_BUCKETS] device, output (for opt->sched_table)
 *   d_cost   float[TC_NUM_BUCKETS][K] device, predicted costs, NULL ok */
int tc_mlp_schedule(const float *d_params, int32_t hidden, int32_t k, const tc_options *opt, int32_t *d_table,
                    float *d_cost, void *stream);

/*
 * The two CSRs of the partition (Algorithm 4, partition loop), for tests and
 * for callers that reuse them.  d_levels: int32[n] device, levels that differ
 * by at most one on every edge (BFS levels do; TC_VALIDATE on tc_count checks
 * it).  orientation: a tc_orientation (else TC_ERR_ARG).  Outputs (device,
 * caller-owned):
 *   d_rp0  int32[n+1], d_c0 int32[nnz]: N0(x) per row = the neighbours of
 *          equal level above x in the orientation (TC_ORIENT_RANK: rank
 *          above, rank(y) = (deg(y), y) lexicographic; TC_ORIENT_ID: id
 *          above), ascending, then the rest, ascending.
 *   d_up0  int32[n]: size of the upper part (N0+) of each N0 row.
 *   d_rp1  int32[n+1], d_c1 int32[nnz]: N1(x) = neighbours of other level,
 *          ascending.
 *   h_e0   host: |E0| (undirected).
 * Synchronises.
 */
int tc_partition_ws(int32_t n, int64_t nnz, size_t *h_ws_bytes);
int tc_partition(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                 const int32_t *d_levels, int32_t orientation, int32_t *d_rp0, int32_t *d_c0, int32_t *d_up0,
                 int32_t *d_rp1, int32_t *d_c1, int64_t *h_e0, void *ws, size_t ws_bytes,
                 void *stream);

/* ------------------------------------------------------------ no allocation */

/*
 * tc_count for callers that cannot allocate: code under graph capture, tight
 * serving loops, harnesses that forbid allocation.  It allocates nothing and
 * takes no workspace: its scratch is a fixed device array of 256 MiB that
 * the library holds on every GPU it runs on until the process ends.  Graphs
 * whose tc_count workspace (tc_count_ws) exceeds 256 MiB -- a Kronecker
 * graph of scale 18 fits, one of scale 19 does not -- are rejected with
 * TC_ERR_TOO_LARGE
 * before any device work.  Levels, when not given, come from a BFS run by a
 * single workgroup (the component loop of tc_bfs_levels, with no host read),
 * so the call is asynchronous and reads nothing back:
 *   d_result   device uint64[4], output: {T, T0, T1, |E0|} when the stream
 *              reaches the end of the call's work
 * Other arguments as for tc_count; TC_TIMING and TC_VALIDATE are rejected
 * (TC_ERR_ARG: both read results on the host).  Every call on a GPU shares
 * that GPU's scratch array: calls that overlap on one GPU (other streams,
 * other host threads) race and must be ordered by the caller.  The scratch
 * keeps the last call's contents; every buffer that must start at zero is
 * cleared by the call's own kernels.
 */
int tc_count_noalloc(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                     const int32_t *d_levels, const tc_options *opt, uint64_t *d_result, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
