/*
 * appd.h -- C ABI of libappd: the all-points minimax path distance (APPD) of an
 * undirected dense graph on AMD Instinct MI355X (gfx950).
 *
 * Method: arXiv 2407.07058, Algorithm 4 ("MMJ distance by Calculation and
 * Copy"), Section 3.  M(i,j) is the smallest possible largest edge weight over
 * all paths from i to j (Section 1, Eq. 1-2); it is read off a minimum spanning
 * tree, because a tree path of a minimum spanning tree is a minimax path
 * (Section 2.1, Section 5).  The widest-path variant (Section 1, Section 4.2)
 * reverses every weight comparison (maximum spanning tree).
 *
 * Conventions shared by every call below.
 *  - W, M, idx are n x n row-major on the device, caller-owned.  W is float32,
 *    bit-symmetric, zero diagonal, NaN-free; +-inf and negative weights are
 *    ordinary weights.  A violated precondition gives unspecified (but
 *    deterministic) output, never an out-of-bounds access.
 *  - Edge total order: e < f iff w(e) < w(f), or w(e) == w(f) and
 *    flat(e) < flat(f), flat(u,v) = min(u,v)*n + max(u,v) (float comparison:
 *    -0.0 == +0.0).  The paper notes equal weights do not change M (Section 5);
 *    this order fixes which edge is reported.  Widest mode: larger weight first,
 *    equal weights by smaller flat index.
 *  - M(i,j) = weight of the bottleneck edge of the pair (float32, -0.0 reported
 *    as +0.0); M(i,i) = +0.0.
 *    idx(i,j) = flat index of that edge (int32); idx(i,i) = -1.
 *    1 <= n <= APPD_MAX_N so that every flat index fits in int32.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Every call only
 *    enqueues work on it and returns; nothing synchronises the host.  The
 *    return value reports argument errors and launch errors; a fault raised
 *    while the kernels run surfaces at the caller's next synchronisation.
 *  - Workspace: calls that take (ws, ws_bytes) use that device buffer (>= the
 *    size the matching *_workspace_bytes call returns, 256-byte aligned) and
 *    allocate nothing; calls without it allocate and free stream-ordered
 *    (hipMallocAsync / hipFreeAsync) on `stream`.
 *  - Return codes: APPD_OK, or a negative APPD_E* code; appd_error_string()
 *    names it and appd_get_last_error() returns the last code any call on this
 *    host thread produced.  No C++ exception crosses this interface.
 */
#ifndef APPD_H
#define APPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define APPD_MAX_N 46340

enum appd_status {
    APPD_OK = 0,
    APPD_EINVAL = -1, /* null pointer, n out of range, workspace too small, bad mode */
    APPD_EHIP = -2,   /* a HIP runtime call or kernel launch failed */
    APPD_ENOMEM = -3, /* a stream-ordered allocation failed */
    APPD_EDATA = -4   /* reported by appd_sync: a forward run with APPD_VALIDATE set
                         read a W with a NaN entry or an asymmetric pair */
};

enum appd_mode {
    APPD_MINIMAX = 0, /* minimax path (Eq. 1-2) */
    APPD_WIDEST = 1   /* widest (maximum capacity) path, Section 4.2 */
};

/* Optional flags or-ed into `mode` of the single-graph calls: how the spanning
 * tree is found.  The tree is unique under the edge total order, so every choice
 * returns identical M, idx, order and parent. */
#define APPD_TREE_AUTO 0x00    /* by size */
#define APPD_TREE_PRIM 0x10    /* Prim's algorithm in one workgroup (Section 3) */
#define APPD_TREE_BORUVKA 0x20 /* Boruvka rounds over per-row candidate lists, then
                                  Prim's attachment order rebuilt from the tree */
/* Testing aid, with APPD_TREE_BORUVKA or APPD_TREE_AUTO: the Boruvka tree gets
 * a single pass over W, so that a graph it cannot finish from that pass's
 * candidate lists goes to the sequential Prim fallback (same results). */
#define APPD_TREE_ONE_PASS 0x40

const char* appd_error_string(int code);
int appd_get_last_error(void);

/*
 * Optional precondition check of W.  The method is defined on an undirected
 * graph with edge weights (Section 1: an undirected graph and its weights
 * e_w), so W must be symmetric; the calls here also ask for a NaN-free W with
 * a zero diagonal.  One pass over W (every element read once) or-s into
 * *flags (one uint32 in device memory, cleared by the call itself):
 *   APPD_VALID_NAN   some entry is NaN
 *   APPD_VALID_ASYM  some pair of non-NaN mirror entries differ (float compare:
 *                    -0.0 and +0.0 are equal weights)
 *   APPD_VALID_DIAG  some diagonal entry is not zero
 * 0 means every precondition holds.  Stream-ordered like every call: the flags
 * are valid once `stream` has reached them.  APPD_EINVAL for a null pointer or
 * n out of range.
 */
#define APPD_VALID_NAN 0x1u
#define APPD_VALID_ASYM 0x2u
#define APPD_VALID_DIAG 0x4u
int appd_validate(const float* W, int n, uint32_t* flags, void* stream);

/*
 * Waits for `stream` and reports what went wrong asynchronously on it, as the
 * return value and as appd_get_last_error() of the calling thread:
 *   APPD_EHIP   the stream reported a HIP error (a failed kernel), or a wait of
 *               the persistent batched forward gave up (its outputs are then
 *               incomplete);
 *   APPD_EDATA  a single-graph forward (appd_forward / _ws / _ex / _noalloc)
 *               enqueued while the environment variable APPD_VALIDATE was set
 *               (to anything but "0") read a W with a NaN entry or an
 *               asymmetric pair (the checks of appd_validate, enqueued before
 *               the forward's kernels; a non-zero diagonal is not an error,
 *               the forward never reads it).  The record is per GPU and is
 *               cleared by the call that reports it;
 *   APPD_OK     otherwise.
 * Not for use under stream capture (it synchronises).  Environment variable
 * APPD_LOG (anything but "0"): every kernel launch is written to stderr.
 */
int appd_sync(void* stream);

/* Bytes of device workspace appd_forward_ws / appd_forward_ex need for n
 * (0 if n is out of range). */
size_t appd_forward_workspace_bytes(int n);

/*
 * Single graph, minimax mode: M and idx of W (Algorithm 4, Section 3).
 * Allocates its O(n) workspace stream-ordered.
 */
int appd_forward(const float* W, int n, float* M, int32_t* idx, void* stream);

/* As appd_forward with a caller-provided workspace (no allocation). */
int appd_forward_ws(const float* W, int n, float* M, int32_t* idx, void* ws, size_t ws_bytes,
                    void* stream);

/*
 * As appd_forward_ws, with no allocation at all and no workspace argument: for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  The workspace is a
 * library-owned device array of APPD_NOALLOC_SCRATCH_BYTES per GPU, held by
 * each GPU the library runs on until the process ends; every n in
 * 1..APPD_MAX_N fits it (APPD_EINVAL otherwise, as for a null pointer).  Calls
 * on one GPU share that array: calls that overlap on one GPU (different
 * streams, or host threads without ordering between them) race, so order them.
 * The device address of the array is looked up on the first call on each
 * device (APPD_EHIP if that fails).  Results equal appd_forward_ws's.
 */
#define APPD_NOALLOC_SCRATCH_BYTES (12u << 20)
int appd_forward_noalloc(const float* W, int n, float* M, int32_t* idx, void* stream);

/*
 * Extended single-graph forward.
 *   mode      APPD_MINIMAX or APPD_WIDEST, optionally or-ed with one
 *             APPD_TREE_* flag.
 *   order     nullable, n int32: order[k] = k-th vertex attached by Prim's
 *             algorithm started at vertex 0 (the first step of Section 3).
 *   parent    nullable, n int32: the spanning-tree neighbour each vertex was
 *             attached through; parent[0] = -1.
 *   ws        nullable: NULL allocates stream-ordered, else >= the workspace
 *             size for n.
 */
int appd_forward_ex(const float* W, int n, int mode, float* M, int32_t* idx, int32_t* order,
                    int32_t* parent, void* ws, size_t ws_bytes, void* stream);

/*
 * The two phases of appd_forward_ex, exposed separately (e.g. to time them).
 * appd_tree: Prim's spanning tree of W from vertex 0 (Section 3, first step)
 *   and the attachment order, written into ws (internal layout; ws must
 *   be >= appd_forward_workspace_bytes(n)).  order / parent as in
 *   appd_forward_ex (nullable).
 * appd_fill: M and idx from the tree that appd_tree left in the same ws
 *   (the calculation-and-copy step of Section 3); same n and mode.
 */
int appd_tree(const float* W, int n, int mode, int32_t* order, int32_t* parent, void* ws,
              size_t ws_bytes, void* stream);

/* What the last spanning-tree run in ws did (for measurement): stats[0] = 1 if
 * the Boruvka path ran (else Prim's algorithm, and the rest are 0), stats[1] =
 * passes over W, stats[2] = Boruvka rounds, stats[3] = 1 if it fell back to
 * Prim, stats[4] = how many of the passes were component-table passes (those
 * read only the upper triangle of W).  stats holds 5 entries.  n and mode as
 * in that run.  Synchronises `stream`. */
int appd_tree_stats(int n, int mode, const void* ws, size_t ws_bytes, int32_t* stats,
                    void* stream);
int appd_fill(int n, int mode, const void* ws, size_t ws_bytes, float* M, int32_t* idx,
              void* stream);

/*
 * Single-linkage dendrogram of W from its spanning tree: the merge sequence of
 * the ascending construction Section 3 describes beside Algorithm 4 (tree edges
 * added best first to an empty forest), whose cophenetic distances are M.
 *   Z     (n-1) x 4 doubles, row-major, device: row i = {a, b, w, size}, the
 *         clusters joined by the i-th merge (a < b; ids below n are vertices,
 *         n + j is the cluster made by merge j), the weight of the joining
 *         edge and the number of vertices in the new cluster.  Merges follow
 *         the edge total order (minimax: ascending weight; widest: descending
 *         weight; equal weights by smaller flat index).  Nothing is written
 *         for n = 1 (Z may then be NULL).
 *   mode  APPD_MINIMAX or APPD_WIDEST, optionally with an APPD_TREE_* flag.
 *   ws    >= appd_forward_workspace_bytes(n) device bytes, 256-byte aligned.
 */
int appd_linkage(const float* W, int n, int mode, double* Z, void* ws, size_t ws_bytes,
                 void* stream);

/* ------------------------------------------------------------------ batches
 * Many independent graphs of uneven size, packed back to back in graph-id
 * order: graph g's W, M, idx (and G, dW) occupy n_g^2 elements starting at
 * element offset sum_{h<g} n_h^2; its O(n) arrays (parent, gradients per
 * vertex) start at sum_{h<g} n_h; its points X (n_g x d) at d * sum_{h<g} n_h.
 * Every graph needs 1 <= n_g <= APPD_BATCH_MAX_N.
 *
 * Graphs are grouped into size classes (n <= 64, 128, 256, 512, 1024, 2048)
 * and listed by decreasing n, so the longest Prim chains start first.  Each
 * class finds its spanning trees (class_tree[c]: Prim's algorithm with one
 * workgroup of class_threads[c] threads per graph, or Boruvka rounds over
 * candidate lists) and then runs the fill (work items of class_rows[c] rows); up to
 * `streams` classes proceed concurrently on library streams forked from and
 * joined back into `stream` (the largest class alone on `stream`, the others
 * in turn on the library streams; with split_count, the largest class's
 * biggest graphs alone on `stream` and the rest of it on the first library
 * stream, so that its smaller graphs' fill runs beside the longest Prim
 * chains).
 *
 * appd_batch_prepare plans the batch on the host (default schedule) and copies
 * the tables into ws with synchronous host-to-device copies; it must precede
 * the other batch calls and is not capturable in a HIP graph.
 * appd_batch_autotune times candidate schedules of appd_forward_batched on the
 * caller's batch and keeps the fastest in *plan (updating the device tables);
 * it synchronises and is not capturable either.  The calls that take a
 * prepared plan only launch kernels (and fork/join events) and can be
 * captured.  `plan` is plain host data.
 */
#define APPD_BATCH_MAX_N 2048
#define APPD_BATCH_CLASSES 6

typedef struct {
    int num_graphs;
    int max_n;
    int64_t total_n;  /* sum of n_g */
    int64_t total_nn; /* sum of n_g^2 */
    int class_first[APPD_BATCH_CLASSES];   /* first position of the class in n-descending order */
    int class_count[APPD_BATCH_CLASSES];   /* graphs in the class */
    int class_chunks[APPD_BATCH_CLASSES];  /* fill work items of the class */
    int class_rows[APPD_BATCH_CLASSES];    /* rows per fill work item */
    int class_threads[APPD_BATCH_CLASSES]; /* Prim workgroup size */
    int streams;      /* classes run concurrently on up to this many streams (1..6) */
    int pair_tiles;   /* work items of the point-to-graph kernel */
    int grad_chunks;  /* work items of the edge-gradient kernel */
    int chain_blocks; /* work items of the point-gradient kernel */
    size_t ws_bytes;  /* workspace the batch needs */
    int split_count;  /* with streams >= 2: the largest class's first split_count graphs
                         (its largest) run as a launch pair of their own on `stream`,
                         the rest of the class on a library stream; 0: one launch pair */
    int split_chunks; /* fill work items of those graphs (set with split_count) */
    uint64_t tables_key; /* stamp of the rows per item and cut the device work tables were
                            built for; a plan whose fields no longer match it is rejected */
    int class_tree[APPD_BATCH_CLASSES];     /* how the class's trees are found:
                                               APPD_BATCH_TREE_PRIM or APPD_BATCH_TREE_BORUVKA */
    int class_vertices[APPD_BATCH_CLASSES]; /* sum of n over the class's graphs */
    int split_vertices; /* sum of n over the graphs launched on their own (set with
                           split_count) */
    int persistent;     /* 1: the whole forward as one persistent launch over a work queue
                           (every class APPD_BATCH_TREE_BORUVKA, every n <= 1024); 0: one
                           launch sequence per class */
    int persist_items;  /* work items of that launch (set with persistent) */
    int stagger;        /* 1: with more than one stream, the other classes start after the
                           largest class's candidate-list pass (that class on Boruvka trees,
                           not cut), so the pass has the GPU to itself and the other
                           classes run beside its per-graph trees and fill; 0: all classes
                           start together */
} appd_batch_plan;

/* class_tree values.  Prim: one workgroup per graph runs Prim's algorithm
 * (n - 1 dependent steps).  Boruvka: a pass over the class's rows keeps each
 * row's 16 smallest entries, then one workgroup per graph runs Boruvka rounds
 * on them and rebuilds Prim's attachment order from the tree (refresh passes,
 * then Prim, for a graph the lists cannot finish).  Identical outputs. */
#define APPD_BATCH_TREE_PRIM 0
#define APPD_BATCH_TREE_BORUVKA 1

/* Workspace bytes for a batch with these sizes (0 on invalid input). */
size_t appd_batch_workspace_bytes(const int32_t* ns_host, int num_graphs);

/* Fill `plan` from the host sizes and upload the device tables into ws. */
int appd_batch_prepare(const int32_t* ns_host, int num_graphs, void* ws, size_t ws_bytes,
                       appd_batch_plan* plan, void* stream);

/* Times candidate schedules (Prim workgroup sizes, fill rows per item, class
 * concurrency) on this batch -- W, M, idx are the caller's packed device
 * buffers; M and idx are overwritten -- and stores the fastest in *plan.
 * best_ms (nullable) receives its time per forward. */
int appd_batch_autotune(const float* W, float* M, int32_t* idx, appd_batch_plan* plan, void* ws,
                        void* stream, float* best_ms);

/* Sets a schedule by hand (for experiments and tests): the plan's
 * class_threads, class_rows, class_tree and streams, and split_count (0: no
 * cut, -1: a cut into two parts of about equal work, else the number of the
 * largest class's biggest graphs launched on their own).  The device work
 * tables are rebuilt for it and the derived fields (class_chunks, split_count,
 * split_chunks, split_vertices, tables_key) set.  Checks the schedule (APPD_EINVAL if it is not
 * one the kernels support); synchronises and is not capturable. */
int appd_batch_set_schedule(appd_batch_plan* plan, void* ws, void* stream);

/* How the last batched forward found each graph's tree (for measurement), by
 * graph id into stats (num_graphs int32, host): -1 Prim's algorithm; else
 * rounds | passes << 8 | fallback << 16 of the Boruvka path (passes over the
 * graph's W; fallback 1 when Prim's algorithm had to finish it).  Synchronises
 * `stream`. */
int appd_batch_tree_stats(const appd_batch_plan* plan, const void* ws, int32_t* stats,
                          void* stream);

/* Batched forward (Algorithm 4 per graph).  parent: nullable, total_n int32. */
int appd_forward_batched(const float* W, int mode, float* M, int32_t* idx, int32_t* parent,
                         const appd_batch_plan* plan, void* ws, void* stream);

/* Complete graphs from packed point sets: W_ij = sqrt(sum_t (x_it - x_jt)^2),
 * summed in increasing t, each operation rounded once (bit-symmetric).
 * 1 <= d <= APPD_MAX_DIM. */
#define APPD_MAX_DIM 64
int appd_pairwise_euclidean_batched(const float* X, int d, float* W, const appd_batch_plan* plan,
                                    void* ws, void* stream);

/*
 * Backward of L = sum_{i != j} G_ij M_ij for point inputs, per graph:
 * dL/dw(e) = sum of G_ij over pairs whose bottleneck edge is e; then through
 * w = ||x_u - x_v||: dX_u += g (x_u - x_v)/w, dX_v -= g (x_u - x_v)/w.  W, idx and
 * parent are those of the forward; dX (total_n x d) is overwritten.  Float
 * atomics: the summation order, hence the last bits, vary between runs.
 */
int appd_backward_points_batched(const float* X, int d, const float* W, const float* G,
                                 const int32_t* idx, const int32_t* parent, float* dX,
                                 const appd_batch_plan* plan, void* ws, void* stream);

/*
 * Backward for packed weight-matrix inputs: per graph, dW[idx(i,j)] += G_ij for
 * i != j (the upper-triangle entry of each pair's bottleneck edge), as
 * appd_backward_w below.  G, idx and dW are packed like W; parent (total_n
 * int32) is the forward's.  dW is overwritten: zero except on tree edges.
 * Float atomics: the summation order, hence the last bits, vary between runs.
 */
int appd_backward_w_batched(const float* G, const int32_t* idx, const int32_t* parent, float* dW,
                            const appd_batch_plan* plan, void* ws, void* stream);

/* ------------------------------------------------------------------ single
 * Single-graph forms of the two calls above.  ws: >= appd_grad_workspace_bytes(n)
 * device bytes (256-byte aligned).  n <= APPD_GRAD_MAX_N for the backward. */
#define APPD_GRAD_MAX_N 32768
size_t appd_grad_workspace_bytes(int n);
int appd_pairwise_euclidean(const float* X, int n, int d, float* W, void* ws, size_t ws_bytes,
                            void* stream);
int appd_backward_points(const float* X, int n, int d, const float* W, const float* G,
                         const int32_t* idx, const int32_t* parent, float* dX, void* ws,
                         size_t ws_bytes, void* stream);

/* Backward for a weight-matrix input: dW[idx(i,j)] += G_ij for i != j, i.e. every
 * pair's gradient goes to the upper-triangle entry (u < v) of its bottleneck
 * edge.  dW (n x n) is overwritten (zero except on tree edges). */
int appd_backward_w(const float* G, const int32_t* idx, const int32_t* parent, int n, float* dW,
                    void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ timing
 * Launch timer for measurement.  appd_timer_start(kernel, capacity) creates
 * 2*capacity HIP events (the only allocation) and from then on brackets every
 * launch of the named kernel (its base name, e.g. "fill_kernel"; "*" = every
 * kernel) by two events recorded on the launch stream.  Launches beyond
 * `capacity` are not recorded and set the overflow flag.  kernel == NULL stops
 * the timer and destroys the events.  Not meant for code under HIP graph
 * capture.  One timer per process (calls are serialised by a mutex).
 * appd_timer_read waits for the recorded events of `kernel` and returns the
 * number of launches and the sum of their durations.  appd_timer_names writes
 * up to `capacity` distinct recorded kernel names (static strings) into
 * `names` (nullable) and returns how many there are.
 */
int appd_timer_start(const char* kernel, int capacity);
int appd_timer_read(const char* kernel, int* launches, double* total_ms, int* overflow);
int appd_timer_names(const char** names, int capacity);

/* ------------------------------------------------------------------ reference points
 * Measurement aids, not part of the method: the figures the kernels are
 * compared with, taken on the same GPU.
 * appd_membench_copy: dst = src, `bytes` (a multiple of 16, both 16-byte
 *   aligned) as a plain streaming copy (non-temporal 16-byte loads and stores,
 *   every CU busy).
 * appd_membench_write: `bytes` of dst set to the 32-bit `value`, store only.
 * appd_membench_chase: one lane follows p = next[p] from `start` for `steps`
 *   dependent loads (indices >= length are taken as 0, so any table stays in
 *   bounds) and writes the final p to *out: the time per step is the latency of
 *   a chain of dependent loads.
 * All device pointers, stream-ordered; APPD_EINVAL for null or misaligned
 * arguments. */
int appd_membench_copy(const void* src, void* dst, size_t bytes, void* stream);
int appd_membench_write(void* dst, size_t bytes, uint32_t value, void* stream);
int appd_membench_chase(const uint32_t* next, uint32_t length, uint32_t start, int steps,
                        uint32_t* out, void* stream);

/* ------------------------------------------------------------------ write-once check
 * Algorithm 4's calculation and copy (Section 3) assigns every entry of M once.
 * These run the forward (appd_forward_ex with ws and no order/parent outputs,
 * resp. appd_forward_batched with no parent output) with every store of an
 * output element counted: counts (device uint32, n*n resp. plan->total_nn, in
 * the layout of M) is cleared first, then each store adds 1 to the counter of
 * every element of M it writes and 0x10000 for idx, so an entry stored exactly
 * once reads 0x00010001 (the diagonal included).  M and idx are the forward's
 * outputs as usual.  For testing: the call synchronises `stream` before and
 * after the forward and is not capturable, and the counting switch is per GPU
 * and process, so no other forward may run on the GPU meanwhile (its stores
 * would be counted, or fault on the counter range).  Errors as the forward's;
 * APPD_EINVAL also for counts == NULL or (single) ws == NULL. */
int appd_debug_write_counts(const float* W, int n, int mode, float* M, int32_t* idx,
                            uint32_t* counts, void* ws, size_t ws_bytes, void* stream);
int appd_debug_write_counts_batched(const float* W, int mode, float* M, int32_t* idx,
                                    uint32_t* counts, const appd_batch_plan* plan, void* ws,
                                    void* stream);

#ifdef __cplusplus
}
#endif

#endif /* APPD_H */
