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
    APPD_ENOMEM = -3  /* a stream-ordered allocation failed */
};

enum appd_mode {
    APPD_MINIMAX = 0, /* minimax path (Eq. 1-2) */
    APPD_WIDEST = 1   /* widest (maximum capacity) path, Section 4.2 */
};

const char* appd_error_string(int code);
int appd_get_last_error(void);

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
 * Extended single-graph forward.
 *   mode      APPD_MINIMAX or APPD_WIDEST.
 *   order     nullable, n int32: order[k] = k-th vertex attached by Prim's
 *             algorithm started at vertex 0 (the first step of Section 3).
 *   parent    nullable, n int32: the spanning-tree neighbour each vertex was
 *             attached through; parent[0] = -1.
 *   ws        nullable: NULL allocates stream-ordered, else >= the workspace
 *             size for n.
 */
int appd_forward_ex(const float* W, int n, int mode, float* M, int32_t* idx, int32_t* order,
                    int32_t* parent, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* APPD_H */
