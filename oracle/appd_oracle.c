/*
 * appd_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately obvious CPU implementation of the all-points
 * minimax path distance (APPD) of an undirected dense graph, written from
 * "An efficient implementation for solving the all pairs minimax path problem
 * in an undirected dense graph" (Liu, arXiv 2407.07058).  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never does, and the two share no code.
 *
 * What is computed
 *   M(i,j) = min over paths p from i to j of the largest edge weight on p
 *   (Section 1, Eq. 1-2).  M(i,i) = +0.0.
 *   idx(i,j) = min(u,v)*n + max(u,v) for the bottleneck edge (u,v) of the pair:
 *   the largest edge, in the total order below, on the minimax path.
 *   idx(i,i) = -1.
 *
 * Edge total order (a reading: the paper says that equal weights "do not
 * matter" for M, Section 5, but they decide which edge is the bottleneck):
 *   edge e < edge f  iff  w(e) < w(f), or w(e) == w(f) and flat(e) < flat(f),
 *   flat(u,v) = min(u,v)*n + max(u,v).  Floating-point comparison, so -0.0 and
 *   +0.0 are equal weights; an output weight of -0.0 is reported as +0.0.
 *   Under this order every edge is distinct, so the minimum spanning tree and
 *   every bottleneck edge are unique.
 *
 * Functions (all weights row-major n x n, symmetric, zero diagonal, no NaN):
 *   oracle_appd_alg4      Algorithm 4 as Section 3 describes it: Prim's MST from
 *                         vertex 0, MST edges sorted in descending order, edges
 *                         removed from the largest down; each removal splits a
 *                         sub-tree into tree1 and tree2, both are traversed and
 *                         every pair across them gets the removed edge
 *                         (Section 3; correctness argument in Section 5).
 *   oracle_appd_alg4_rows The same procedure, writing only the requested rows
 *                         (for graphs whose full n x n output is too large).
 *   oracle_appd_fw        Minimax Floyd-Warshall over the total order: the
 *                         definition (Eq. 1-2) evaluated in O(n^3) (Section 1,
 *                         Figure 2 caption).  Used only to pin the above.
 *   oracle_appd_widest    The widest-path (maximum capacity) variant of
 *                         Section 4.2: maximum spanning tree, edges removed from
 *                         the smallest up.  Reversed total order: larger weight
 *                         first, equal weights ordered by smaller flat index.
 *   oracle_mst_prim       Prim's MST alone (order of attachment, parent, keys).
 *   oracle_linkage        The single-linkage dendrogram (scipy's linkage-matrix
 *                         layout) from the ascending construction: tree edges
 *                         added best first, union-find over clusters.
 *   oracle_pairwise_euclidean_f32 / _f64
 *                         Complete graph from a point set (Section 1, a dataset
 *                         "can be straightforwardly converted to a complete
 *                         graph"): W_ij = sqrt(sum_t (x_it - x_jt)^2), the sum
 *                         taken in increasing t, one rounding per operation.
 *   oracle_grad_points    d/dX of L = sum_{i != j} G_ij M_ij, accumulated in
 *                         double through the bottleneck edges named by idx and
 *                         the Euclidean edge weights (not in the paper: the
 *                         gradient of the selection the forward makes).
 *
 * Every double weight path also accepts float input (is64 = 0); float values
 * convert to double exactly, so comparisons and selections are unchanged.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    const float* w32;
    const double* w64;
    int64_t n;
} wmat;

static double wat(const wmat* m, int64_t i, int64_t j) {
    int64_t k = i * m->n + j;
    return m->w32 ? (double)m->w32[k] : m->w64[k];
}

static int64_t flat_of(int64_t u, int64_t v, int64_t n) {
    return u < v ? u * n + v : v * n + u;
}

/* a < b in the minimax total order */
static int key_less(double wa, int64_t fa, double wb, int64_t fb) {
    return wa < wb || (wa == wb && fa < fb);
}

/* a "better" than b for the spanning tree: minimax -> smaller, widest -> larger
 * weight, equal weights by smaller flat index in both cases */
static int tree_better(int widest, double wa, int64_t fa, double wb, int64_t fb) {
    if (widest) return wa > wb || (wa == wb && fa < fb);
    return key_less(wa, fa, wb, fb);
}

static double canon_zero(double w) { return w == 0.0 ? 0.0 : w; }

typedef struct {
    int64_t u, v; /* u = the vertex already in the tree, v = the one attached */
    double w;
    int64_t f;
} oedge;

/*
 * Prim's algorithm on the dense graph (Section 3: "construct a minimum
 * spanning tree ... with prim's algorithm", O(n^2)).  Starts from vertex 0
 * (the paper does not name a start vertex).  Each step attaches the unvisited
 * vertex whose best connecting edge is smallest in the total order; a key is
 * replaced only by a strictly better edge.  For widest = 1 "smaller" becomes
 * "larger weight" (a maximum spanning tree).  Fills edges[0..n-2] in
 * attachment order; order[k] = k-th vertex attached (order[0] = 0).
 */
static int prim_tree(const wmat* m, int widest, oedge* edges, int64_t* order) {
    int64_t n = m->n;
    double* kw = (double*)malloc(sizeof(double) * (size_t)n);
    int64_t* kf = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* kp = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    char* vis = (char*)calloc((size_t)n, 1);
    if (!kw || !kf || !kp || !vis) {
        free(kw); free(kf); free(kp); free(vis);
        return -3;
    }
    vis[0] = 1;
    if (order) order[0] = 0;
    for (int64_t v = 1; v < n; ++v) {
        kw[v] = wat(m, 0, v);
        kf[v] = flat_of(0, v, n);
        kp[v] = 0;
    }
    for (int64_t k = 1; k < n; ++k) {
        int64_t p = -1;
        for (int64_t v = 0; v < n; ++v) {
            if (vis[v]) continue;
            if (p < 0 || tree_better(widest, kw[v], kf[v], kw[p], kf[p])) p = v;
        }
        vis[p] = 1;
        if (order) order[k] = p;
        edges[k - 1].u = kp[p];
        edges[k - 1].v = p;
        edges[k - 1].w = kw[p];
        edges[k - 1].f = kf[p];
        for (int64_t v = 0; v < n; ++v) {
            if (vis[v]) continue;
            double w = wat(m, p, v);
            int64_t f = flat_of(p, v, n);
            if (tree_better(widest, w, f, kw[v], kf[v])) {
                kw[v] = w;
                kf[v] = f;
                kp[v] = p;
            }
        }
    }
    free(kw); free(kf); free(kp); free(vis);
    return 0;
}

static int g_widest_for_sort = 0;

/* qsort comparator: the removal order.  Minimax: descending (largest first,
 * Section 3).  Widest: ascending weight first (Section 4.2), i.e. the reverse
 * of the widest tree order. */
static int removal_cmp(const void* pa, const void* pb) {
    const oedge* a = (const oedge*)pa;
    const oedge* b = (const oedge*)pb;
    /* "a before b" iff b is better for the tree than a */
    if (tree_better(g_widest_for_sort, b->w, b->f, a->w, a->f)) return -1;
    if (tree_better(g_widest_for_sort, a->w, a->f, b->w, b->f)) return 1;
    return 0;
}

/* Forest stored as adjacency lists over the n-1 tree edges (CSR). */
typedef struct {
    int64_t* start; /* n+1 */
    int64_t* eid;   /* 2(n-1): edge id of each incidence */
    char* removed;  /* n-1 */
    int64_t* stack;
    int64_t* stamp;
    int64_t cur;
} forest;

static int forest_init(forest* F, const oedge* edges, int64_t n) {
    int64_t m = n - 1;
    F->start = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    F->eid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
    F->removed = (char*)calloc((size_t)m + 1, 1);
    F->stack = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    F->stamp = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    F->cur = 0;
    if (!F->start || !F->eid || !F->removed || !F->stack || !F->stamp) return -3;
    for (int64_t e = 0; e < m; ++e) {
        F->start[edges[e].u + 1]++;
        F->start[edges[e].v + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) F->start[i + 1] += F->start[i];
    int64_t* fillpos = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!fillpos) return -3;
    memcpy(fillpos, F->start, sizeof(int64_t) * (size_t)n);
    for (int64_t e = 0; e < m; ++e) {
        F->eid[fillpos[edges[e].u]++] = e;
        F->eid[fillpos[edges[e].v]++] = e;
    }
    free(fillpos);
    return 0;
}

static void forest_free(forest* F) {
    free(F->start); free(F->eid); free(F->removed); free(F->stack); free(F->stamp);
}

/* Traverse the sub-tree containing s over edges not yet removed (depth-first,
 * explicit stack).  Writes its vertices to out[], returns their count. */
static int64_t collect(forest* F, const oedge* edges, int64_t s, int64_t* out) {
    F->cur++;
    int64_t top = 0, cnt = 0;
    F->stack[top++] = s;
    F->stamp[s] = F->cur;
    while (top) {
        int64_t x = F->stack[--top];
        out[cnt++] = x;
        for (int64_t k = F->start[x]; k < F->start[x + 1]; ++k) {
            int64_t e = F->eid[k];
            if (F->removed[e]) continue;
            int64_t y = edges[e].u == x ? edges[e].v : edges[e].u;
            if (F->stamp[y] != F->cur) {
                F->stamp[y] = F->cur;
                F->stack[top++] = y;
            }
        }
    }
    return cnt;
}

/*
 * Algorithm 4 ("MMJ distance by Calculation and Copy"), Section 3, with the
 * output restricted to rows whose rowslot[] is >= 0 (rowslot == NULL: all rows,
 * row r goes to slot r).  M and idx are nrows x n.
 */
static int alg4_core(const wmat* m, int widest, const int64_t* rowslot, double* Md,
                     float* Mf, int32_t* idx) {
    int64_t n = m->n;
    oedge* edges = (oedge*)malloc(sizeof(oedge) * (size_t)(n > 1 ? n - 1 : 1));
    int64_t* t1 = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* t2 = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!edges || !t1 || !t2) {
        free(edges); free(t1); free(t2);
        return -3;
    }
    int rc = 0;
    /* diagonal */
    for (int64_t i = 0; i < n; ++i) {
        int64_t s = rowslot ? rowslot[i] : i;
        if (s < 0) continue;
        if (Md) Md[s * n + i] = 0.0;
        if (Mf) Mf[s * n + i] = 0.0f;
        idx[s * n + i] = -1;
    }
    if (n == 1) goto done;
    rc = prim_tree(m, widest, edges, NULL);
    if (rc) goto done;
    /* sort the tree edges: largest first (minimax) / smallest first (widest) */
    g_widest_for_sort = widest;
    qsort(edges, (size_t)(n - 1), sizeof(oedge), removal_cmp);
    {
        forest F;
        if (forest_init(&F, edges, n)) {
            forest_free(&F);
            rc = -3;
            goto done;
        }
        for (int64_t e = 0; e < n - 1; ++e) {
            /* remove edge e: it is the extreme edge of the sub-tree holding it */
            F.removed[e] = 1;
            int64_t c1 = collect(&F, edges, edges[e].u, t1); /* tree1 */
            int64_t c2 = collect(&F, edges, edges[e].v, t2); /* tree2 */
            double w = canon_zero(edges[e].w);
            int32_t f = (int32_t)edges[e].f;
            for (int64_t a = 0; a < c1; ++a) {
                int64_t p = t1[a];
                int64_t sp = rowslot ? rowslot[p] : p;
                for (int64_t b = 0; b < c2; ++b) {
                    int64_t q = t2[b];
                    int64_t sq = rowslot ? rowslot[q] : q;
                    if (sp >= 0) {
                        if (Md) Md[sp * n + q] = w;
                        if (Mf) Mf[sp * n + q] = (float)w;
                        idx[sp * n + q] = f;
                    }
                    if (sq >= 0) {
                        if (Md) Md[sq * n + p] = w;
                        if (Mf) Mf[sq * n + p] = (float)w;
                        idx[sq * n + p] = f;
                    }
                }
            }
        }
        forest_free(&F);
    }
done:
    free(edges); free(t1); free(t2);
    return rc;
}

static int bad_n(int64_t n) { return n < 1 || n > 46340; }

int oracle_appd_alg4(const float* W, int64_t n, float* M, int32_t* idx) {
    if (bad_n(n) || !W || !M || !idx) return -1;
    wmat m = {W, NULL, n};
    return alg4_core(&m, 0, NULL, NULL, M, idx);
}

int oracle_appd_alg4_f64(const double* W, int64_t n, double* M, int32_t* idx) {
    if (bad_n(n) || !W || !M || !idx) return -1;
    wmat m = {NULL, W, n};
    return alg4_core(&m, 0, NULL, M, NULL, idx);
}

int oracle_appd_widest(const float* W, int64_t n, float* M, int32_t* idx) {
    if (bad_n(n) || !W || !M || !idx) return -1;
    wmat m = {W, NULL, n};
    return alg4_core(&m, 1, NULL, NULL, M, idx);
}

/* rows[0..nrows-1] distinct vertex ids; output row r of M/idx is vertex rows[r] */
int oracle_appd_alg4_rows(const float* W, int64_t n, const int64_t* rows, int64_t nrows,
                          int widest, float* M, int32_t* idx) {
    if (bad_n(n) || !W || !M || !idx || !rows || nrows < 0) return -1;
    int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!slot) return -3;
    for (int64_t i = 0; i < n; ++i) slot[i] = -1;
    for (int64_t r = 0; r < nrows; ++r) {
        if (rows[r] < 0 || rows[r] >= n || slot[rows[r]] >= 0) {
            free(slot);
            return -1;
        }
        slot[rows[r]] = r;
    }
    wmat m = {W, NULL, n};
    int rc = alg4_core(&m, widest, slot, NULL, M, idx);
    free(slot);
    return rc;
}

/*
 * Prim's tree alone: order[k] = k-th vertex attached, parent[v] = the tree
 * vertex it attached to (parent[0] = -1), attach_w[k] / attach_f[k] = weight and
 * flat index of the edge that attached order[k] (k >= 1; slot 0 is unused).
 */
int oracle_mst_prim(const float* W, int64_t n, int widest, int64_t* order, int64_t* parent,
                    float* attach_w, int64_t* attach_f) {
    if (bad_n(n) || !W || !order || !parent) return -1;
    wmat m = {W, NULL, n};
    oedge* edges = (oedge*)malloc(sizeof(oedge) * (size_t)(n > 1 ? n - 1 : 1));
    if (!edges) return -3;
    int rc = n > 1 ? prim_tree(&m, widest, edges, order) : 0;
    if (n == 1) order[0] = 0;
    parent[0] = -1;
    if (attach_w) attach_w[0] = 0.0f;
    if (attach_f) attach_f[0] = -1;
    for (int64_t k = 1; k < n && rc == 0; ++k) {
        parent[edges[k - 1].v] = edges[k - 1].u;
        if (attach_w) attach_w[k] = (float)edges[k - 1].w;
        if (attach_f) attach_f[k] = edges[k - 1].f;
    }
    free(edges);
    return rc;
}

static int g_widest_for_link = 0;

/* qsort comparator: the spanning-tree order (best edge first). */
static int tree_order_cmp(const void* pa, const void* pb) {
    const oedge* a = (const oedge*)pa;
    const oedge* b = (const oedge*)pb;
    if (tree_better(g_widest_for_link, a->w, a->f, b->w, b->f)) return -1;
    if (tree_better(g_widest_for_link, b->w, b->f, a->w, a->f)) return 1;
    return 0;
}

static int64_t uf_find(int64_t* up, int64_t x) {
    while (up[x] != x) {
        up[x] = up[up[x]];
        x = up[x];
    }
    return x;
}

/*
 * Single-linkage dendrogram by the ascending construction that Section 3
 * mentions beside Algorithm 4: the spanning-tree edges are added one by one,
 * best first (minimax: ascending (w, flat); widest: larger weight first, equal
 * weights by smaller flat index), to an empty forest; each edge joins two
 * clusters.  Z[4i .. 4i+3] = {a, b, w, size}: the clusters joined by the i-th
 * edge (a < b; ids below n are vertices, n + j is the cluster made by edge j),
 * the edge's weight, and the number of vertices in the new cluster.
 */
int oracle_linkage(const float* W, int64_t n, int widest, double* Z) {
    if (bad_n(n) || !W || !Z) return -1;
    if (n == 1) return 0;
    wmat m = {W, NULL, n};
    oedge* edges = (oedge*)malloc(sizeof(oedge) * (size_t)(n - 1));
    int64_t* up = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* cid = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* csz = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!edges || !up || !cid || !csz) {
        free(edges); free(up); free(cid); free(csz);
        return -3;
    }
    int rc = prim_tree(&m, widest, edges, NULL);
    if (rc == 0) {
        g_widest_for_link = widest;
        qsort(edges, (size_t)(n - 1), sizeof(oedge), tree_order_cmp);
        for (int64_t v = 0; v < n; ++v) {
            up[v] = v;
            cid[v] = v;
            csz[v] = 1;
        }
        for (int64_t i = 0; i < n - 1; ++i) {
            const int64_t ra = uf_find(up, edges[i].u), rb = uf_find(up, edges[i].v);
            const int64_t a = cid[ra], b = cid[rb];
            Z[4 * i + 0] = (double)(a < b ? a : b);
            Z[4 * i + 1] = (double)(a < b ? b : a);
            Z[4 * i + 2] = canon_zero(edges[i].w);
            Z[4 * i + 3] = (double)(csz[ra] + csz[rb]);
            up[ra] = rb;
            cid[rb] = n + i;
            csz[rb] += csz[ra];
        }
    }
    free(edges); free(up); free(cid); free(csz);
    return rc;
}

/*
 * Minimax Floyd-Warshall over the edge total order: after relaxing through
 * every intermediate vertex k, K(i,j) is the smallest possible "largest edge"
 * over all paths i -> j, i.e. Eq. 1-2 with the bottleneck edge attached.
 * widest = 1: the largest possible "smallest edge" (reversed order).
 */
int oracle_appd_fw(const float* W, int64_t n, int widest, float* M, int32_t* idx) {
    if (bad_n(n) || !W || !M || !idx) return -1;
    double* kw = (double*)malloc(sizeof(double) * (size_t)(n * n));
    int64_t* kf = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n * n));
    if (!kw || !kf) {
        free(kw); free(kf);
        return -3;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            kw[i * n + j] = (double)W[i * n + j];
            kf[i * n + j] = i == j ? -1 : flat_of(i, j, n);
        }
    for (int64_t k = 0; k < n; ++k)
        for (int64_t i = 0; i < n; ++i) {
            if (i == k) continue;
            for (int64_t j = 0; j < n; ++j) {
                if (j == k || j == i) continue;
                /* bottleneck of the walk i -> k -> j: the worse of its two legs */
                double aw = kw[i * n + k], bw = kw[k * n + j];
                int64_t af = kf[i * n + k], bf = kf[k * n + j];
                double cw;
                int64_t cf;
                if (tree_better(widest, aw, af, bw, bf)) { cw = bw; cf = bf; }
                else { cw = aw; cf = af; }
                if (tree_better(widest, cw, cf, kw[i * n + j], kf[i * n + j])) {
                    kw[i * n + j] = cw;
                    kf[i * n + j] = cf;
                }
            }
        }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            M[i * n + j] = i == j ? 0.0f : (float)canon_zero(kw[i * n + j]);
            idx[i * n + j] = i == j ? -1 : (int32_t)kf[i * n + j];
        }
    free(kw); free(kf);
    return 0;
}

/* W_ij = sqrt(sum over t = 0..d-1, in that order, of (x_it - x_jt)^2), each
 * subtraction, product, sum and the square root rounded to float once
 * (this file is compiled without floating-point contraction). */
int oracle_pairwise_euclidean_f32(const float* X, int64_t n, int64_t d, float* W) {
    if (bad_n(n) || d < 1 || !X || !W) return -1;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            if (i == j) {
                W[i * n + j] = 0.0f;
                continue;
            }
            float acc = 0.0f;
            for (int64_t t = 0; t < d; ++t) {
                float diff = X[i * d + t] - X[j * d + t];
                float sq = diff * diff;
                acc = acc + sq;
            }
            W[i * n + j] = sqrtf(acc);
        }
    return 0;
}

int oracle_pairwise_euclidean_f64(const double* X, int64_t n, int64_t d, double* W) {
    if (bad_n(n) || d < 1 || !X || !W) return -1;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t t = 0; t < d && i != j; ++t) {
                double diff = X[i * d + t] - X[j * d + t];
                acc += diff * diff;
            }
            W[i * n + j] = sqrt(acc);
        }
    return 0;
}

/*
 * dL/dX for L = sum_{i != j} G_ij * M_ij, where M_ij is the weight of the edge
 * idx(i,j) and that weight is ||x_u - x_v||.  Each pair passes its G_ij to its
 * bottleneck edge (u,v); each edge then passes g * (x_u - x_v) / ||x_u - x_v||
 * to x_u and the negative to x_v (zero for a zero-length edge).  All in double.
 * dX (n x d) is overwritten.  gedge (optional, n*n) receives the per-edge sums
 * at the upper-triangle position u*n+v, u < v.
 */
int oracle_grad_points(const double* X, int64_t n, int64_t d, const double* G,
                       const int32_t* idx, double* dX, double* gedge) {
    if (bad_n(n) || d < 1 || !X || !G || !idx || !dX) return -1;
    double* g = gedge;
    int own = 0;
    if (!g) {
        g = (double*)calloc((size_t)(n * n), sizeof(double));
        if (!g) return -3;
        own = 1;
    } else {
        memset(g, 0, sizeof(double) * (size_t)(n * n));
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            if (i == j) continue;
            int32_t e = idx[i * n + j];
            if (e < 0) continue;
            g[e] += G[i * n + j];
        }
    memset(dX, 0, sizeof(double) * (size_t)(n * d));
    for (int64_t u = 0; u < n; ++u)
        for (int64_t v = u + 1; v < n; ++v) {
            double ge = g[u * n + v];
            if (ge == 0.0) continue;
            double r2 = 0.0;
            for (int64_t t = 0; t < d; ++t) {
                double df = X[u * d + t] - X[v * d + t];
                r2 += df * df;
            }
            double r = sqrt(r2);
            if (r == 0.0) continue;
            for (int64_t t = 0; t < d; ++t) {
                double df = X[u * d + t] - X[v * d + t];
                dX[u * d + t] += ge * df / r;
                dX[v * d + t] -= ge * df / r;
            }
        }
    if (own) free(g);
    return 0;
}

/* sum_{i != j} G_ij * M_ij with Neumaier compensated summation (for central
 * finite differences of the loss). */
double oracle_loss_f64(const double* G, const double* M, int64_t n) {
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            if (i == j) continue;
            double x = G[i * n + j] * M[i * n + j];
            double t = s + x;
            if (fabs(s) >= fabs(x)) c += (s - t) + x;
            else c += (x - t) + s;
            s = t;
        }
    return s + c;
}
