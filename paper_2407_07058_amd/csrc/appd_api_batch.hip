// C ABI of the batched and gradient calls (include/appd.h): host planning,
// workspace carving, argument checks.  All compute runs in the kernels.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "appd.h"
#include "appd_internal.h"

namespace {

int fail(int code) {
    appd::set_last_error(code);
    return code;
}

int ok() {
    appd::set_last_error(APPD_OK);
    return APPD_OK;
}

// Device tables of a batch, at the start of its workspace.
struct Tables {
    int32_t* ns;
    int64_t* offsets;
    int64_t* noff;
    int64_t* xoff;
    int32_t* perm;
    int32_t* chunk_start;
    int32_t* tile_start;
    int32_t* gchunk_start;
    int32_t* vstart;
    int32_t* rstart;
    int32_t* rgraph;
    // tree and gradient scratch
    int32_t* order;
    int32_t* parent;
    int32_t* pos;
    uint64_t* ek;
    float* gedge;
    appd::BatchBlk blk;
    uint64_t* lists;
    int32_t* tstats;
    size_t table_bytes;  // bytes of the region uploaded by prepare
    size_t total_bytes;
};

Tables carve(void* ws, int G, int64_t total_n) {
    using appd::align_up;
    const uintptr_t b = (uintptr_t)ws;  // null when only the size is wanted
    Tables t;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = (char*)(b + off);
        off = align_up(off + bytes);
        return p;
    };
    t.ns = (int32_t*)take(4 * (size_t)G);
    t.offsets = (int64_t*)take(8 * (size_t)G);
    t.noff = (int64_t*)take(8 * (size_t)G);
    t.perm = (int32_t*)take(4 * (size_t)G);
    t.chunk_start = (int32_t*)take(4 * (size_t)G);
    t.tile_start = (int32_t*)take(4 * (size_t)G);
    t.gchunk_start = (int32_t*)take(4 * (size_t)G);
    t.vstart = (int32_t*)take(4 * (size_t)G);
    t.rstart = (int32_t*)take(4 * (size_t)G);
    t.rgraph = (int32_t*)take(4 * (size_t)total_n);
    t.table_bytes = off;
    t.xoff = (int64_t*)take(8 * (size_t)G);
    t.order = (int32_t*)take(4 * (size_t)total_n);
    t.parent = (int32_t*)take(4 * (size_t)total_n);
    t.pos = (int32_t*)take(4 * (size_t)total_n);
    t.ek = (uint64_t*)take(8 * (size_t)total_n);
    t.gedge = (float*)take(4 * (size_t)total_n);
    t.blk.sp = (uint16_t*)take(2 * (size_t)total_n);
    t.blk.slot = (uint16_t*)take(2 * (size_t)total_n);
    t.blk.code = (uint32_t*)take(4 * (size_t)total_n);
    t.blk.dM = (float*)take(4 * (size_t)total_n);
    t.blk.dI = (int32_t*)take(4 * (size_t)total_n);
    t.blk.sorted = (uint64_t*)take(8 * (size_t)total_n);
    t.lists = (uint64_t*)take(8 * 16 * (size_t)total_n);
    t.tstats = (int32_t*)take(4 * (size_t)G);
    t.total_bytes = off;
    return t;
}

bool sizes_ok(const int32_t* ns, int G, int64_t* total_n) {
    if (!ns || G < 1) return false;
    int64_t tn = 0;
    for (int g = 0; g < G; ++g) {
        if (ns[g] < 1 || ns[g] > APPD_BATCH_MAX_N) return false;
        tn += ns[g];
    }
    *total_n = tn;
    return true;
}

bool plan_ok(const appd_batch_plan* p, const void* ws) {
    return p && ws && p->num_graphs >= 1 && p->ws_bytes > 0 && ((uintptr_t)ws & 255u) == 0;
}

appd::BatchPlan device_plan(const appd_batch_plan* p, const Tables& t) {
    appd::BatchPlan bp;
    bp.perm = t.perm;
    bp.noff = t.noff;
    bp.chunk_start = t.chunk_start;
    bp.rstart = t.rstart;
    bp.rgraph = t.rgraph;
    bp.lists = t.lists;
    bp.tstats = t.tstats;
    for (int c = 0; c < appd::kBatchClasses; ++c) {
        bp.class_first[c] = p->class_first[c];
        bp.class_count[c] = p->class_count[c];
        bp.class_chunks[c] = p->class_chunks[c];
        bp.class_rows[c] = p->class_rows[c];
        bp.class_threads[c] = p->class_threads[c];
        bp.class_tree[c] = p->class_tree[c];
        bp.class_vertices[c] = p->class_vertices[c];
    }
    bp.streams = p->streams;
    bp.split_count = p->split_count;
    bp.split_chunks = p->split_chunks;
    bp.split_vertices = p->split_vertices;
    return bp;
}

// Stamp of what the device work tables (chunk_start) were built for: the rows
// per fill item of every class and the cut of the largest class, which fix the
// chunk numbering the fill kernels search.  FNV-1a over those fields.
uint64_t tables_key_of(const appd_batch_plan* p) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (uint64_t)((v >> (8 * b)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    mix(p->num_graphs);
    mix(p->total_n);
    mix(p->total_nn);
    for (int c = 0; c < appd::kBatchClasses; ++c) {
        mix(p->class_first[c]);
        mix(p->class_count[c]);
        mix(p->class_rows[c]);
        mix(p->class_chunks[c]);
        mix(p->class_vertices[c]);
    }
    mix(p->split_count);
    mix(p->split_chunks);
    mix(p->split_vertices);
    return h;
}

bool schedule_ok(const appd_batch_plan* p) {
    // the fields that index the device tables must be the ones they were built for
    if (p->tables_key != tables_key_of(p)) return false;
    if (p->streams < 1 || p->streams > appd::kBatchClasses) return false;
    int top = -1;  // the largest class present
    for (int c = 0; c < appd::kBatchClasses; ++c)
        if (p->class_count[c]) top = c;
    if (p->split_count < 0 || p->split_chunks < 0 || p->split_vertices < 0) return false;
    if (p->split_count && (top < 0 || p->split_count >= p->class_count[top] ||
                           p->split_chunks < 1 || p->split_chunks >= p->class_chunks[top]))
        return false;
    for (int c = 0; c < appd::kBatchClasses; ++c) {
        if (!p->class_count[c]) continue;
        if (p->class_rows[c] < 1 || p->class_rows[c] > APPD_BATCH_MAX_N) return false;
        if (!appd::batch_threads_ok(c, p->class_threads[c])) return false;
        if (p->class_tree[c] != APPD_BATCH_TREE_PRIM && p->class_tree[c] != APPD_BATCH_TREE_BORUVKA)
            return false;
    }
    return true;
}

// Fill work items per class for the plan's rows per item; chunk_start[i] is the
// first item of the i-th graph (n-descending order) within its class.  split:
// 0 no cut; -1 a cut of the largest class into two parts of about equal work:
// with Boruvka trees (a pass over W and a fill, both n^2 per graph) where the
// running sum of n^2 reaches half the class's, with Prim trees after its graphs
// of n >= 0.84 n_max (a Prim chain grows with n and a fill with n^2, and for
// sizes spread evenly on a log scale over one class (n_max / 2, n_max] this cut
// gives the two parts about the same Prim + fill time); h > 0 the cut after its
// first h graphs.  Sets class_chunks, split_count, split_chunks, split_vertices
// and the tables' stamp.
void build_chunks(const int32_t* ns_host, const std::vector<int32_t>& perm, appd_batch_plan* p,
                  std::vector<int32_t>& chunk_start, int split) {
    const int G = p->num_graphs;
    chunk_start.assign(G, 0);
    for (int c = 0; c < appd::kBatchClasses; ++c) p->class_chunks[c] = 0;
    for (int i = 0; i < G; ++i) {
        const int n = ns_host[perm[i]];
        const int c = appd::batch_class_of(n);
        const int rows = p->class_rows[c];
        chunk_start[i] = p->class_chunks[c];
        p->class_chunks[c] += (n + rows - 1) / rows;
    }
    p->split_count = p->split_chunks = p->split_vertices = 0;
    int top = -1;
    for (int c = 0; c < appd::kBatchClasses; ++c)
        if (p->class_count[c]) top = c;
    if (split != 0 && top >= 0) {
        const int first = p->class_first[top], count = p->class_count[top];
        const int nmax = ns_host[perm[first]];
        int h = split;
        if (split < 0 && p->class_tree[top] == APPD_BATCH_TREE_BORUVKA) {
            int64_t all = 0, run = 0;
            for (int i = 0; i < count; ++i) all += (int64_t)ns_host[perm[first + i]] * ns_host[perm[first + i]];
            h = 0;
            while (h < count && 2 * run < all) {
                run += (int64_t)ns_host[perm[first + h]] * ns_host[perm[first + h]];
                ++h;
            }
        } else if (split < 0) {
            h = 0;
            while (h < count && 100 * (int64_t)ns_host[perm[first + h]] >= 84 * (int64_t)nmax) ++h;
        }
        if (h > 0 && h < count && chunk_start[first + h] > 0 &&
            chunk_start[first + h] < p->class_chunks[top]) {
            p->split_count = h;
            p->split_chunks = chunk_start[first + h];
            for (int i = 0; i < h; ++i) p->split_vertices += ns_host[perm[first + i]];
        }
    }
    p->tables_key = tables_key_of(p);
}

// Default schedule: Boruvka trees for every class (Prim workgroups, when a
// schedule picks Prim, of 64 threads up to n = 256 and 256 above); 16 rows per
// fill item; classes in order on the caller's stream.
void default_schedule(appd_batch_plan* p) {
    static const int threads[appd::kBatchClasses] = {64, 64, 64, 256, 256, 256};
    for (int c = 0; c < appd::kBatchClasses; ++c) {
        p->class_threads[c] = threads[c];
        p->class_rows[c] = 16;
        p->class_tree[c] = APPD_BATCH_TREE_BORUVKA;
    }
    p->streams = 1;
}

int hip_status(hipError_t e) {
    if (e == hipSuccess) return ok();
    (void)hipGetLastError();
    return fail(APPD_EHIP);
}

}  // namespace

extern "C" {

size_t appd_batch_workspace_bytes(const int32_t* ns_host, int num_graphs) {
    int64_t tn;
    if (!sizes_ok(ns_host, num_graphs, &tn)) return 0;
    return carve(nullptr, num_graphs, tn).total_bytes;
}

int appd_batch_prepare(const int32_t* ns_host, int num_graphs, void* ws, size_t ws_bytes,
                       appd_batch_plan* plan, void* stream) {
    int64_t tn;
    if (!plan || !ws || ((uintptr_t)ws & 255u) || !sizes_ok(ns_host, num_graphs, &tn))
        return fail(APPD_EINVAL);
    const int G = num_graphs;
    Tables lay = carve(nullptr, G, tn);
    if (ws_bytes < lay.total_bytes) return fail(APPD_EINVAL);

    appd_batch_plan p;
    std::memset(&p, 0, sizeof(p));
    p.num_graphs = G;
    p.total_n = tn;
    p.ws_bytes = lay.total_bytes;
    std::vector<int32_t> perm(G);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(),
                     [&](int a, int b) { return ns_host[a] > ns_host[b]; });
    std::vector<int64_t> offsets(G), noff(G);
    std::vector<int32_t> chunk_start(G), tile_start(G), gchunk_start(G), vstart(G), rstart(G);
    int64_t o = 0, no = 0;
    int64_t tiles = 0, gch = 0, vb = 0;
    const int tile = appd::pairwise_tile();
    for (int g = 0; g < G; ++g) {
        const int64_t n = ns_host[g];
        offsets[g] = o;
        noff[g] = no;
        tile_start[g] = (int32_t)tiles;
        gchunk_start[g] = (int32_t)gch;
        vstart[g] = (int32_t)vb;
        o += n * n;
        no += n;
        const int64_t nt = (n + tile - 1) / tile;
        tiles += nt * nt;
        gch += (n + appd::kGradRows - 1) / appd::kGradRows;
        vb += (n + appd::kChainThreads - 1) / appd::kChainThreads;
        p.max_n = std::max(p.max_n, (int)n);
    }
    if (tiles > INT32_MAX || gch > INT32_MAX || vb > INT32_MAX) return fail(APPD_EINVAL);
    p.total_nn = o;
    p.pair_tiles = (int)tiles;
    p.grad_chunks = (int)gch;
    p.chain_blocks = (int)vb;
    // classes are contiguous in perm (n descending, class ascending in n)
    for (int c = 0; c < appd::kBatchClasses; ++c) p.class_first[c] = -1;
    int64_t rs = 0;
    for (int i = 0; i < G; ++i) {
        const int c = appd::batch_class_of(ns_host[perm[i]]);
        if (p.class_first[c] < 0) p.class_first[c] = i;
        p.class_count[c]++;
        p.class_vertices[c] += ns_host[perm[i]];
        rstart[i] = (int32_t)rs;
        rs += ns_host[perm[i]];
    }
    if (rs > INT32_MAX) return fail(APPD_EINVAL);
    for (int c = 0; c < appd::kBatchClasses; ++c)
        if (p.class_first[c] < 0) p.class_first[c] = 0;
    default_schedule(&p);
    build_chunks(ns_host, perm, &p, chunk_start, 0);

    // one host image of the table region, one synchronous copy
    std::vector<char> img(lay.table_bytes, 0);
    Tables h = carve(img.data(), G, tn);
    std::memcpy(h.ns, ns_host, 4 * (size_t)G);
    std::memcpy(h.offsets, offsets.data(), 8 * (size_t)G);
    std::memcpy(h.noff, noff.data(), 8 * (size_t)G);
    std::memcpy(h.perm, perm.data(), 4 * (size_t)G);
    std::memcpy(h.chunk_start, chunk_start.data(), 4 * (size_t)G);
    std::memcpy(h.tile_start, tile_start.data(), 4 * (size_t)G);
    std::memcpy(h.gchunk_start, gchunk_start.data(), 4 * (size_t)G);
    std::memcpy(h.vstart, vstart.data(), 4 * (size_t)G);
    std::memcpy(h.rstart, rstart.data(), 4 * (size_t)G);
    for (int i = 0; i < G; ++i)
        std::fill(h.rgraph + rstart[i], h.rgraph + rstart[i] + ns_host[perm[i]], (int32_t)i);
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(ws, img.data(), lay.table_bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        return fail(APPD_EHIP);
    }
    *plan = p;
    return ok();
}

int appd_batch_autotune(const float* W, float* M, int32_t* idx, appd_batch_plan* plan, void* ws,
                        void* stream, float* best_ms) {
    if (!W || !M || !idx || !plan_ok(plan, ws) || !schedule_ok(plan)) return fail(APPD_EINVAL);
    hipStream_t s = (hipStream_t)stream;
    const int G = plan->num_graphs;
    Tables t = carve(ws, G, plan->total_n);
    std::vector<int32_t> ns(G), perm(G), chunk_start;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto hip_fail = [&](hipError_t e) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipGetLastError();
        (void)e;
        return fail(APPD_EHIP);
    };
    hipError_t e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess ||
        (e = hipMemcpy(ns.data(), t.ns, 4 * (size_t)G, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(perm.data(), t.perm, 4 * (size_t)G, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
        return hip_fail(e);
    // candidates: Prim workgroup sizes (narrow / wide), fill rows per item,
    // classes in order or on concurrent streams
    static const int narrow[appd::kBatchClasses] = {64, 64, 64, 256, 256, 256};
    static const int wide[appd::kBatchClasses] = {64, 128, 256, 512, 512, 1024};
    static const int rows_opt[3] = {16, 32, 64};
    // at most 4 streams: a process gets 4 hardware queues by default, and a
    // fifth stream shares one with another (a kernel trace of a HIP-graph
    // replay showed a small class queued behind the largest one)
    static const int streams_opt[3] = {1, 3, 4};
    appd_batch_plan best = *plan;
    float best_t = -1.f;
    for (int wsel = 0; wsel < 2; ++wsel)
        for (int ri = 0; ri < 3; ++ri)
            for (int si = 0; si < 3; ++si)
              for (int sp = 0; sp < 2; ++sp) {
                if (sp && streams_opt[si] == 1) continue;  // a split needs two streams
                appd_batch_plan p = *plan;
                for (int c = 0; c < appd::kBatchClasses; ++c) {
                    p.class_threads[c] = wsel ? wide[c] : narrow[c];
                    p.class_rows[c] = rows_opt[ri];
                }
                p.streams = streams_opt[si];
                build_chunks(ns.data(), perm, &p, chunk_start, sp ? -1 : 0);
                if ((e = hipStreamSynchronize(s)) != hipSuccess ||
                    (e = hipMemcpy(t.chunk_start, chunk_start.data(), 4 * (size_t)G,
                                   hipMemcpyHostToDevice)) != hipSuccess)
                    return hip_fail(e);
                appd::BatchTree tree{t.order, t.ek, t.pos, t.parent};
                appd::BatchPlan bp = device_plan(&p, t);
                float tt = 0.f;
                for (int rep = 0; rep < 3; ++rep) {  // one warm-up, two timed
                    if (rep == 1 && (e = hipEventRecord(e0, s)) != hipSuccess) return hip_fail(e);
                    if ((e = appd::run_batched(W, t.offsets, t.ns, bp, tree, t.blk, APPD_MINIMAX, M,
                                               idx, s)) != hipSuccess)
                        return hip_fail(e);
                }
                if ((e = hipEventRecord(e1, s)) != hipSuccess ||
                    (e = hipEventSynchronize(e1)) != hipSuccess ||
                    (e = hipEventElapsedTime(&tt, e0, e1)) != hipSuccess)
                    return hip_fail(e);
                tt *= 0.5f;
                if (best_t < 0.f || tt < best_t) {
                    best_t = tt;
                    best = p;
                }
            }
    build_chunks(ns.data(), perm, &best, chunk_start, best.split_count);
    if ((e = hipMemcpy(t.chunk_start, chunk_start.data(), 4 * (size_t)G,
                       hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *plan = best;
    if (best_ms) *best_ms = best_t;
    return ok();
}

int appd_batch_set_schedule(appd_batch_plan* plan, void* ws, void* stream) {
    if (!plan_ok(plan, ws) || plan->streams < 1 || plan->streams > appd::kBatchClasses ||
        plan->split_count < -1)
        return fail(APPD_EINVAL);
    for (int c = 0; c < appd::kBatchClasses; ++c) {
        if (!plan->class_count[c]) continue;
        if (plan->class_rows[c] < 1 || plan->class_rows[c] > APPD_BATCH_MAX_N ||
            !appd::batch_threads_ok(c, plan->class_threads[c]))
            return fail(APPD_EINVAL);
    }
    const int G = plan->num_graphs;
    Tables t = carve(ws, G, plan->total_n);
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> ns(G), perm(G), chunk_start;
    if (hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(ns.data(), t.ns, 4 * (size_t)G, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(perm.data(), t.perm, 4 * (size_t)G, hipMemcpyDeviceToHost) != hipSuccess)
        return hip_status(hipErrorUnknown);
    appd_batch_plan p = *plan;
    const int want = p.split_count;
    build_chunks(ns.data(), perm, &p, chunk_start, want);
    if (want > 0 && p.split_count != want) return fail(APPD_EINVAL);  // cut out of range
    if (hipMemcpy(t.chunk_start, chunk_start.data(), 4 * (size_t)G, hipMemcpyHostToDevice) !=
        hipSuccess)
        return hip_status(hipErrorUnknown);
    *plan = p;
    return ok();
}

int appd_batch_tree_stats(const appd_batch_plan* plan, const void* ws, int32_t* stats,
                          void* stream) {
    if (!stats || !plan_ok(plan, const_cast<void*>(ws))) return fail(APPD_EINVAL);
    Tables t = carve(const_cast<void*>(ws), plan->num_graphs, plan->total_n);
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(stats, t.tstats, 4 * (size_t)plan->num_graphs, hipMemcpyDeviceToHost) != hipSuccess)
        return hip_status(hipErrorUnknown);
    return ok();
}

int appd_forward_batched(const float* W, int mode, float* M, int32_t* idx, int32_t* parent,
                         const appd_batch_plan* plan, void* ws, void* stream) {
    if (!W || !M || !idx || !plan_ok(plan, ws) || !schedule_ok(plan) ||
        (mode != APPD_MINIMAX && mode != APPD_WIDEST))
        return fail(APPD_EINVAL);
    Tables t = carve(ws, plan->num_graphs, plan->total_n);
    appd::BatchTree tree{t.order, t.ek, t.pos, parent ? parent : t.parent};
    appd::BatchPlan bp = device_plan(plan, t);
    return hip_status(appd::run_batched(W, t.offsets, t.ns, bp, tree, t.blk, mode, M, idx,
                                        (hipStream_t)stream));
}

int appd_pairwise_euclidean_batched(const float* X, int d, float* W, const appd_batch_plan* plan,
                                    void* ws, void* stream) {
    if (!X || !W || !plan_ok(plan, ws) || d < 1 || d > APPD_MAX_DIM) return fail(APPD_EINVAL);
    Tables t = carve(ws, plan->num_graphs, plan->total_n);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = appd::run_scale_offsets(t.noff, plan->num_graphs, d, t.xoff, s);
    if (e == hipSuccess)
        e = appd::run_pairwise(X, t.xoff, t.offsets, t.ns, t.tile_start, plan->num_graphs,
                               plan->pair_tiles, d, W, s);
    return hip_status(e);
}

int appd_backward_points_batched(const float* X, int d, const float* W, const float* G,
                                 const int32_t* idx, const int32_t* parent, float* dX,
                                 const appd_batch_plan* plan, void* ws, void* stream) {
    if (!X || !W || !G || !idx || !parent || !dX || !plan_ok(plan, ws) || d < 1 ||
        d > APPD_MAX_DIM)
        return fail(APPD_EINVAL);
    Tables t = carve(ws, plan->num_graphs, plan->total_n);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = appd::run_zero(t.gedge, 4 * (size_t)plan->total_n, s);
    if (e == hipSuccess) e = appd::run_zero(dX, 4 * (size_t)plan->total_n * d, s);
    if (e == hipSuccess) e = appd::run_scale_offsets(t.noff, plan->num_graphs, d, t.xoff, s);
    if (e == hipSuccess)
        e = appd::run_edge_grad(G, idx, t.offsets, t.noff, t.ns, parent, t.gchunk_start,
                                plan->num_graphs, plan->grad_chunks, appd::kGradRows, plan->max_n,
                                t.gedge, s);
    if (e == hipSuccess)
        e = appd::run_chain(X, t.xoff, W, t.offsets, t.noff, t.ns, parent, t.gedge, t.vstart,
                            plan->num_graphs, plan->chain_blocks, d, dX, s);
    return hip_status(e);
}

// ---- single-graph forms: a one-graph table written by a kernel (capture-safe)
size_t appd_grad_workspace_bytes(int n) {
    if (n < 1 || n > APPD_MAX_N) return 0;
    return carve(nullptr, 1, n).total_bytes;
}

static int single_tables(int n, void* ws, size_t ws_bytes, Tables* t, hipStream_t s) {
    if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < appd_grad_workspace_bytes(n)) return APPD_EINVAL;
    *t = carve(ws, 1, n);
    if (appd::run_single_table(n, t->ns, t->offsets, t->noff, t->tile_start, t->gchunk_start,
                               t->vstart, s) != hipSuccess)
        return APPD_EHIP;
    return APPD_OK;
}

int appd_pairwise_euclidean(const float* X, int n, int d, float* W, void* ws, size_t ws_bytes,
                            void* stream) {
    if (!X || !W || n < 1 || n > APPD_MAX_N || d < 1 || d > APPD_MAX_DIM) return fail(APPD_EINVAL);
    hipStream_t s = (hipStream_t)stream;
    Tables t;
    int rc = single_tables(n, ws, ws_bytes, &t, s);
    if (rc != APPD_OK) return rc == APPD_EHIP ? hip_status(hipErrorUnknown) : fail(rc);
    const int64_t nt = (n + appd::pairwise_tile() - 1) / appd::pairwise_tile();
    hipError_t e = appd::run_scale_offsets(t.noff, 1, d, t.xoff, s);
    if (e == hipSuccess)
        e = appd::run_pairwise(X, t.xoff, t.offsets, t.ns, t.tile_start, 1, (int)(nt * nt), d, W, s);
    return hip_status(e);
}

int appd_backward_points(const float* X, int n, int d, const float* W, const float* G,
                         const int32_t* idx, const int32_t* parent, float* dX, void* ws,
                         size_t ws_bytes, void* stream) {
    if (!X || !W || !G || !idx || !parent || !dX || n < 1 || n > APPD_GRAD_MAX_N || d < 1 ||
        d > APPD_MAX_DIM)
        return fail(APPD_EINVAL);
    hipStream_t s = (hipStream_t)stream;
    Tables t;
    int rc = single_tables(n, ws, ws_bytes, &t, s);
    if (rc != APPD_OK) return rc == APPD_EHIP ? hip_status(hipErrorUnknown) : fail(rc);
    const int chunks = (n + appd::kGradRows - 1) / appd::kGradRows;
    const int vblocks = (n + appd::kChainThreads - 1) / appd::kChainThreads;
    hipError_t e = appd::run_zero(t.gedge, 4 * (size_t)n, s);
    if (e == hipSuccess) e = appd::run_zero(dX, 4 * (size_t)n * d, s);
    if (e == hipSuccess) e = appd::run_scale_offsets(t.noff, 1, d, t.xoff, s);
    if (e == hipSuccess)
        e = appd::run_edge_grad(G, idx, t.offsets, t.noff, t.ns, parent, t.gchunk_start, 1,
                                chunks, appd::kGradRows, n, t.gedge, s);
    if (e == hipSuccess)
        e = appd::run_chain(X, t.xoff, W, t.offsets, t.noff, t.ns, parent, t.gedge, t.vstart, 1,
                            vblocks, d, dX, s);
    return hip_status(e);
}

int appd_backward_w(const float* G, const int32_t* idx, const int32_t* parent, int n, float* dW,
                    void* ws, size_t ws_bytes, void* stream) {
    if (!G || !idx || !parent || !dW || n < 1 || n > APPD_GRAD_MAX_N) return fail(APPD_EINVAL);
    hipStream_t s = (hipStream_t)stream;
    Tables t;
    int rc = single_tables(n, ws, ws_bytes, &t, s);
    if (rc != APPD_OK) return rc == APPD_EHIP ? hip_status(hipErrorUnknown) : fail(rc);
    const int chunks = (n + appd::kGradRows - 1) / appd::kGradRows;
    hipError_t e = appd::run_zero(t.gedge, 4 * (size_t)n, s);
    if (e == hipSuccess) e = appd::run_zero(dW, 4 * (size_t)n * n, s);
    if (e == hipSuccess)
        e = appd::run_edge_grad(G, idx, t.offsets, t.noff, t.ns, parent, t.gchunk_start, 1,
                                chunks, appd::kGradRows, n, t.gedge, s);
    if (e == hipSuccess)
        e = appd::run_edge_to_w(t.gedge, parent, t.offsets, t.noff, t.ns, t.vstart, 1,
                                (n + appd::kChainThreads - 1) / appd::kChainThreads, dW, s);
    return hip_status(e);
}

int appd_backward_w_batched(const float* G, const int32_t* idx, const int32_t* parent, float* dW,
                            const appd_batch_plan* plan, void* ws, void* stream) {
    if (!G || !idx || !parent || !dW || !plan_ok(plan, ws)) return fail(APPD_EINVAL);
    Tables t = carve(ws, plan->num_graphs, plan->total_n);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = appd::run_zero(t.gedge, 4 * (size_t)plan->total_n, s);
    if (e == hipSuccess) e = appd::run_zero(dW, 4 * (size_t)plan->total_nn, s);
    if (e == hipSuccess)
        e = appd::run_edge_grad(G, idx, t.offsets, t.noff, t.ns, parent, t.gchunk_start,
                                plan->num_graphs, plan->grad_chunks, appd::kGradRows, plan->max_n,
                                t.gedge, s);
    if (e == hipSuccess)
        e = appd::run_edge_to_w(t.gedge, parent, t.offsets, t.noff, t.ns, t.vstart,
                                plan->num_graphs, plan->chain_blocks, dW, s);
    return hip_status(e);
}

}  // extern "C"
