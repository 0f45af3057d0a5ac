// C ABI of the batched and gradient calls (include/appd.h): host planning,
// workspace carving, argument checks.  All compute runs in the kernels.
#include <stdio.h>
#include <stdlib.h>
#include <unistd.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "appd.h"
#include "appd_internal.h"
#include "appd_wcount.h"

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
    uint2* items;  // work queue of the persistent form
    int* ctr;      // its counters
    size_t table_bytes;  // bytes of the region uploaded by prepare
    size_t total_bytes;
};

// Work items of the persistent form, at most: one pass item per
// kPersistThreads / 64 rows, one tree item per graph, one fill item per row.
size_t items_capacity(int G, int64_t total_n) {
    return (size_t)total_n + (size_t)(total_n + 7) / 8 + (size_t)G + 2;
}

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
    t.items = (uint2*)take(8 * items_capacity(G, total_n));
    t.ctr = (int*)take(4 * (2 + 2 * (size_t)G));
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
    bp.persistent = p->persistent;
    bp.persist_items = p->persist_items;
    bp.stagger = p->stagger;
    bp.num_graphs = p->num_graphs;
    bp.total_n = (int)p->total_n;
    bp.items = t.items;
    bp.ctr = t.ctr;
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
    mix(p->persistent);
    mix(p->persist_items);
    return h;
}

// The persistent form takes Boruvka classes of n <= kPersistMaxN only.
bool persistent_ok(const appd_batch_plan* p) {
    for (int c = 0; c < appd::kBatchClasses; ++c) {
        if (!p->class_count[c]) continue;
        if (appd::kClassMaxN[c] > appd::kPersistMaxN) return false;
        if (p->class_tree[c] != APPD_BATCH_TREE_BORUVKA) return false;
    }
    return true;
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
    if (p->persistent != 0 && p->persistent != 1) return false;
    if (p->stagger != 0 && p->stagger != 1) return false;
    if (p->persistent && !persistent_ok(p)) return false;
    if (p->persistent &&
        (p->persist_items < 1 || (size_t)p->persist_items > items_capacity(p->num_graphs, p->total_n)))
        return false;
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
                  std::vector<int32_t>& chunk_start, int split, std::vector<uint2>* items) {
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
    p->persist_items = 0;
    if (items) items->clear();
    if (p->persistent && items) {
        // pass items over the rows in perm order, each graph's tree item after
        // the pass item holding its last row; then the fill items, largest
        // graphs first
        constexpr int NW = appd::kPersistThreads / 64;  // one row per wave
        const int64_t total = p->total_n;
        int gi = 0;
        int64_t gend = ns_host[perm[0]];
        for (int64_t r = 0; r < total; r += NW) {
            items->push_back(make_uint2(appd::kItemPass << 30 | (uint32_t)r, 0u));
            const int64_t rend = std::min<int64_t>(total, r + NW);
            while (gi < G && gend <= rend) {
                items->push_back(make_uint2(appd::kItemTree << 30 | (uint32_t)gi, 0u));
                if (++gi < G) gend += ns_host[perm[gi]];
            }
        }
        for (int i = 0; i < G; ++i) {
            const int n = ns_host[perm[i]];
            const int rows = p->class_rows[appd::batch_class_of(n)];
            for (int r0 = 0; r0 < n; r0 += rows)
                items->push_back(make_uint2(appd::kItemFill << 30 | (uint32_t)i,
                                            (uint32_t)r0 | (uint32_t)std::min(rows, n - r0) << 16));
        }
        p->persist_items = (int)items->size();
    }
    p->tables_key = tables_key_of(p);
}

// Uploads what build_chunks made (synchronous copies).
hipError_t upload_schedule(const Tables& t, int G, const std::vector<int32_t>& chunk_start,
                           const std::vector<uint2>& items) {
    hipError_t e = hipMemcpy(t.chunk_start, chunk_start.data(), 4 * (size_t)G, hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(t.items, items.data(), 8 * items.size(), hipMemcpyHostToDevice);
    return e;
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

// ---- autotuner: candidate schedules and the plan cache

constexpr int kTuneReps = 5;  // timed forwards per candidate (the median counts)

// What a schedule sets (split: the cut argument of build_chunks, 0 or -1).
struct TuneEntry {
    int streams = 1, split = 0, persistent = 0, stagger = 0;
    int rows[appd::kBatchClasses] = {};
    int tree[appd::kBatchClasses] = {};
    int threads[appd::kBatchClasses] = {};
    float ms = -1.f;
};

TuneEntry entry_of(const appd_batch_plan* p) {
    TuneEntry e;
    e.streams = p->streams;
    e.split = p->split_count ? -1 : 0;
    e.persistent = p->persistent;
    e.stagger = p->stagger;
    for (int c = 0; c < appd::kBatchClasses; ++c) {
        e.rows[c] = p->class_rows[c];
        e.tree[c] = p->class_tree[c];
        e.threads[c] = p->class_threads[c];
    }
    return e;
}

void apply_entry(const TuneEntry& e, appd_batch_plan* p) {
    p->streams = e.streams;
    p->persistent = e.persistent;
    p->stagger = e.stagger;
    for (int c = 0; c < appd::kBatchClasses; ++c) {
        p->class_rows[c] = e.rows[c];
        p->class_tree[c] = e.tree[c];
        p->class_threads[c] = e.threads[c];
    }
}

// Cache key: the device (architecture and name) and the batch's class
// histogram (graphs per size class).
std::string tune_key(const appd_batch_plan* p) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return std::string();
    }
    std::string k = std::string(prop.gcnArchName) + "|" + prop.name + "|classes";
    for (int c = 0; c < appd::kBatchClasses; ++c) k += ":" + std::to_string(p->class_count[c]);
    for (char& ch : k)
        if (ch == '"' || ch == '\\' || (unsigned char)ch < 0x20) ch = '_';
    return k;
}

// The cache file is one JSON object, one entry per line:
//   "key": {"streams": 3, "split": -1, "persistent": 0, "stagger": 1, "rows": [...6],
//           "trees": [...6], "threads": [...6], "ms": 1.234}
std::string entry_line(const std::string& key, const TuneEntry& e) {
    char buf[512];
    std::string r = "\"" + key + "\": {";
    snprintf(buf, sizeof buf, "\"streams\": %d, \"split\": %d, \"persistent\": %d, \"stagger\": %d",
             e.streams, e.split, e.persistent, e.stagger);
    r += buf;
    const int* arr[3] = {e.rows, e.tree, e.threads};
    const char* names[3] = {"rows", "trees", "threads"};
    for (int a = 0; a < 3; ++a) {
        r += std::string(", \"") + names[a] + "\": [";
        for (int c = 0; c < appd::kBatchClasses; ++c) r += (c ? ", " : "") + std::to_string(arr[a][c]);
        r += "]";
    }
    snprintf(buf, sizeof buf, ", \"ms\": %.4f}", e.ms);
    return r + buf;
}

bool parse_entry(const std::string& line, std::string* key, TuneEntry* e) {
    const size_t q0 = line.find('"');
    const size_t q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
    if (q1 == std::string::npos) return false;
    *key = line.substr(q0 + 1, q1 - q0 - 1);
    const char* s = line.c_str() + q1 + 1;
    int v[4 + 3 * appd::kBatchClasses];
    float ms = 0.f;
    int used = 0;
    if (sscanf(s, ": {\"streams\": %d, \"split\": %d, \"persistent\": %d, \"stagger\": %d%n", &v[0],
               &v[1], &v[2], &v[3], &used) != 4)
        return false;
    s += used;
    const char* names[3] = {"rows", "trees", "threads"};
    for (int a = 0; a < 3; ++a) {
        const std::string head = std::string(", \"") + names[a] + "\": [";
        if (strncmp(s, head.c_str(), head.size()) != 0) return false;
        s += head.size();
        for (int c = 0; c < appd::kBatchClasses; ++c) {
            if (sscanf(s, c ? ", %d%n" : "%d%n", &v[4 + a * appd::kBatchClasses + c], &used) != 1)
                return false;
            s += used;
        }
        if (*s++ != ']') return false;
    }
    if (sscanf(s, ", \"ms\": %f", &ms) != 1) return false;
    e->streams = v[0];
    e->split = v[1];
    e->persistent = v[2];
    e->stagger = v[3];
    for (int c = 0; c < appd::kBatchClasses; ++c) {
        e->rows[c] = v[4 + c];
        e->tree[c] = v[4 + appd::kBatchClasses + c];
        e->threads[c] = v[4 + 2 * appd::kBatchClasses + c];
    }
    e->ms = ms;
    return true;
}

std::vector<std::string> read_lines(const char* path) {
    std::vector<std::string> out;
    FILE* f = fopen(path, "r");
    if (!f) return out;
    char buf[4096];
    while (fgets(buf, sizeof buf, f)) {
        std::string l(buf);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r' || l.back() == ',')) l.pop_back();
        if (!l.empty() && l[0] == '"') out.push_back(l);
    }
    fclose(f);
    return out;
}

bool cache_lookup(const char* path, const std::string& key, TuneEntry* e) {
    for (const std::string& l : read_lines(path)) {
        std::string k;
        TuneEntry x;
        if (parse_entry(l, &k, &x) && k == key) {
            *e = x;
            return true;
        }
    }
    return false;
}

// Replaces or adds the key's entry; the file is written beside and renamed
// over the old one, so a reader never sees half a file.
void cache_store(const char* path, const std::string& key, const TuneEntry& e) {
    std::vector<std::string> lines;
    for (const std::string& l : read_lines(path)) {
        std::string k;
        TuneEntry x;
        if (parse_entry(l, &k, &x) && k != key) lines.push_back(l);
    }
    lines.push_back(entry_line(key, e));
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fputs("{\n", f);
    for (size_t i = 0; i < lines.size(); ++i)
        fprintf(f, "%s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
    fputs("}\n", f);
    const bool good = fclose(f) == 0;
    if (good) rename(tmp.c_str(), path);
    else remove(tmp.c_str());
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
        tiles += nt * (nt + 1) / 2;  // upper-triangle tile pairs
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
    std::vector<uint2> items;
    build_chunks(ns_host, perm, &p, chunk_start, 0, &items);

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
        hipStreamSynchronize(s) != hipSuccess ||
        (!items.empty() && upload_schedule(carve(ws, G, tn), G, chunk_start, items) != hipSuccess)) {
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
    std::vector<uint2> items;
    hipEvent_t ev[kTuneReps + 1] = {};
    auto hip_fail = [&]() {
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
        (void)hipGetLastError();
        return fail(APPD_EHIP);
    };
    if (hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(ns.data(), t.ns, 4 * (size_t)G, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(perm.data(), t.perm, 4 * (size_t)G, hipMemcpyDeviceToHost) != hipSuccess)
        return hip_fail();
    // a schedule from the plan cache, when one is kept for this device and
    // class histogram
    const char* cache = getenv("APPD_TUNE_CACHE");
    const std::string key = tune_key(plan);
    TuneEntry hit;
    if (cache && *cache && !key.empty() && cache_lookup(cache, key, &hit)) {
        appd_batch_plan p = *plan;
        apply_entry(hit, &p);
        build_chunks(ns.data(), perm, &p, chunk_start, hit.split, &items);
        if (schedule_ok(&p) && upload_schedule(t, G, chunk_start, items) == hipSuccess) {
            *plan = p;
            if (best_ms) *best_ms = hit.ms;
            return ok();
        }
    }
    for (hipEvent_t& x : ev)
        if (hipEventCreate(&x) != hipSuccess) return hip_fail();
    // time of one candidate: the median over kTuneReps forwards after one
    // warm-up forward (split: the cut argument of build_chunks)
    auto measure = [&](appd_batch_plan* p, int split, float* ms) -> bool {
        build_chunks(ns.data(), perm, p, chunk_start, split, &items);
        if (!schedule_ok(p)) return false;
        if (hipStreamSynchronize(s) != hipSuccess || upload_schedule(t, G, chunk_start, items) != hipSuccess)
            return false;
        appd::BatchTree tree{t.order, t.ek, t.pos, t.parent};
        const appd::BatchPlan bp = device_plan(p, t);
        if (appd::run_batched(W, t.offsets, t.ns, bp, tree, t.blk, APPD_MINIMAX, M, idx, s) != hipSuccess)
            return false;
        for (int r = 0; r < kTuneReps; ++r) {
            if (hipEventRecord(ev[r], s) != hipSuccess ||
                appd::run_batched(W, t.offsets, t.ns, bp, tree, t.blk, APPD_MINIMAX, M, idx, s) != hipSuccess)
                return false;
        }
        if (hipEventRecord(ev[kTuneReps], s) != hipSuccess || hipEventSynchronize(ev[kTuneReps]) != hipSuccess)
            return false;
        float v[kTuneReps];
        for (int r = 0; r < kTuneReps; ++r)
            if (hipEventElapsedTime(&v[r], ev[r], ev[r + 1]) != hipSuccess) return false;
        std::sort(v, v + kTuneReps);
        *ms = v[kTuneReps / 2];
        return true;
    };
    TuneEntry best;
    best.ms = -1.f;
    auto consider = [&](const TuneEntry& cand) -> bool {
        appd_batch_plan p = *plan;
        apply_entry(cand, &p);
        float ms = 0.f;
        if (!measure(&p, cand.split, &ms)) return false;
        if (best.ms < 0.f || ms < best.ms) {
            best = cand;
            best.ms = ms;
        }
        return true;
    };
    // 1. the launch forms with 16 rows per fill item everywhere and Boruvka
    //    trees: classes in order, on 3 or 4 streams (all starting at once,
    //    staggered after the largest class's pass, or with the largest class
    //    cut), and the persistent launch
    TuneEntry base = entry_of(plan);
    for (int c = 0; c < appd::kBatchClasses; ++c) {
        base.rows[c] = 16;
        base.tree[c] = APPD_BATCH_TREE_BORUVKA;
    }
    base.persistent = 0;
    base.stagger = 0;
    static const int streams_opt[3] = {1, 3, 4};
    for (int si = 0; si < 3; ++si)
        for (int form = 0; form < 3; ++form) {  // 0: at once, 1: staggered, 2: cut
            if (form && streams_opt[si] == 1) continue;  // both need two streams
            TuneEntry c = base;
            c.streams = streams_opt[si];
            c.stagger = form == 1;
            c.split = form == 2 ? -1 : 0;
            if (!consider(c)) return hip_fail();
        }
    {
        appd_batch_plan p = *plan;
        TuneEntry c = base;
        c.persistent = 1;
        c.streams = 1;
        c.split = 0;
        apply_entry(c, &p);
        if (persistent_ok(&p) && !consider(c)) return hip_fail();
    }
    // 2. per class, largest first: rows per fill item and (launch sequence
    //    only) the tree: Boruvka, or Prim with a narrow or a wide workgroup
    static const int narrow[appd::kBatchClasses] = {64, 64, 64, 256, 256, 256};
    static const int wide[appd::kBatchClasses] = {64, 128, 256, 512, 512, 1024};
    static const int rows_opt[3] = {8, 16, 32};
    for (int c = appd::kBatchClasses - 1; c >= 0; --c) {
        if (!plan->class_count[c]) continue;
        const TuneEntry cur = best;
        for (int ri = 0; ri < 3; ++ri)
            for (int tr = 0; tr < (cur.persistent ? 1 : 3); ++tr) {
                TuneEntry x = cur;
                x.rows[c] = rows_opt[ri];
                x.tree[c] = tr == 0 ? APPD_BATCH_TREE_BORUVKA : APPD_BATCH_TREE_PRIM;
                x.threads[c] = tr == 2 ? wide[c] : narrow[c];
                if (x.rows[c] == cur.rows[c] && x.tree[c] == cur.tree[c] &&
                    (x.tree[c] == APPD_BATCH_TREE_BORUVKA || x.threads[c] == cur.threads[c]))
                    continue;
                if (!consider(x)) return hip_fail();
            }
    }
    // 3. the other start of the classes for the schedule found (the trees
    //    chosen per class change what runs beside the largest class)
    if (best.streams > 1 && !best.split && !best.persistent) {
        TuneEntry x = best;
        x.stagger = !best.stagger;
        if (!consider(x)) return hip_fail();
    }
    for (hipEvent_t& x : ev) {
        (void)hipEventDestroy(x);
        x = nullptr;
    }
    appd_batch_plan p = *plan;
    apply_entry(best, &p);
    build_chunks(ns.data(), perm, &p, chunk_start, best.split, &items);
    if (hipStreamSynchronize(s) != hipSuccess || upload_schedule(t, G, chunk_start, items) != hipSuccess)
        return hip_fail();
    if (cache && *cache && !key.empty()) cache_store(cache, key, best);
    *plan = p;
    if (best_ms) *best_ms = best.ms;
    return ok();
}

int appd_batch_set_schedule(appd_batch_plan* plan, void* ws, void* stream) {
    if (!plan_ok(plan, ws) || plan->streams < 1 || plan->streams > appd::kBatchClasses ||
        plan->split_count < -1 || (plan->persistent != 0 && plan->persistent != 1) ||
        (plan->stagger != 0 && plan->stagger != 1) || (plan->persistent && !persistent_ok(plan)))
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
    std::vector<uint2> items;
    if (hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(ns.data(), t.ns, 4 * (size_t)G, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(perm.data(), t.perm, 4 * (size_t)G, hipMemcpyDeviceToHost) != hipSuccess)
        return hip_status(hipErrorUnknown);
    appd_batch_plan p = *plan;
    const int want = p.split_count;
    build_chunks(ns.data(), perm, &p, chunk_start, want, &items);
    if (want > 0 && p.split_count != want) return fail(APPD_EINVAL);  // cut out of range
    if (upload_schedule(t, G, chunk_start, items) != hipSuccess) return hip_status(hipErrorUnknown);
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

int appd_debug_write_counts_batched(const float* W, int mode, float* M, int32_t* idx,
                                    uint32_t* counts, const appd_batch_plan* plan, void* ws,
                                    void* stream) {
    if (!counts || !plan_ok(plan, ws)) return fail(APPD_EINVAL);
    hipStream_t s = (hipStream_t)stream;
    const appd::WriteCount on{counts, M, idx}, off{nullptr, nullptr, nullptr};
    hipError_t e = appd::run_zero(counts, (size_t)plan->total_nn * 4, s);
    if (e == hipSuccess) e = appd::set_write_count_batched(on, s);
    if (e == hipSuccess) e = appd::set_write_count_persist(on, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(APPD_EHIP);
    }
    const int rc = appd_forward_batched(W, mode, M, idx, nullptr, plan, ws, stream);
    e = hipStreamSynchronize(s);
    const hipError_t e_off1 = appd::set_write_count_batched(off, s);
    const hipError_t e_off2 = appd::set_write_count_persist(off, s);
    const hipError_t e_sync = hipStreamSynchronize(s);
    if (rc != APPD_OK) return rc;
    if (e != hipSuccess || e_off1 != hipSuccess || e_off2 != hipSuccess || e_sync != hipSuccess) {
        (void)hipGetLastError();
        return fail(APPD_EHIP);
    }
    return ok();
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
    // dX needs no clearing: the chain's first launch writes every entry
    hipError_t e = appd::run_zero(t.gedge, 4 * (size_t)plan->total_n, s);
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
        e = appd::run_pairwise(X, t.xoff, t.offsets, t.ns, t.tile_start, 1, (int)(nt * (nt + 1) / 2),
                               d, W, s);
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
    // dX needs no clearing: the chain's first launch writes every entry
    hipError_t e = appd::run_zero(t.gedge, 4 * (size_t)n, s);
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
