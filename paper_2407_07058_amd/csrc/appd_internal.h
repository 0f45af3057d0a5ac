// Host-side declarations shared by the translation units of libappd.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace appd {

void set_last_error(int code);

// Launch timer (appd_timer_start): events around the launches of the selected
// kernel, recorded on the launch stream.  Off by default: one relaxed load.
bool timer_wants(const char* name);
void timer_begin(const char* name, hipStream_t s);
void timer_end(hipStream_t s);

// Launch log (environment variable APPD_LOG, read once): one stderr line per
// kernel launch.
bool log_on();
void log_launch(const char* name, hipStream_t s);

// Input checks of the single-graph forward (environment variable
// APPD_VALIDATE, read at each call): the validation pass or-s its flags into a
// per-GPU record that appd_sync reports and clears.
bool validate_requested();
hipError_t enqueue_input_check(const float* W, int n, hipStream_t s);
#define APPD_LAUNCH(name, stream, ...)                        \
    do {                                                      \
        if (::appd::log_on()) ::appd::log_launch(name, (stream)); \
        const bool appd_timed_ = ::appd::timer_wants(name);   \
        if (appd_timed_) ::appd::timer_begin(name, (stream)); \
        __VA_ARGS__;                                          \
        if (appd_timed_) ::appd::timer_end(stream);           \
    } while (0)

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Carved single-graph workspace (device pointers).
struct SingleWs {
    int32_t* order;
    int32_t* parent;
    int32_t* pos;
    uint64_t* ek;
    uint16_t* blk_sp;     // per column block: attachment positions of the columns, sorted
    uint16_t* blk_slot;   // slot of each column in that order
    uint32_t* blk_code;   // slot codes (order-preserving stand-ins for the gap keys)
    float* blk_dM;        // decoded weight of each slot's gap key (entry 0: diagonal)
    int32_t* blk_dI;      // decoded flat index of each slot's gap key
    uint64_t* blk_sorted; // the block's gap keys in ascending order
    void* tree_ws;  // scratch of the parallel tree
};

size_t tree_workspace_bytes(int n);
struct PrimOut;
hipError_t run_tree_parallel(const float* W, int n, int mode, const PrimOut& out, void* tws,
                             hipStream_t s);
hipError_t tree_stats(const void* tws, int n, int32_t* passes, int32_t* rounds, int32_t* fallback,
                      int32_t* tables, hipStream_t s);
hipError_t run_linkage(const float* W, int n, int mode, const PrimOut& out, void* tws, double* Z,
                       hipStream_t s);
bool valid_mode(int mode);
int parallel_tree_min_n();

size_t single_workspace_bytes(int n);
SingleWs carve_single(void* ws, int n);
hipError_t run_tree(const float* W, int n, int mode, const SingleWs& w, hipStream_t s);
hipError_t run_fill(int n, int mode, float* M, int32_t* idx, const SingleWs& w, hipStream_t s);
hipError_t run_single(const float* W, int n, int mode, float* M, int32_t* idx,
                      const SingleWs& w, hipStream_t s);

// ---- batched path
constexpr int kBatchClasses = 6;
constexpr int kClassMaxN[kBatchClasses] = {64, 128, 256, 512, 1024, 2048};

struct BatchTree {
    int32_t* order;
    uint64_t* ek;
    int32_t* pos;
    int32_t* parent;
};

// Per-graph column-block tables of the coded fill (graphs with n > 256): the
// entries of graph g's block b sit at noff[g] + 1024 * b + k, k < the block's
// column count (see fill_prep_block).
struct BatchBlk {
    uint16_t* sp;
    uint16_t* slot;
    uint32_t* code;
    float* dM;
    int32_t* dI;
    uint64_t* sorted;
};

struct BatchPlan {
    const int32_t* perm;         // [G] graph ids, n descending (device)
    const int64_t* noff;         // [G] start of graph g's O(n) arrays (device, by graph id)
    const int32_t* chunk_start;  // [G] first fill item of perm[i] within its class (device)
    const int32_t* rstart;       // [G] sum of n over perm[0 .. i) (device)
    const int32_t* rgraph;       // [total_n] i of row r, rows in perm order (device)
    uint64_t* lists;             // candidate lists of the Boruvka classes, K per vertex
    int32_t* tstats;             // [G] per graph, by graph id: how its tree was found
    int class_tree[kBatchClasses];
    int class_vertices[kBatchClasses];
    int split_vertices;
    int class_first[kBatchClasses];
    int class_count[kBatchClasses];
    int class_chunks[kBatchClasses];
    int class_rows[kBatchClasses];
    int class_threads[kBatchClasses];
    int streams;
    int split_count;   // largest class: graphs launched first on their own (0: no split)
    int split_chunks;  // their fill work items
    // the persistent form (see appd_persist.hip)
    int persistent;
    int persist_items;
    int stagger;  // the other classes' streams start after the largest class's pass
    int num_graphs;
    int total_n;
    const uint2* items;  // [persist_items] work queue (device)
    int* ctr;            // [2 + 2 G] queue head, rows done and tree done per graph, abort (device)
};

int batch_class_of(int n);
hipError_t launch_btree(int c, int first, int count, int rows_in_class, int mode, const float* W,
                        const int64_t* offsets, const int32_t* ns, const BatchPlan& plan,
                        const BatchTree& tree, const BatchBlk& blk, uint64_t* lists,
                        hipStream_t s, hipEvent_t after_pass = nullptr);
bool batch_threads_ok(int c, int threads);
hipError_t run_batched(const float* W, const int64_t* offsets, const int32_t* ns,
                       const BatchPlan& plan, const BatchTree& tree, const BatchBlk& blk,
                       int mode, float* M, int32_t* idx, hipStream_t s);
hipError_t run_persistent(const float* W, const int64_t* offsets, const int32_t* ns,
                          const BatchPlan& plan, const BatchTree& tree, const BatchBlk& blk,
                          int mode, float* M, int32_t* idx, hipStream_t s);
// Persistent form: rows per pass item (one per wave of its workgroup) and the
// class limit.
constexpr int kPersistThreads = 512;
constexpr int kPersistMaxN = 1024;
// Work item words: x = type << 30 | first row (pass) or graph position (tree,
// fill); y (fill) = first row | row count << 16.
constexpr uint32_t kItemPass = 0u, kItemTree = 1u, kItemFill = 2u;

// Per-GPU status record read and cleared by appd_sync: validation flags of
// checked forwards, and kStatusWaitTimeout.
uint32_t* device_status_word();
constexpr uint32_t kStatusWaitTimeout = 0x100u;

// ---- points / gradients
hipError_t run_pairwise(const float* X, const int64_t* xoff, const int64_t* offsets,
                        const int32_t* ns, const int32_t* tile_start, int num_graphs,
                        int total_tiles, int d, float* W, hipStream_t s);
hipError_t run_edge_grad(const float* G, const int32_t* idx, const int64_t* offsets,
                         const int64_t* noff, const int32_t* ns, const int32_t* parent,
                         const int32_t* chunk_start, int num_graphs, int total_chunks,
                         int rows_per_wg, int max_n, float* gedge, hipStream_t s);
hipError_t run_chain(const float* X, const int64_t* xoff, const float* W, const int64_t* offsets,
                     const int64_t* noff, const int32_t* ns, const int32_t* parent,
                     float* gedge, const int32_t* vstart, int num_graphs, int total_vblocks,
                     int d, float* dX, hipStream_t s);
hipError_t run_zero(void* p, size_t bytes, hipStream_t s);
hipError_t run_scale_offsets(const int64_t* noff, int num_graphs, int d, int64_t* xoff,
                             hipStream_t s);
hipError_t run_single_table(int n, int32_t* ns, int64_t* offsets, int64_t* noff,
                            int32_t* tile_start, int32_t* gchunk_start, int32_t* vstart,
                            hipStream_t s);
hipError_t run_edge_to_w(const float* gedge, const int32_t* parent, const int64_t* offsets,
                         const int64_t* noff, const int32_t* ns, const int32_t* vstart,
                         int num_graphs, int total_vblocks, float* dW, hipStream_t s);
int pairwise_tile();
int pairwise_max_d();
constexpr int kGradRows = 32;
constexpr int kChainThreads = 256;

}  // namespace appd
