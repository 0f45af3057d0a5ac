// Host-side declarations shared by the translation units of libappd.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace appd {

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Carved single-graph workspace (device pointers).
struct SingleWs {
    int32_t* order;
    int32_t* parent;
    int32_t* pos;
    uint64_t* ek;
    uint16_t* blk_sp;
    uint16_t* blk_slot;
    uint64_t* blk_gap;
};

size_t single_workspace_bytes(int n);
SingleWs carve_single(void* ws, int n);
hipError_t run_single(const float* W, int n, int mode, float* M, int32_t* idx,
                      const SingleWs& w, hipStream_t s);

}  // namespace appd
