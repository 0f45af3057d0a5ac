// Write-count check of the fills (appd_debug_write_counts): Algorithm 4's
// calculation and copy assigns every entry of M (and here of idx) once.  While
// a translation unit's copy of c_write_count holds a counter array, every
// store of output elements adds 1 (M) or 0x10000 (idx) to the counters of the
// elements it writes, so an entry stored exactly once reads 0x00010001.  The
// switch is a constant read once per kernel: with it off a store site costs
// one uniform branch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace appd {

struct WriteCount {
    uint32_t* counts;    // one counter per output element, or null (off)
    const float* M;      // the outputs the counters index
    const int32_t* idx;
};

// One copy per translation unit (no relocatable device code): each unit with
// a fill sets its own through its set_write_count_* function.
static __constant__ WriteCount c_write_count = {nullptr, nullptr, nullptr};

__device__ __forceinline__ void count_writes(const float* p, int k) {
    uint32_t* c = c_write_count.counts;
    if (c) {
        const size_t e = (size_t)(p - c_write_count.M);
        for (int q = 0; q < k; ++q) atomicAdd(c + e + q, 1u);
    }
}

__device__ __forceinline__ void count_writes(const int32_t* p, int k) {
    uint32_t* c = c_write_count.counts;
    if (c) {
        const size_t e = (size_t)(p - c_write_count.idx);
        for (int q = 0; q < k; ++q) atomicAdd(c + e + q, 0x10000u);
    }
}

// Host setters, one per translation unit that stores outputs (stream-ordered).
hipError_t set_write_count_single(const WriteCount& wc, hipStream_t s);
hipError_t set_write_count_batched(const WriteCount& wc, hipStream_t s);
hipError_t set_write_count_persist(const WriteCount& wc, hipStream_t s);

}  // namespace appd
