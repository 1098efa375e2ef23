// Small device helpers shared by the kernel files of libdfamin.
#pragma once

#include "dfamin_internal.h"

namespace dfamin {
namespace {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Multiply-xorshift mixing of 32-bit words into a 64-bit hash.
__device__ __forceinline__ uint64_t mix_step(uint64_t h, uint32_t w) {
    h ^= w;
    h *= 0x9E3779B97F4A7C15ull;
    h ^= h >> 32;
    return h;
}
__device__ __forceinline__ uint64_t mix_final(uint64_t h) {
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 32;
    return h;
}
constexpr uint64_t kHashSeed = 0x6A09E667F3BCC909ull;

__device__ __forceinline__ size_t global_tid() {
    return static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
}
__device__ __forceinline__ size_t grid_stride() {
    return static_cast<size_t>(gridDim.x) * blockDim.x;
}

// Workgroup sum of per-thread values, added with one atomic per workgroup to
// one of kSpread counters (consecutive workgroups use different lines).
// Every thread of the workgroup must call it.
// The tiles (of `tile` states, covering n states) that this workgroup
// handles, as first, end and step.  Workgroups are dispatched to the 8 XCDs
// round-robin; with a grid that is a multiple of 8, each XCD takes one
// contiguous eighth of the tiles, so in a union (whose transitions stay
// inside each operand) the gathers of an XCD stay inside one operand, a
// footprint half as large for its L2.  Other grids stride over all tiles.
struct TileRange {
    size_t first, end, step;
};

__device__ __forceinline__ TileRange xcd_tiles(size_t n, size_t tile) {
    const size_t tiles = (n + tile - 1) / tile;
    TileRange t{blockIdx.x, tiles, gridDim.x};
    if (gridDim.x % 8 == 0) {
        const size_t x = blockIdx.x % 8;
        t.first = tiles * x / 8 + blockIdx.x / 8;
        t.end = tiles * (x + 1) / 8;
        t.step = gridDim.x / 8;
    }
    return t;
}

template <uint32_t NT = kBlock>  // threads of the workgroup
__device__ __forceinline__ void wg_add_spread(uint32_t *counters, int word, uint32_t v) {
    __shared__ uint32_t part[NT / 64];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    __syncthreads();
    if (lane_id() == 0) part[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < static_cast<int>(NT / 64); ++w) s += part[w];
        if (s) atomicAdd(counters + (blockIdx.x % kSpread) * kSpreadStride + word, s);
    }
}

// Sets *flag = 1 (a plain store: every writer stores the same value) if any
// active lane has `pred`; skips the store once the flag reads as set.
__device__ __forceinline__ void wave_set_flag(uint32_t *flag, bool pred) {
    const unsigned long long m = __ballot(pred);
    if (m == 0) return;
    const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
    if (static_cast<int>(lane_id()) == leader && *flag == 0u) *flag = 1u;
}

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long v) {
    uint32_t lo = static_cast<uint32_t>(v), hi = static_cast<uint32_t>(v >> 32);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        lo |= __shfl_xor(lo, d, 64);
        hi |= __shfl_xor(hi, d, 64);
    }
    return (static_cast<unsigned long long>(hi) << 32) | lo;
}


__device__ __forceinline__ bool rows_equal(const uint32_t *__restrict__ sig, size_t W, size_t a,
                                           size_t b) {
    const uint32_t *ra = sig + a * W;
    const uint32_t *rb = sig + b * W;
    for (size_t i = 0; i < W; ++i)
        if (ra[i] != rb[i]) return false;
    return true;
}

// The columns a kernel reads, resolved once per thread: the column list
// does not change during a launch, and holding the pointers in registers
// keeps the compiler from reloading the list after every store.
template <int KC>
struct ColPtrs {
    const uint32_t *c[KC > 0 ? KC : 1];
    __device__ __forceinline__ ColPtrs(const uint32_t *cols, const uint32_t *colmap, size_t N) {
#pragma unroll
        for (int j = 0; j < KC; ++j) c[j] = cols + static_cast<size_t>(colmap[j]) * N;
    }
};

// Marks block `id` as having two or more members after round r.
__device__ __forceinline__ void mark_multi(uint32_t *multi, uint32_t id, uint32_t tag) {
    if (multi[id] != tag) multi[id] = tag;
}

// Sets the summary bits of the groups holding a changed state, from a wave's
// changed-id mask (states first .. first + 63, first a multiple of 64).
__device__ __forceinline__ void set_summary(unsigned long long *sum, size_t first,
                                            unsigned long long cm) {
    constexpr uint32_t G = 1u << kSumShift;  // states per bit
    unsigned long long bits = 0;
    if constexpr (G >= 64) {
        bits = cm ? 1ull : 0ull;
    } else {
#pragma unroll
        for (uint32_t g = 0; g < 64 / G; ++g)
            if ((cm >> (g * G)) & ((1ull << G) - 1ull)) bits |= 1ull << g;
    }
    if (bits) atomicOr(sum + (first >> kSumWordShift), bits << ((first >> kSumShift) & 63));
}

// Whether state t's group is marked in a summary.
__device__ __forceinline__ bool summary_bit(const unsigned long long *sum, uint32_t t) {
    return ((sum[t >> kSumWordShift] >> ((t >> kSumShift) & 63)) & 1ull) != 0;
}

}  // namespace
}  // namespace dfamin
