// Breadth-first exploration of the synchronous product of two DFAs on the
// GPU: the naive Hopcroft-Karp of Section 4, where the relation is the plain
// set of reached pairs (a lock-free hash set of 64-bit keys p << 32 | q in
// HBM) and no transitive closure is maintained.  Inclusion L(A) <= L(B) is
// refuted by a reached pair with p accepting in A and q rejecting in B;
// equivalence by a pair with exactly one accepting side.
#include "device_common.h"

namespace dfamin {
namespace {

constexpr unsigned long long kEmpty = ~0ull;

// Slot of a pair key: the library's key mixing over its two 32-bit halves.
__device__ __forceinline__ uint64_t pair_hash(uint64_t key) {
    return mix_final(mix_step(mix_step(kHashSeed, static_cast<uint32_t>(key >> 32)),
                              static_cast<uint32_t>(key)));
}

// Inserts key; returns true if it was not present.
__device__ __forceinline__ bool set_insert(unsigned long long *tab, uint64_t mask,
                                           unsigned long long key) {
    uint64_t s = pair_hash(key) & mask;
    for (;;) {
        unsigned long long e = __hip_atomic_load(tab + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (e == key) return false;
        if (e == kEmpty) {
            const unsigned long long prev = atomicCAS(tab + s, kEmpty, key);
            if (prev == kEmpty) return true;
            if (prev == key) return false;
        }
        s = (s + 1) & mask;
    }
}

__global__ __launch_bounds__(kBlock) void k_product_level(ProductArgs a) {
    const uint32_t lane = __lane_id();
    const uint64_t mask = a.visited_cap - 1;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
         i < a.frontier_size; i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const unsigned long long key = a.frontier[i];
        const uint32_t p = static_cast<uint32_t>(key >> 32), q = static_cast<uint32_t>(key);
        const bool fa = a.accA[p] != 0, fb = a.accB[q] != 0;
        const bool bad = a.mode == 0 ? (fa && !fb) : (fa != fb);
        if (bad) atomicOr(a.bad, 1u);
        for (uint32_t c = 0; c < a.k; ++c) {
            const unsigned long long nk =
                (static_cast<unsigned long long>(a.dA[static_cast<size_t>(p) * a.k + c]) << 32) |
                a.dB[static_cast<size_t>(q) * a.k + c];
            const bool fresh = !bad && set_insert(a.visited, mask, nk);
            // wave-aggregated append to the next frontier
            const unsigned long long m = __ballot(fresh);
            if (m == 0) continue;
            const int leader = __ffsll(m) - 1;
            uint32_t base = 0;
            if (static_cast<int>(lane) == leader) base = atomicAdd(a.next_size, static_cast<uint32_t>(__popcll(m)));
            base = __shfl(base, leader, 64);
            if (fresh) {
                const unsigned long long below = lane ? (m & ((1ull << lane) - 1ull)) : 0ull;
                const uint32_t slot = base + static_cast<uint32_t>(__popcll(below));
                if (slot < a.next_cap)
                    a.next[slot] = nk;
                else
                    atomicOr(a.overflow, 1u);
            }
        }
    }
}

// One workgroup expands levels while the frontier times k fits an LDS queue
// (long, thin explorations such as C_n's products, where a launch and a host
// round trip per level would dominate).  Pairs are inserted into the same
// HBM set as by k_product_level; new pairs go to the other LDS queue.  Stops
// when the frontier is empty, a refuting pair is expanded, the next
// frontier could overflow the queue, or after max_levels levels; the
// remaining frontier is written back to `frontier`, and out[] receives
// (frontier size, pairs added, levels expanded, refuted).
__global__ __launch_bounds__(kProductNarrowThreads) void k_product_narrow(ProductArgs a,
                                                                          uint32_t max_levels,
                                                                          uint32_t *out) {
    __shared__ unsigned long long buf[2][kProductNarrowCap];
    __shared__ uint32_t next_size, refuted;
    const uint32_t tx = threadIdx.x;
    const uint64_t mask = a.visited_cap - 1;
    unsigned long long *frontier = const_cast<unsigned long long *>(a.frontier);
    uint32_t s = a.frontier_size;
    if (static_cast<uint64_t>(s) * a.k > kProductNarrowCap) return;  // the host checked; stay safe
    for (uint32_t i = tx; i < s; i += kProductNarrowThreads) buf[0][i] = frontier[i];
    if (tx == 0) refuted = 0;
    uint32_t cur = 0, levels = 0, added = 0;
    for (;;) {
        if (s == 0 || levels == max_levels || static_cast<uint64_t>(s) * a.k > kProductNarrowCap) break;
        if (tx == 0) next_size = 0;
        __syncthreads();
        for (uint32_t i = tx; i < s; i += kProductNarrowThreads) {
            const unsigned long long key = buf[cur][i];
            const uint32_t p = static_cast<uint32_t>(key >> 32), q = static_cast<uint32_t>(key);
            const bool fa = a.accA[p] != 0, fb = a.accB[q] != 0;
            const bool bad = a.mode == 0 ? (fa && !fb) : (fa != fb);
            if (bad) {
                refuted = 1;
                continue;
            }
            for (uint32_t c = 0; c < a.k; ++c) {
                const unsigned long long nk =
                    (static_cast<unsigned long long>(a.dA[static_cast<size_t>(p) * a.k + c]) << 32) |
                    a.dB[static_cast<size_t>(q) * a.k + c];
                // at most s * k fresh pairs <= kProductNarrowCap
                if (set_insert(a.visited, mask, nk)) buf[cur ^ 1u][atomicAdd(&next_size, 1u)] = nk;
            }
        }
        __syncthreads();
        ++levels;
        const uint32_t n = next_size;
        const bool stop = refuted != 0;
        __syncthreads();  // every thread has read next_size before it is reset
        if (stop) {
            s = 0;
            if (tx == 0) out[3] = 1;
            break;
        }
        added += n;
        s = n;
        cur ^= 1u;
    }
    for (uint32_t i = tx; i < s; i += kProductNarrowThreads) frontier[i] = buf[cur][i];
    if (tx == 0) {
        out[0] = s;
        out[1] = added;
        out[2] = levels;
    }
}

__global__ __launch_bounds__(kBlock) void k_visited_clear(unsigned long long *tab, uint64_t cap) {
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < cap;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        tab[i] = kEmpty;
}

__global__ void k_visited_insert_start(unsigned long long *tab, uint64_t cap,
                                       unsigned long long key) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_insert(tab, cap - 1, key);
}

__global__ __launch_bounds__(kBlock) void k_rehash(const unsigned long long *old_tab, uint64_t old_cap,
                                                    unsigned long long *new_tab, uint64_t new_cap) {
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < old_cap;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const unsigned long long key = old_tab[i];
        if (key != kEmpty) set_insert(new_tab, new_cap - 1, key);
    }
}

unsigned grid_for(size_t work) {
    size_t g = (work + kBlock - 1) / kBlock;
    if (g == 0) g = 1;
    if (g > (1u << 20)) g = 1u << 20;
    return static_cast<unsigned>(g);
}

}  // namespace

void launch_product_level(const ProductArgs &a, hipStream_t s) {
    launch_kernel(k_product_level, dim3(grid_for(a.frontier_size)), dim3(kBlock), 0, s, a);
}

void launch_product_narrow(const ProductArgs &a, uint32_t max_levels, uint32_t *out,
                           hipStream_t s) {
    launch_kernel(k_product_narrow, dim3(1), dim3(kProductNarrowThreads), 0, s, a, max_levels,
                       out);
}

void launch_visited_clear(unsigned long long *visited, uint64_t cap, hipStream_t s) {
    launch_kernel(k_visited_clear, dim3(grid_for(cap)), dim3(kBlock), 0, s, visited, cap);
}

void launch_visited_insert_start(unsigned long long *visited, uint64_t cap,
                                 unsigned long long key, hipStream_t s) {
    launch_kernel(k_visited_insert_start, dim3(1), dim3(64), 0, s, visited, cap, key);
}

void launch_rehash(const unsigned long long *old_tab, uint64_t old_cap,
                   unsigned long long *new_tab, uint64_t new_cap, hipStream_t s) {
    launch_kernel(k_rehash, dim3(grid_for(old_cap)), dim3(kBlock), 0, s, old_tab, old_cap,
                       new_tab, new_cap);
}

}  // namespace dfamin
