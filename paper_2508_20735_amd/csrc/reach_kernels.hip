// Reachability from the start state (breadth-first search) and the
// sub-automaton of the reachable states, for minimisation restricted to the
// reachable part (the usual minimal DFA; the paper itself prunes nothing,
// Section 2).
//
// The search keeps a visited bitmap (one bit per state) and two frontier
// queues.  A frontier of at most kNarrowCap / k states is expanded inside one
// workgroup, level after level, with both queues in LDS (long thin searches,
// such as chains, then cost no launch per level); a larger frontier is
// expanded by a grid-wide launch per level, appending with one atomic per
// wave.  Every state enters a queue once, so both loops end.
#include "device_common.h"

namespace dfamin {
namespace {

constexpr uint32_t kNarrowThreads = 1024;
constexpr uint32_t kNarrowCap = 4096;  // LDS queue entries (two queues: 32 KB)

// Sets t's visited bit; true if this call set it.
__device__ __forceinline__ bool visit(unsigned long long *visited, uint32_t t) {
    const unsigned long long bit = 1ull << (t & 63);
    unsigned long long *w = visited + (t >> 6);
    if (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit) return false;
    return (atomicOr(w, bit) & bit) == 0;
}

// *err = 1 if some target is >= n (every later step indexes with targets).
__global__ __launch_bounds__(kBlock) void k_check_targets(const uint32_t *__restrict__ delta,
                                                          uint64_t total, uint32_t n,
                                                          uint32_t *err) {
    bool bad = false;
    for (uint64_t i = global_tid(); i < total; i += grid_stride()) bad |= delta[i] >= n;
    wave_set_flag(err, bad);
}

__global__ void k_bfs_init(ReachArgs a, uint32_t start) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    a.visited[start >> 6] |= 1ull << (start & 63);
    a.qa[0] = start;
    a.sizes[0] = 1;
    a.sizes[1] = 0;
}

// One workgroup: expands levels while the frontier times k fits kNarrowCap,
// then leaves the frontier in qa / sizes[0].
__global__ __launch_bounds__(kNarrowThreads) void k_bfs_narrow(ReachArgs a) {
    __shared__ uint32_t buf[2][kNarrowCap];
    __shared__ uint32_t sz[2];
    const uint32_t tx = threadIdx.x;
    const uint32_t k = a.k;
    uint32_t s = a.sizes[0];
    if (static_cast<uint64_t>(s) * k > kNarrowCap) return;  // the host checked; stay safe
    for (uint32_t i = tx; i < s; i += kNarrowThreads) buf[0][i] = a.qa[i];
    if (tx == 0) sz[0] = s;
    __syncthreads();
    uint32_t cur = 0;
    for (;;) {
        s = sz[cur];
        // uniform: every thread read the same size after the barrier
        if (s == 0 || static_cast<uint64_t>(s) * k > kNarrowCap) break;
        const uint32_t nxt = cur ^ 1u;
        if (tx == 0) sz[nxt] = 0;
        __syncthreads();
        const uint32_t work = s * k;
        for (uint32_t i = tx; i < work; i += kNarrowThreads) {
            const uint32_t q = buf[cur][i / k];
            const uint32_t t = a.delta[static_cast<size_t>(q) * k + (i % k)];
            // at most one entry per (state, letter) pair: pos < s * k <= kNarrowCap
            if (visit(a.visited, t)) buf[nxt][atomicAdd(&sz[nxt], 1u)] = t;
        }
        __syncthreads();
        cur = nxt;
    }
    s = sz[cur];
    for (uint32_t i = tx; i < s; i += kNarrowThreads) a.qa[i] = buf[cur][i];
    if (tx == 0) a.sizes[0] = s;
}

// One level over a large frontier: qa (sizes[0] entries) -> qb (sizes[1]).
__global__ __launch_bounds__(kBlock) void k_bfs_wide(ReachArgs a) {
    const uint64_t work = static_cast<uint64_t>(a.sizes[0]) * a.k;
    const uint32_t lane = lane_id();
    for (uint64_t base = static_cast<uint64_t>(blockIdx.x) * kBlock; base < work;
         base += static_cast<uint64_t>(gridDim.x) * kBlock) {
        const uint64_t i = base + threadIdx.x;
        bool fresh = false;
        uint32_t t = 0;
        if (i < work) {
            const uint32_t q = a.qa[i / a.k];
            t = a.delta[static_cast<size_t>(q) * a.k + (i % a.k)];
            fresh = visit(a.visited, t);
        }
        const unsigned long long m = __ballot(fresh);
        if (m == 0) continue;
        const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
        uint32_t pos = 0;
        if (static_cast<int>(lane) == leader) pos = atomicAdd(a.sizes + 1, static_cast<uint32_t>(__popcll(m)));
        pos = __shfl(pos, leader, 64);
        if (fresh) {
            const unsigned long long below = lane ? (m & ((1ull << lane) - 1ull)) : 0ull;
            a.qb[pos + static_cast<uint32_t>(__popcll(below))] = t;
        }
    }
}

__global__ void k_bfs_next(uint32_t *sizes) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sizes[0] = sizes[1];
        sizes[1] = 0;
    }
}

// flags[q] = q for reachable q, all ones otherwise (the input of the dense
// numbering, which numbers the states with flags[q] == q).
__global__ __launch_bounds__(kBlock) void k_reach_flags(const unsigned long long *visited, size_t n,
                                                        uint32_t *flags) {
    for (size_t q = global_tid(); q < n; q += grid_stride())
        flags[q] = ((visited[q >> 6] >> (q & 63)) & 1ull) ? static_cast<uint32_t>(q) : ~0u;
}

// Sub-automaton: row i is the reachable state orig[i], targets renumbered.
__global__ __launch_bounds__(kBlock) void k_sub_dfa(const uint32_t *__restrict__ delta,
                                                    const uint8_t *__restrict__ acc, uint32_t k,
                                                    const uint32_t *__restrict__ orig,
                                                    const uint32_t *__restrict__ dense,
                                                    const uint32_t *m_dev,
                                                    uint32_t *__restrict__ sub_delta,
                                                    uint8_t *__restrict__ sub_acc) {
    const uint64_t m = *m_dev;
    const uint64_t work = m * k;
    for (uint64_t i = global_tid(); i < work; i += grid_stride()) {
        const uint64_t row = i / k;
        const uint32_t q = orig[row];
        sub_delta[i] = dense[delta[static_cast<size_t>(q) * k + (i % k)]];
        if (i % k == 0) sub_acc[row] = acc[q];
    }
}

// block_out[q] = orig[sub_block[dense[q]]] for reachable q, kUnreachable
// otherwise (sub_block is canonical, and dense keeps the original order, so
// the result is the smallest reachable state of the block).
__global__ __launch_bounds__(kBlock) void k_reach_expand(const unsigned long long *visited,
                                                         size_t n, const uint32_t *dense,
                                                         const uint32_t *orig,
                                                         const uint32_t *sub_block,
                                                         uint32_t *block_out) {
    for (size_t q = global_tid(); q < n; q += grid_stride()) {
        const bool r = (visited[q >> 6] >> (q & 63)) & 1ull;
        block_out[q] = r ? orig[sub_block[dense[q]]] : 0xFFFFFFFFu;
    }
}

unsigned grid_of(uint64_t work, unsigned cap = 8192) {
    uint64_t g = (work + kBlock - 1) / kBlock;
    if (g == 0) g = 1;
    if (g > cap) g = cap;
    return static_cast<unsigned>(g);
}

}  // namespace

void launch_check_targets(const uint32_t *delta, uint64_t total, uint32_t n, uint32_t *err,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_check_targets, dim3(grid_of(total)), dim3(kBlock), 0, s, delta, total, n,
                       err);
}

void launch_bfs_init(const ReachArgs &a, uint32_t start, hipStream_t s) {
    hipLaunchKernelGGL(k_bfs_init, dim3(1), dim3(64), 0, s, a, start);
}

void launch_bfs_narrow(const ReachArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_bfs_narrow, dim3(1), dim3(kNarrowThreads), 0, s, a);
}

void launch_bfs_wide(const ReachArgs &a, uint32_t frontier, hipStream_t s) {
    hipLaunchKernelGGL(k_bfs_wide, dim3(grid_of(static_cast<uint64_t>(frontier) * a.k)),
                       dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_bfs_next, dim3(1), dim3(64), 0, s, a.sizes);
}

uint32_t bfs_narrow_cap() { return kNarrowCap; }

void launch_reach_flags(const unsigned long long *visited, size_t n, uint32_t *flags,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_reach_flags, dim3(grid_of(n)), dim3(kBlock), 0, s, visited, n, flags);
}

void launch_sub_dfa(const uint32_t *delta, const uint8_t *acc, uint32_t k, const uint32_t *orig,
                    const uint32_t *dense, const uint32_t *m_dev, uint32_t m_host,
                    uint32_t *sub_delta, uint8_t *sub_acc, hipStream_t s) {
    hipLaunchKernelGGL(k_sub_dfa, dim3(grid_of(static_cast<uint64_t>(m_host) * k)), dim3(kBlock),
                       0, s, delta, acc, k, orig, dense, m_dev, sub_delta, sub_acc);
}

void launch_reach_expand(const unsigned long long *visited, size_t n, const uint32_t *dense,
                         const uint32_t *orig, const uint32_t *sub_block, uint32_t *block_out,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_reach_expand, dim3(grid_of(n)), dim3(kBlock), 0, s, visited, n, dense,
                       orig, sub_block, block_out);
}

}  // namespace dfamin
