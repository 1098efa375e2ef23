// Reachability from the start state (breadth-first search) and the
// sub-automaton of the reachable states, for minimisation restricted to the
// reachable part (the usual minimal DFA; the paper itself prunes nothing,
// Section 2).
//
// The search keeps a mark byte per state (0 unvisited, 1 settled, 2 / 3 in
// the frontier of an even / odd level) and a frontier queue.  A frontier of
// at most kNarrowCap / k states is expanded inside one workgroup, level after
// level, with both queues in LDS (long thin searches, such as chains, then
// cost no launch per level; a visited bitmap with atomics dedupes within the
// workgroup).  A larger frontier is expanded by dense levels: every state is
// scanned, the frontier ones expand, and unvisited targets get the next
// level's mark by plain stores (several writers store the same value), so
// wide levels use no atomics on the visited set.  Every state is marked once,
// so both loops end.
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
    a.mark[start] = 1;
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
            // at most one entry per (state, letter) pair: pos < s * k <= kNarrowCap;
            // states settled by dense levels carry a mark, not a bit
            if (a.mark[t] == 0 && visit(a.visited, t)) {
                a.mark[t] = 1;
                buf[nxt][atomicAdd(&sz[nxt], 1u)] = t;
            }
        }
        __syncthreads();
        cur = nxt;
    }
    s = sz[cur];
    for (uint32_t i = tx; i < s; i += kNarrowThreads) a.qa[i] = buf[cur][i];
    if (tx == 0) a.sizes[0] = s;
}

// Queue -> marks: the listed states become the frontier of a dense level.
__global__ __launch_bounds__(kBlock) void k_bfs_list_to_marks(ReachArgs a, uint8_t f) {
    const uint32_t s = a.sizes[0];
    for (size_t i = global_tid(); i < s; i += grid_stride()) a.mark[a.qa[i]] = f;
}

// One dense level: states marked f expand (unvisited targets get nf) and
// settle.  sizes[1] += number of marks stored (an upper bound of the new
// states: two lanes may store the same target; zero iff none was stored).
__global__ __launch_bounds__(kBlock) void k_bfs_dense(ReachArgs a, uint8_t f, uint8_t nf) {
    uint32_t stored = 0;
    for (size_t q = global_tid(); q < a.n; q += grid_stride()) {
        if (a.mark[q] != f) continue;
        const uint32_t *row = a.delta + q * a.k;
        // letters in groups of 8: the row entries, then their marks, are
        // loaded together before any store
        for (uint32_t j0 = 0; j0 < a.k; j0 += 8) {
            const uint32_t m = a.k - j0 < 8 ? a.k - j0 : 8;
            uint32_t t[8];
            uint8_t mk[8];
#pragma unroll
            for (uint32_t j = 0; j < 8; ++j) t[j] = j < m ? row[j0 + j] : static_cast<uint32_t>(q);
#pragma unroll
            for (uint32_t j = 0; j < 8; ++j) mk[j] = a.mark[t[j]];
#pragma unroll
            for (uint32_t j = 0; j < 8; ++j)
                if (j < m && mk[j] == 0) {
                    a.mark[t[j]] = nf;
                    ++stored;
                }
        }
        a.mark[q] = 1;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) stored += __shfl_xor(stored, d, 64);
    if (lane_id() == 0 && stored) atomicAdd(a.sizes + 1, stored);
}

// Marks -> queue: the states marked f settle and are listed in qa (one
// append atomic per wave); sizes[0] = their number.
__global__ __launch_bounds__(kBlock) void k_bfs_marks_to_list(ReachArgs a, uint8_t f) {
    const uint32_t lane = lane_id();
    for (size_t base = static_cast<size_t>(blockIdx.x) * kBlock; base < a.n;
         base += static_cast<size_t>(gridDim.x) * kBlock) {
        const size_t q = base + threadIdx.x;
        const bool hit = q < a.n && a.mark[q] == f;
        const unsigned long long m = __ballot(hit);
        if (m == 0) continue;
        const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
        uint32_t pos = 0;
        if (static_cast<int>(lane) == leader)
            pos = atomicAdd(a.sizes, static_cast<uint32_t>(__popcll(m)));
        pos = __shfl(pos, leader, 64);
        if (hit) {
            const unsigned long long below = lane ? (m & ((1ull << lane) - 1ull)) : 0ull;
            a.qa[pos + static_cast<uint32_t>(__popcll(below))] = static_cast<uint32_t>(q);
            a.mark[q] = 1;
        }
    }
}

__global__ void k_bfs_set(uint32_t *sizes, uint32_t i0, uint32_t v0, uint32_t i1, uint32_t v1) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sizes[i0] = v0;
        sizes[i1] = v1;
    }
}

// flags[q] = q for reachable q, all ones otherwise (the input of the dense
// numbering, which numbers the states with flags[q] == q).
__global__ __launch_bounds__(kBlock) void k_reach_flags(const uint8_t *mark, size_t n,
                                                        uint32_t *flags) {
    for (size_t q = global_tid(); q < n; q += grid_stride())
        flags[q] = mark[q] ? static_cast<uint32_t>(q) : ~0u;
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
__global__ __launch_bounds__(kBlock) void k_reach_expand(const uint8_t *mark, size_t n,
                                                         const uint32_t *dense,
                                                         const uint32_t *orig,
                                                         const uint32_t *sub_block,
                                                         uint32_t *block_out) {
    for (size_t q = global_tid(); q < n; q += grid_stride())
        block_out[q] = mark[q] ? orig[sub_block[dense[q]]] : 0xFFFFFFFFu;
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
    launch_kernel(k_check_targets, dim3(grid_of(total)), dim3(kBlock), 0, s, delta, total, n,
                       err);
}

void launch_bfs_init(const ReachArgs &a, uint32_t start, hipStream_t s) {
    launch_kernel(k_bfs_init, dim3(1), dim3(64), 0, s, a, start);
}

void launch_bfs_narrow(const ReachArgs &a, hipStream_t s) {
    launch_kernel(k_bfs_narrow, dim3(1), dim3(kNarrowThreads), 0, s, a);
}

void launch_bfs_list_to_marks(const ReachArgs &a, uint32_t count, uint8_t f, hipStream_t s) {
    launch_kernel(k_bfs_list_to_marks, dim3(grid_of(count)), dim3(kBlock), 0, s, a, f);
}

void launch_bfs_dense(const ReachArgs &a, uint8_t f, uint8_t nf, hipStream_t s) {
    launch_kernel(k_bfs_set, dim3(1), dim3(64), 0, s, a.sizes, 1u, 0u, 1u, 0u);
    launch_kernel(k_bfs_dense, dim3(grid_of(a.n)), dim3(kBlock), 0, s, a, f, nf);
}

void launch_bfs_marks_to_list(const ReachArgs &a, uint8_t f, hipStream_t s) {
    launch_kernel(k_bfs_set, dim3(1), dim3(64), 0, s, a.sizes, 0u, 0u, 0u, 0u);
    launch_kernel(k_bfs_marks_to_list, dim3(grid_of(a.n)), dim3(kBlock), 0, s, a, f);
}

uint32_t bfs_narrow_cap() { return kNarrowCap; }

void launch_reach_flags(const uint8_t *mark, size_t n, uint32_t *flags, hipStream_t s) {
    launch_kernel(k_reach_flags, dim3(grid_of(n)), dim3(kBlock), 0, s, mark, n, flags);
}

void launch_sub_dfa(const uint32_t *delta, const uint8_t *acc, uint32_t k, const uint32_t *orig,
                    const uint32_t *dense, const uint32_t *m_dev, uint32_t m_host,
                    uint32_t *sub_delta, uint8_t *sub_acc, hipStream_t s) {
    launch_kernel(k_sub_dfa, dim3(grid_of(static_cast<uint64_t>(m_host) * k)), dim3(kBlock),
                       0, s, delta, acc, k, orig, dense, m_dev, sub_delta, sub_acc);
}

void launch_reach_expand(const uint8_t *mark, size_t n, const uint32_t *dense,
                         const uint32_t *orig, const uint32_t *sub_block, uint32_t *block_out,
                         hipStream_t s) {
    launch_kernel(k_reach_expand, dim3(grid_of(n)), dim3(kBlock), 0, s, mark, n, dense,
                       orig, sub_block, block_out);
}

}  // namespace dfamin
