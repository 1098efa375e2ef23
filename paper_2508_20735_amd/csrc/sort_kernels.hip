// Sort-based grouping of the refined states (the grouping of sortPR, Section
// 3.3, Algorithm 4): instead of the hash table, the round's refined states
// are compacted (in increasing state order), their (64-bit key hash, state)
// pairs are sorted by a stable least-significant-digit radix sort, and every
// run of equal hashes is split into its distinct keys by comparing rows.
// Because the sort is stable and its input is in state order, the first
// state of a key in its run is the smallest state with that key: it becomes
// the block's id (ids stay canonical, and an unsplit block keeps its id).
// Equal hashes of different keys (collisions) only make a run longer: each
// state takes the first state of its run with an equal row, so grouping
// stays exact.
//
// Radix sort: 8 passes of 8-bit digits.  A pass is a per-tile digit
// histogram, an exclusive scan of the digit-major histogram table, and a
// stable scatter in which each tile walks its items stripe by stripe; within
// a stripe a wave ranks its lanes by digit with eight ballots.  All launch
// sizes depend on N only (the count m of refined states is read on the
// device), so the round can be replayed from a graph.
#include <algorithm>

#include "device_common.h"

namespace dfamin {
namespace {

constexpr uint32_t kSortThreads = 256;
constexpr uint32_t kSortItems = 16;
constexpr uint32_t kSortTile = kSortThreads * kSortItems;  // elements per tile
constexpr uint32_t kRadixBits = 8;
constexpr uint32_t kRadixBins = 1u << kRadixBits;
constexpr uint32_t kScanBlock = kSortTile;  // entries per block of the generic scans
constexpr uint32_t kCompactTile = 64 * 64;  // states per compaction tile (one wave, 64 words)

static_assert(kSortThreads == kRadixBins, "one thread per digit value");

struct SumOp {
    __device__ static uint32_t id() { return 0u; }
    __device__ static uint32_t op(uint32_t a, uint32_t b) { return a + b; }
};
struct MaxOp {
    __device__ static uint32_t id() { return 0u; }
    __device__ static uint32_t op(uint32_t a, uint32_t b) { return a > b ? a : b; }
};

// Scan of one value per thread across the workgroup (256 threads): the
// inclusive and the exclusive result of this thread.
template <class Op>
__device__ __forceinline__ void block_scan(uint32_t v, uint32_t *wtot, uint32_t &incl,
                                           uint32_t &excl) {
    const uint32_t lane = lane_id(), w = threadIdx.x / 64;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (static_cast<int>(lane) >= d) x = Op::op(x, y);
    }
    uint32_t xe = __shfl_up(x, 1, 64);
    if (lane == 0) xe = Op::id();
    if (lane == 63) wtot[w] = x;
    __syncthreads();
    uint32_t carry = Op::id();
    for (uint32_t i = 0; i < w; ++i) carry = Op::op(carry, wtot[i]);
    __syncthreads();
    incl = Op::op(carry, x);
    excl = Op::op(carry, xe);
}

// ---- generic three-step scan over `len` entries (len read from *len_dev
// when given, else len_host) ----

// partials[b] = reduction of block b (kScanBlock entries).
template <class Op>
__global__ __launch_bounds__(kSortThreads) void k_scan_reduce(const uint32_t *in, uint64_t len_host,
                                                              const uint32_t *len_dev,
                                                              uint32_t *partials) {
    __shared__ uint32_t wtot[kSortThreads / 64];
    const uint64_t len = len_dev ? *len_dev : len_host;
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanBlock;
    uint32_t v = Op::id();
    for (uint32_t i = 0; i < kSortItems; ++i) {
        const uint64_t e = base + i * kSortThreads + threadIdx.x;
        if (e < len) v = Op::op(v, in[e]);
    }
    uint32_t incl, excl;
    block_scan<Op>(v, wtot, incl, excl);
    if (threadIdx.x == kSortThreads - 1) partials[blockIdx.x] = incl;
}

// Exclusive scan of nb partials in one workgroup (in place).
template <class Op>
__global__ __launch_bounds__(kSortThreads) void k_scan_partials_op(uint32_t *partials, uint32_t nb) {
    __shared__ uint32_t wtot[kSortThreads / 64];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = Op::id();
    __syncthreads();
    for (uint32_t base = 0; base < nb; base += kSortThreads) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < nb ? partials[i] : Op::id();
        uint32_t incl, excl;
        block_scan<Op>(v, wtot, incl, excl);
        const uint32_t c = carry;
        if (i < nb) partials[i] = Op::op(c, excl);
        __syncthreads();
        if (threadIdx.x == kSortThreads - 1) carry = Op::op(c, incl);
        __syncthreads();
    }
}

// In-place scan of each block, combined with its block's exclusive prefix.
template <class Op, bool kInclusive>
__global__ __launch_bounds__(kSortThreads) void k_scan_apply(uint32_t *data, uint64_t len_host,
                                                             const uint32_t *len_dev,
                                                             const uint32_t *partials) {
    __shared__ uint32_t wtot[kSortThreads / 64];
    __shared__ uint32_t carry;
    const uint64_t len = len_dev ? *len_dev : len_host;
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanBlock;
    if (base >= len) return;
    if (threadIdx.x == 0) carry = partials[blockIdx.x];
    __syncthreads();
    for (uint32_t i = 0; i < kSortItems; ++i) {
        const uint64_t e = base + i * kSortThreads + threadIdx.x;
        const uint32_t v = e < len ? data[e] : Op::id();
        uint32_t incl, excl;
        block_scan<Op>(v, wtot, incl, excl);
        const uint32_t c = carry;
        if (e < len) data[e] = Op::op(c, kInclusive ? incl : excl);
        __syncthreads();
        if (threadIdx.x == kSortThreads - 1) carry = Op::op(c, incl);
        __syncthreads();
    }
}

// ---- compaction of the refined states ----

// partials[tile] = refined states in the tile (one wave per tile, a word per lane).
__global__ __launch_bounds__(64) void k_compact_count(const unsigned long long *active, size_t N,
                                                      uint32_t *partials) {
    const size_t words = (N + 63) / 64;
    const size_t w = static_cast<size_t>(blockIdx.x) * 64 + lane_id();
    uint32_t c = w < words ? static_cast<uint32_t>(__popcll(active[w])) : 0u;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if (lane_id() == 0) partials[blockIdx.x] = c;
}

// After the exclusive scan of the tile counts: the (hash, state) pairs of the
// refined states in increasing state order; *m = their number.
__global__ __launch_bounds__(64) void k_compact_write(const unsigned long long *active, size_t N,
                                                      const uint64_t *hash,
                                                      const uint32_t *partials, uint32_t ntiles,
                                                      unsigned long long *keys, uint32_t *vals,
                                                      uint32_t *m) {
    const size_t words = (N + 63) / 64;
    const uint32_t lane = lane_id();
    const size_t w = static_cast<size_t>(blockIdx.x) * 64 + lane;
    unsigned long long bits = w < words ? active[w] : 0ull;
    const uint32_t c = static_cast<uint32_t>(__popcll(bits));
    uint32_t incl = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 64);
        if (static_cast<int>(lane) >= d) incl += y;
    }
    uint32_t pos = partials[blockIdx.x] + incl - c;
    while (bits) {
        const uint32_t b = static_cast<uint32_t>(__ffsll(bits) - 1);
        bits &= bits - 1;
        const size_t q = w * 64 + b;
        keys[pos] = hash[q];
        vals[pos] = static_cast<uint32_t>(q);
        ++pos;
    }
    if (blockIdx.x == ntiles - 1 && lane == 63) *m = partials[blockIdx.x] + incl;
}

// ---- radix sort passes ----

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const unsigned long long *keys,
                                                             const uint32_t *m_dev, uint32_t shift,
                                                             uint32_t *hist, uint32_t tiles) {
    __shared__ uint32_t h[kRadixBins];
    const uint32_t m = *m_dev;
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kSortTile;
    h[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i = 0; i < kSortItems; ++i) {
        const uint64_t e = base + i * kSortThreads + threadIdx.x;
        if (e < m) atomicAdd(h + ((keys[e] >> shift) & (kRadixBins - 1)), 1u);
    }
    __syncthreads();
    // digit-major: all tiles of digit 0, then digit 1, ... (tiles past m count 0)
    hist[static_cast<size_t>(threadIdx.x) * tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const unsigned long long *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
    unsigned long long *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
    const uint32_t *m_dev, uint32_t shift, const uint32_t *__restrict__ offsets, uint32_t tiles) {
    __shared__ uint32_t base[kRadixBins];
    __shared__ uint32_t wcnt[kSortThreads / 64][kRadixBins];
    const uint32_t m = *m_dev;
    const uint64_t tile0 = static_cast<uint64_t>(blockIdx.x) * kSortTile;
    if (tile0 >= m) return;
    const uint32_t tx = threadIdx.x, lane = lane_id(), w = tx / 64;
    base[tx] = offsets[static_cast<size_t>(tx) * tiles + blockIdx.x];
    for (uint32_t i = 0; i < kSortThreads / 64; ++i) wcnt[i][tx] = 0;
    __syncthreads();
    const unsigned long long lt = lane ? ((1ull << lane) - 1ull) : 0ull;
    for (uint32_t i = 0; i < kSortItems; ++i) {
        const uint64_t e = tile0 + i * kSortThreads + tx;
        const bool valid = e < m;
        const unsigned long long key = valid ? keys_in[e] : 0ull;
        const uint32_t val = valid ? vals_in[e] : 0u;
        const uint32_t d = static_cast<uint32_t>((key >> shift) & (kRadixBins - 1));
        // lanes of this wave with the same digit
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (uint32_t b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long ones = __ballot(valid && bit);
            peers &= bit ? ones : ~ones;
        }
        const uint32_t rank = static_cast<uint32_t>(__popcll(peers & lt));
        if (valid && rank == 0) wcnt[w][d] = static_cast<uint32_t>(__popcll(peers));
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + rank;
            for (uint32_t v = 0; v < w; ++v) pos += wcnt[v][d];
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (uint32_t v = 0; v < kSortThreads / 64; ++v) {
            add += wcnt[v][tx];
            wcnt[v][tx] = 0;
        }
        base[tx] += add;
        __syncthreads();
    }
}

// ---- runs and ids ----

// headpos[p] = p if the hash at p starts a run, else 0.
__global__ __launch_bounds__(kBlock) void k_run_heads(const unsigned long long *keys,
                                                     const uint32_t *m_dev, uint32_t *headpos) {
    const uint32_t m = *m_dev;
    for (size_t p = global_tid(); p < m; p += grid_stride())
        headpos[p] = (p == 0 || keys[p] != keys[p - 1]) ? static_cast<uint32_t>(p) : 0u;
}

struct AssignArgs {
    const uint32_t *vals;      // sorted states
    const uint32_t *runhead;   // position of each element's run head
    const uint32_t *m;
    const uint32_t *sig;
    uint32_t W;
    uint32_t *blockA, *blockB;
    uint32_t *multi;
    uint32_t *counters;
    const RoundCtl *ctl;
};

// Each state takes the first state of its run with an equal row as its id.
__global__ __launch_bounds__(kBlock) void k_sort_assign(AssignArgs a) {
    if (a.ctl->done) return;
    const uint32_t r = a.ctl->round;
    uint32_t *__restrict__ Y = (r & 1u) ? a.blockA : a.blockB;
    const uint32_t m = *a.m;
    uint32_t claims = 0;
    for (size_t p = global_tid(); p < m; p += grid_stride()) {
        const uint32_t q = a.vals[p];
        uint32_t id = q;
        bool joined = false;
        for (size_t j = a.runhead[p]; j < p; ++j) {
            const uint32_t c = a.vals[j];
            if (rows_equal(a.sig, a.W, q, c)) {
                id = c;
                joined = true;
                break;
            }
        }
        Y[q] = id;
        if (joined)
            mark_multi(a.multi, id, r + 1);
        else
            ++claims;
    }
    wg_add_spread(a.counters, 0, claims);
    wg_add_spread(a.counters, 3, claims);
}

// State order: changed-id bits and the counts the table kernels keep.
__global__ __launch_bounds__(kBlock) void k_sort_finish(const unsigned long long *active, size_t N,
                                                       uint32_t *blockA, uint32_t *blockB,
                                                       unsigned long long *chg,
                                                       unsigned long long *chg_sum,
                                                       uint32_t *counters, const RoundCtl *ctl) {
    if (ctl->done) return;
    const uint32_t r = ctl->round;
    const uint32_t *__restrict__ X = (r & 1u) ? blockB : blockA;
    const uint32_t *__restrict__ Y = (r & 1u) ? blockA : blockB;
    uint32_t idle = 0, changed = 0;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kBlock; base < N;
         base += static_cast<size_t>(gridDim.x) * kBlock) {
        const size_t q = base + threadIdx.x;
        const size_t first = base + (threadIdx.x & ~63u);
        const unsigned long long am = first < N ? active[first >> 6] : 0ull;
        const bool valid = q < N;
        const bool act = valid && ((am >> lane_id()) & 1ull);
        idle += (valid && !act) ? 1u : 0u;
        const bool ch = act && Y[q] != X[q];
        const unsigned long long cm = __ballot(ch);
        if (lane_id() == 0 && first < N) {
            chg[first >> 6] = cm;
            // the round's changed-id summary
            set_summary(chg_sum + (r & 1u) * summary_words(N), first, cm);
        }
        changed += ch ? 1u : 0u;
    }
    wg_add_spread(counters, 1, idle);
    wg_add_spread(counters, 2, changed);
}

unsigned grid_n(uint64_t work, unsigned cap = 8192) {
    uint64_t g = (work + kBlock - 1) / kBlock;
    if (g == 0) g = 1;
    if (g > cap) g = cap;
    return static_cast<unsigned>(g);
}

}  // namespace

SortPlan sort_plan(size_t N) {
    SortPlan s;
    s.sort_tiles = static_cast<uint32_t>((N + kSortTile - 1) / kSortTile);
    if (s.sort_tiles == 0) s.sort_tiles = 1;
    s.compact_tiles = static_cast<uint32_t>((N + kCompactTile - 1) / kCompactTile);
    if (s.compact_tiles == 0) s.compact_tiles = 1;
    const uint64_t hist_len = static_cast<uint64_t>(kRadixBins) * s.sort_tiles;
    s.hist_words = hist_len;
    s.hist_blocks = static_cast<uint32_t>((hist_len + kScanBlock - 1) / kScanBlock);
    s.run_blocks = static_cast<uint32_t>((N + kScanBlock - 1) / kScanBlock);
    if (s.run_blocks == 0) s.run_blocks = 1;
    s.partial_words = std::max<uint64_t>(
        {static_cast<uint64_t>(s.compact_tiles), s.hist_blocks, s.run_blocks}) + 1;
    return s;
}

void launch_sort_group(const RoundArgs &a, hipStream_t s) {
    const SortBuffers &b = a.sort;
    const SortPlan pl = sort_plan(a.N);
    // compaction of the refined states, in state order
    launch_kernel(k_compact_count, dim3(pl.compact_tiles), dim3(64), 0, s, a.active, a.N,
                       b.partials);
    launch_kernel(k_scan_partials_op<SumOp>, dim3(1), dim3(kSortThreads), 0, s, b.partials,
                       pl.compact_tiles);
    launch_kernel(k_compact_write, dim3(pl.compact_tiles), dim3(64), 0, s, a.active, a.N,
                       a.hash, b.partials, pl.compact_tiles, b.keys[0], b.vals[0], b.m);
    // stable radix sort by hash, 8 passes
    for (uint32_t pass = 0; pass < 64 / kRadixBits; ++pass) {
        const uint32_t in = pass & 1u, out = in ^ 1u;
        const uint32_t shift = pass * kRadixBits;
        launch_kernel(k_radix_hist, dim3(pl.sort_tiles), dim3(kSortThreads), 0, s, b.keys[in],
                           b.m, shift, b.hist, pl.sort_tiles);
        launch_kernel(k_scan_reduce<SumOp>, dim3(pl.hist_blocks), dim3(kSortThreads), 0, s,
                           b.hist, pl.hist_words, nullptr, b.partials);
        launch_kernel(k_scan_partials_op<SumOp>, dim3(1), dim3(kSortThreads), 0, s,
                           b.partials, pl.hist_blocks);
        launch_kernel((k_scan_apply<SumOp, false>), dim3(pl.hist_blocks), dim3(kSortThreads),
                           0, s, b.hist, pl.hist_words, nullptr, b.partials);
        launch_kernel(k_radix_scatter, dim3(pl.sort_tiles), dim3(kSortThreads), 0, s,
                           b.keys[in], b.vals[in], b.keys[out], b.vals[out], b.m, shift, b.hist,
                           pl.sort_tiles);
    }
    // runs of equal hashes: position of each element's run head
    launch_kernel(k_run_heads, dim3(grid_n(a.N)), dim3(kBlock), 0, s, b.keys[0], b.m,
                       b.runhead);
    launch_kernel(k_scan_reduce<MaxOp>, dim3(pl.run_blocks), dim3(kSortThreads), 0, s,
                       b.runhead, 0, b.m, b.partials);
    launch_kernel(k_scan_partials_op<MaxOp>, dim3(1), dim3(kSortThreads), 0, s, b.partials,
                       pl.run_blocks);
    launch_kernel((k_scan_apply<MaxOp, true>), dim3(pl.run_blocks), dim3(kSortThreads), 0, s,
                       b.runhead, 0, b.m, b.partials);
    const AssignArgs aa{b.vals[0], b.runhead, b.m,        a.sig,      a.k_eff + 1,
                        a.blockA,  a.blockB,  a.multi,    a.counters, a.ctl};
    launch_kernel(k_sort_assign, dim3(grid_n(a.N)), dim3(kBlock), 0, s, aa);
    launch_kernel(k_sort_finish, dim3(grid_n(a.N)), dim3(kBlock), 0, s, a.active, a.N,
                       a.blockA, a.blockB, a.chg, a.chg_sum, a.counters, a.ctl);
}

}  // namespace dfamin
