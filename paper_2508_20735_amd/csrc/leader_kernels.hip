// Leader-based partition refinement (naivePR, Section 3.2, Algorithm 2) on
// the GPU.
//
// Every block is named by its smallest state, its leader.  The initial
// leaders are the smallest accepting and the smallest rejecting state.  One
// round is three launches:
//   k_leader_elect  every state q that is not a leader compares, letter by
//                   letter, the block of delta(q, a) with the block of
//                   delta(block[q], a).  The first difference separates q:
//                   its bit is set in the round's per-wave mask, and q is
//                   offered as the leader of the states leaving block[q] by a
//                   64-bit atomicMin of (round tag | q).  The smallest
//                   separated state wins, so ids stay canonical; the tag
//                   decreases with the round, so a slot written in an earlier
//                   round loses to any offer of the current one and the slots
//                   are never cleared.  Offers are first reduced per
//                   workgroup in a small LDS table (a block split by many
//                   states costs one global atomic per workgroup, not one per
//                   state).
//   k_leader_move   separated states take the elected leader as their block;
//                   each elected leader is one new block.  The test of the
//                   elect kernel used the partition the round started from,
//                   so moving a state never changes another state's test of
//                   the same round.
//   k_leader_end    one workgroup: the round counter and the stop tests (no
//                   separated state: stable; the start states of an
//                   equivalence split; the round budget).
// A leader never differs from itself, so states with block[q] == q (among
// them every singleton block) cost one coalesced read per round.
#include <hip/hip_cooperative_groups.h>

#include "device_common.h"

namespace dfamin {
namespace {

constexpr uint32_t kElectSlots = kBlock;  // LDS election table per workgroup
constexpr uint32_t kElectProbes = 8;
constexpr uint32_t kNoKey = 0xFFFFFFFFu;
constexpr unsigned kLeaderGridCap = 2048;  // 8 workgroups per CU on 256 CUs

__host__ __device__ inline unsigned leader_grid(size_t N) {
    const size_t g = (N + kBlock - 1) / kBlock;
    return static_cast<unsigned>(g == 0 ? 1 : (g < kLeaderGridCap ? g : kLeaderGridCap));
}

// lead[0] = smallest accepting state, lead[1] = smallest rejecting state
// (both preset to kNoKey); bits of accbits at or beyond N are ignored.
__global__ __launch_bounds__(kBlock) void k_class_leaders(const unsigned long long *accbits,
                                                          size_t N, uint32_t *lead) {
    __shared__ uint32_t red[2][kBlock / 64];
    const size_t words = (N + 63) / 64;
    uint32_t mf = kNoKey, mr = kNoKey;
    for (size_t w = global_tid(); w < words; w += grid_stride()) {
        const unsigned long long m = accbits[w];
        const unsigned tail = static_cast<unsigned>(N - w * 64);
        const unsigned long long valid = tail >= 64 ? ~0ull : ((1ull << tail) - 1ull);
        const unsigned long long f = m & valid, r = ~m & valid;
        if (f) mf = min(mf, static_cast<uint32_t>(w * 64 + __ffsll(f) - 1));
        if (r) mr = min(mr, static_cast<uint32_t>(w * 64 + __ffsll(r) - 1));
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        mf = min(mf, static_cast<uint32_t>(__shfl_xor(mf, d, 64)));
        mr = min(mr, static_cast<uint32_t>(__shfl_xor(mr, d, 64)));
    }
    if (lane_id() == 0) {
        red[0][threadIdx.x / 64] = mf;
        red[1][threadIdx.x / 64] = mr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            mf = min(mf, red[0][w]);
            mr = min(mr, red[1][w]);
        }
        if (mf != kNoKey) atomicMin(lead + 0, mf);
        if (mr != kNoKey) atomicMin(lead + 1, mr);
    }
}

__global__ __launch_bounds__(kBlock) void k_leader_blocks(const unsigned long long *accbits,
                                                          size_t N, const uint32_t *lead,
                                                          uint32_t *__restrict__ block) {
    const uint32_t lf = lead[0], lr = lead[1];
    for (size_t q = global_tid(); q < N; q += grid_stride())
        block[q] = ((accbits[q >> 6] >> (q & 63)) & 1ull) ? lf : lr;
}

__device__ __forceinline__ void leader_elect_body(const LeaderArgs &a) {
    __shared__ uint32_t ckey[kElectSlots];
    __shared__ uint32_t cmin[kElectSlots];
    if (a.ctl->done) return;
    const uint32_t r = a.ctl->round;
    const unsigned long long tag = static_cast<unsigned long long>(0xFFFFFFFFu - r) << 32;
    const uint32_t tx = threadIdx.x;
    const size_t N = a.N;
    const uint32_t *__restrict__ block = a.block;
    ckey[tx] = kNoKey;
    cmin[tx] = kNoKey;
    __syncthreads();
    uint32_t processed = 0;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kBlock; base < N;
         base += static_cast<size_t>(gridDim.x) * kBlock) {
        const size_t q = base + tx;
        bool sep = false;
        uint32_t b = 0;
        if (q < N) {
            b = block[q];
            if (b != q) {
                ++processed;
                // four letters per step: the eight gathers of a step are
                // independent, the early exit is taken between steps
                for (uint32_t j = 0; j < a.k_eff && !sep; j += 4) {
                    uint32_t tq[4] = {0, 0, 0, 0}, tb[4] = {0, 0, 0, 0};
#pragma unroll
                    for (uint32_t i = 0; i < 4; ++i) {
                        if (j + i < a.k_eff) {
                            const uint32_t *col = a.cols + static_cast<size_t>(a.colmap[j + i]) * N;
                            tq[i] = col[q];
                            tb[i] = col[b];
                        }
                    }
#pragma unroll
                    for (uint32_t i = 0; i < 4; ++i)
                        if (j + i < a.k_eff && block[tq[i]] != block[tb[i]]) sep = true;
                }
            }
        }
        const unsigned long long m = __ballot(sep);
        const size_t first = base + (tx & ~63u);
        if (lane_id() == 0 && first < N) a.moved[first >> 6] = m;
        if (sep) {
            uint32_t s = (b * 0x9E3779B1u) >> 24;  // 8 bits: kElectSlots == 256
            bool cached = false;
            for (uint32_t p = 0; p < kElectProbes; ++p) {
                const uint32_t prev = atomicCAS(ckey + s, kNoKey, b);
                if (prev == kNoKey || prev == b) {
                    atomicMin(cmin + s, static_cast<uint32_t>(q));
                    cached = true;
                    break;
                }
                s = (s + 1) & (kElectSlots - 1);
            }
            if (!cached) atomicMin(a.new_leader + b, tag | static_cast<uint32_t>(q));
        }
    }
    __syncthreads();
    if (ckey[tx] != kNoKey) atomicMin(a.new_leader + ckey[tx], tag | cmin[tx]);
    wg_add_spread(a.counters, 2, processed);
}

__device__ __forceinline__ void leader_move_body(const LeaderArgs &a) {
    if (a.ctl->done) return;
    const size_t N = a.N;
    uint32_t fresh = 0, moved = 0;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kBlock; base < N;
         base += static_cast<size_t>(gridDim.x) * kBlock) {
        const size_t q = base + threadIdx.x;
        const size_t first = base + (threadIdx.x & ~63u);
        const unsigned long long m = first < N ? a.moved[first >> 6] : 0ull;
        // bits of states >= N are never set by the elect kernel
        if ((m >> lane_id()) & 1ull) {
            const uint32_t b = a.block[q];
            const uint32_t l = static_cast<uint32_t>(a.new_leader[b]);
            a.block[q] = l;
            ++moved;
            if (l == q) ++fresh;
        }
    }
    wg_add_spread(a.counters, 0, fresh);
    wg_add_spread(a.counters, 1, moved);
}

__device__ __forceinline__ void leader_end_body(RoundCtl *ctl, const uint32_t *block,
                                                uint32_t *counters) {
    __shared__ uint32_t red[3][kBlock / 64];
    if (ctl->done) return;
    uint32_t v[3] = {0, 0, 0};
    for (uint32_t i = threadIdx.x; i < kSpread; i += kBlock)
        for (int w = 0; w < 3; ++w) {
            v[w] += counters[i * kSpreadStride + w];
            counters[i * kSpreadStride + w] = 0;
        }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        for (int w = 0; w < 3; ++w) v[w] += __shfl_xor(v[w], d, 64);
    if (lane_id() == 0)
        for (int w = 0; w < 3; ++w) red[w][threadIdx.x / 64] = v[w];
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 0; w < 3; ++w) {
        v[w] = 0;
        for (int i = 0; i < kBlock / 64; ++i) v[w] += red[w][i];
    }
    const uint32_t fresh = v[0], moved = v[1], processed = v[2];
    const uint32_t r = ctl->round;
    ctl->last_gain = fresh;
    ctl->last_active = processed;
    ctl->last_claims = moved;
    ctl->active_sum += processed;
    ctl->active_hist[r % kActiveHist] = processed;
    ctl->gain_hist[r % kActiveHist] = fresh;
    if (moved == 0) {
        ctl->stable = 1;
        ctl->done = 1;
    } else {
        ctl->changing += 1;
        ctl->prev_count += fresh;
    }
    if (ctl->check_eq && block[ctl->eq_a] != block[ctl->eq_b]) {
        ctl->separated = 1;
        ctl->done = 1;
    }
    ctl->round = r + 1;
    if (!ctl->done && ctl->max_rounds && r + 1 >= ctl->max_rounds) {
        ctl->limit = 1;
        ctl->done = 1;
    }
}

__global__ __launch_bounds__(kBlock) void k_leader_elect(LeaderArgs a) { leader_elect_body(a); }

__global__ __launch_bounds__(kBlock) void k_leader_move(LeaderArgs a) { leader_move_body(a); }

__global__ __launch_bounds__(kBlock) void k_leader_end(RoundCtl *ctl, const uint32_t *block,
                                                       uint32_t *counters) {
    leader_end_body(ctl, block, counters);
}

// Persistent loop of leader rounds: the three phases of a round separated by
// grid barriers inside one cooperative launch (the stop flag is read right
// after a barrier and written only by the last phase, so every workgroup
// takes the same barriers).
__global__ __launch_bounds__(kBlock) void k_leader_persistent(LeaderArgs a, uint32_t rounds) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    for (uint32_t i = 0; i < rounds; ++i) {
        if (__hip_atomic_load(&a.ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        leader_elect_body(a);
        grid.sync();
        leader_move_body(a);
        grid.sync();
        if (blockIdx.x == 0) leader_end_body(a.ctl, a.block, a.counters);
        grid.sync();
    }
}

}  // namespace

hipError_t launch_leader_persistent(const LeaderArgs &a, uint32_t rounds, hipStream_t s) {
    const void *kernel = reinterpret_cast<const void *>(&k_leader_persistent);
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0);
    if (e != hipSuccess) return e;
    if (cus <= 0 || per_cu <= 0) return hipErrorInvalidConfiguration;
    // at most one workgroup per CU: a grid barrier's cost grows with the
    // workgroups that arrive at it
    const unsigned fit = static_cast<unsigned>(cus) *
                         std::min(static_cast<unsigned>(per_cu), kPersistentGroupsPerCu);
    const unsigned grid = std::min(leader_grid(a.N), fit);
    LeaderArgs args_a = a;
    void *args[] = {&args_a, &rounds};
    return hipLaunchCooperativeKernel(kernel, dim3(grid), dim3(kBlock), args, 0, s);
}

void launch_leader_init(const unsigned long long *accbits, size_t N, uint32_t *lead,
                        uint32_t *block, hipStream_t s) {
    const unsigned g = leader_grid(N);
    launch_kernel(k_class_leaders, dim3(leader_grid((N + 63) / 64)), dim3(kBlock), 0, s,
                       accbits, N, lead);
    launch_kernel(k_leader_blocks, dim3(g), dim3(kBlock), 0, s, accbits, N, lead, block);
}

void launch_leader_elect(const LeaderArgs &a, hipStream_t s) {
    launch_kernel(k_leader_elect, dim3(leader_grid(a.N)), dim3(kBlock), 0, s, a);
}

void launch_leader_move(const LeaderArgs &a, hipStream_t s) {
    launch_kernel(k_leader_move, dim3(leader_grid(a.N)), dim3(kBlock), 0, s, a);
}

void launch_leader_end(const LeaderArgs &a, hipStream_t s) {
    launch_kernel(k_leader_end, dim3(1), dim3(kBlock), 0, s, a.ctl, a.block, a.counters);
}

void launch_leader_round(const LeaderArgs &a, hipStream_t s) {
    launch_leader_elect(a, s);
    launch_leader_move(a, s);
    launch_leader_end(a, s);
}

}  // namespace dfamin
