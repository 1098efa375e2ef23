// Batched refinement of small DFAs inside single workgroups.
//
// One workgroup refines one job at a time: a DFA (minimisation) or the
// disjoint union of two DFAs (equivalence), with the whole signature loop of
// Section 3.3 (Algorithm 4: signature = own block id and the successors'
// block ids; equal signatures form the next blocks; stop when the block
// count does not grow) on the device.  Block ids and the grouping table sit
// in LDS, so every successor-id gather and every probe is an LDS access;
// rounds are separated by workgroup barriers, with no launch and no host
// round trip per round.  The transition rows are read from the caller's
// row-major arrays (L2-resident for DFAs of this size).  Workgroups take jobs
// from a counter, largest first.
//
// Ids inside a round are the index of the state that first claimed its
// signature's slot; the final ids are made canonical (smallest member) in
// LDS.  The round counts are those of plain signature rounds from the
// initial partition {F, Q \ F}, as in the segmented path; a pair stops at the
// round that separates its start states.
#include "device_common.h"

namespace dfamin {
namespace {

constexpr uint32_t kEmptySlot = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t small_table_slots(uint32_t n) {
    uint32_t t = 64;
    while (t < 2 * n) t <<= 1;
    return t;
}

// Local state i of a job: its row and the offset of its targets.
struct JobView {
    const uint32_t *da, *db;
    const uint8_t *aa, *ab;
    uint32_t na, n, k;
    __device__ __forceinline__ const uint32_t *row(uint32_t i) const {
        return i < na ? da + static_cast<size_t>(i) * k : db + static_cast<size_t>(i - na) * k;
    }
    __device__ __forceinline__ uint32_t base(uint32_t i) const { return i < na ? 0u : na; }
    __device__ __forceinline__ bool accepting(uint32_t i) const {
        return (i < na ? aa[i] : ab[i - na]) != 0;
    }
};

// Signature of local state i from the ids in `cur` (LDS): w0 and w[0..k).
// A target outside its DFA sets `bad` and reads state 0 of that DFA instead
// (the call then fails; no access leaves the job's arrays).
__device__ __forceinline__ void small_key(const JobView &v, const uint16_t *cur, uint32_t i,
                                          uint32_t &w0, uint32_t *w, bool &bad) {
    const uint32_t *r = v.row(i);
    const uint32_t b = v.base(i);
    const uint32_t lim = i < v.na ? v.na : v.n - v.na;
    w0 = cur[i];
    uint32_t t[kSmallMaxK];
#pragma unroll
    for (uint32_t a = 0; a < kSmallMaxK; ++a)
        if (a < v.k) t[a] = r[a];
#pragma unroll
    for (uint32_t a = 0; a < kSmallMaxK; ++a)
        if (a < v.k) {
            if (t[a] >= lim) {
                bad = true;
                t[a] = 0;
            }
            w[a] = cur[b + t[a]];
        }
}

// Whether local state j's signature is (w0, w).  j already passed through
// small_key in this round, so its targets are in range or `bad` is set;
// they are clamped the same way here.
__device__ __forceinline__ bool small_key_equal(const JobView &v, const uint16_t *cur, uint32_t j,
                                                uint32_t w0, const uint32_t *w) {
    if (cur[j] != w0) return false;
    const uint32_t *r = v.row(j);
    const uint32_t b = v.base(j);
    const uint32_t lim = j < v.na ? v.na : v.n - v.na;
    for (uint32_t a = 0; a < v.k; ++a) {
        const uint32_t t = r[a];
        if (cur[b + (t < lim ? t : 0u)] != w[a]) return false;
    }
    return true;
}

__device__ __forceinline__ uint32_t wg_sum(uint32_t v, uint32_t *red) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x / 64] = v;
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (uint32_t w = 0; w < kSmallThreads / 64; ++w) s += red[w];
    return s;
}

__global__ __launch_bounds__(kSmallThreads) void k_small_refine(const SmallJob *__restrict__ jobs,
                                                                uint32_t njobs, uint32_t *next_job,
                                                                uint32_t *out_blocks,
                                                                SmallResult *results,
                                                                uint32_t max_rounds,
                                                                uint32_t *err) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t red[kSmallThreads / 64];
    __shared__ uint32_t job_id;
    const uint32_t tx = threadIdx.x;
    for (;;) {
        if (tx == 0) job_id = atomicAdd(next_job, 1u);
        __syncthreads();
        const uint32_t j = job_id;
        __syncthreads();  // every thread has read job_id before it changes
        if (j >= njobs) return;
        const SmallJob J = jobs[j];
        const JobView v{J.delta_a, J.delta_b, J.acc_a, J.acc_b, J.na, J.na + J.nb, J.k};
        const uint32_t n = v.n;
        const uint32_t T = small_table_slots(n);
        // LDS: table (T words), then two id arrays of n halves
        uint32_t *table = reinterpret_cast<uint32_t *>(lds);
        uint16_t *ida = reinterpret_cast<uint16_t *>(table + T);
        uint16_t *idb = ida + ((n + 1) & ~1u);
        // initial partition {F, Q \ F}: labels 1 / 0
        uint32_t has_acc = 0, has_rej = 0;
        for (uint32_t i = tx; i < n; i += kSmallThreads) {
            const bool f = v.accepting(i);
            ida[i] = f ? 1 : 0;
            has_acc |= f ? 1u : 0u;
            has_rej |= f ? 0u : 1u;
        }
        uint32_t prev = (wg_sum(has_acc, red) ? 1u : 0u);
        prev += (wg_sum(has_rej, red) ? 1u : 0u);
        uint16_t *cur = ida, *nxt = idb;
        uint32_t round = 0, changing = 0, limit = 0;
        bool bad = false;
        for (;;) {
            for (uint32_t s = tx; s < T; s += kSmallThreads) table[s] = kEmptySlot;
            __syncthreads();
            uint32_t claims = 0;
            for (uint32_t i = tx; i < n; i += kSmallThreads) {
                uint32_t w0, w[kSmallMaxK];
                small_key(v, cur, i, w0, w, bad);
                uint64_t h = mix_step(kHashSeed, w0);
#pragma unroll
                for (uint32_t a = 0; a < kSmallMaxK; ++a)
                    if (a < v.k) h = mix_step(h, w[a]);
                h = mix_final(h);
                const uint32_t tag = static_cast<uint32_t>(h >> 48);
                const uint32_t want = (tag << 16) | i;
                uint32_t s = static_cast<uint32_t>(h) & (T - 1);
                uint32_t id;
                for (;;) {
                    uint32_t e = __hip_atomic_load(table + s, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (e == kEmptySlot) {
                        const uint32_t prevs = atomicCAS(table + s, kEmptySlot, want);
                        if (prevs == kEmptySlot) {
                            id = i;
                            ++claims;
                            break;
                        }
                        e = prevs;
                    }
                    if ((e >> 16) == tag && small_key_equal(v, cur, e & 0xFFFFu, w0, w)) {
                        id = e & 0xFFFFu;
                        break;
                    }
                    s = (s + 1) & (T - 1);
                }
                nxt[i] = static_cast<uint16_t>(id);
            }
            const uint32_t count = wg_sum(claims, red);  // (its barriers order nxt too)
            ++round;
            // stable: nxt holds the same partition as cur, with state ids
            if (count == prev) break;
            prev = count;
            ++changing;
            uint16_t *t = cur;
            cur = nxt;
            nxt = t;
            // a pair is decided once its start states are separated (the
            // refinement never merges them again)
            if (J.nb && cur[J.start_a] != cur[J.na + J.start_b]) {
                nxt = cur;
                break;
            }
            if (max_rounds && round >= max_rounds) {
                limit = 1;
                nxt = cur;  // the last round's ids
                break;
            }
        }
        if (__syncthreads_or(bad) && tx == 0) *err = 1u;
        // canonical ids (smallest member) in the table's words; the ids in
        // nxt are state indices (< n)
        const uint16_t *fin = nxt;
        uint32_t *minof = table;
        for (uint32_t i = tx; i < n; i += kSmallThreads) minof[i] = kEmptySlot;
        __syncthreads();
        for (uint32_t i = tx; i < n; i += kSmallThreads) atomicMin(minof + fin[i], i);
        __syncthreads();
        if (J.nb == 0) {
            uint32_t *out = out_blocks + J.out;
            for (uint32_t i = tx; i < n; i += kSmallThreads) out[i] = minof[fin[i]];
        }
        if (tx == 0) {
            SmallResult r;
            r.num_blocks = prev;
            r.rounds = round;
            r.changing = changing;
            r.verdict = J.nb ? (fin[J.start_a] == fin[J.na + J.start_b] ? 1u : 0u) : 0u;
            r.limit = limit;
            results[J.index] = r;
        }
        __syncthreads();
    }
}

__global__ void k_small_counter_reset(uint32_t *next_job, uint32_t *err) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *next_job = 0;
        *err = 0;
    }
}

}  // namespace

uint32_t small_refine_lds_bytes(uint32_t n) {
    uint32_t t = 64;
    while (t < 2 * n) t <<= 1;
    return t * 4u + 2u * ((n + 1) & ~1u) * 2u;
}

int small_refine_max_groups(uint32_t lds_bytes, int device_cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_small_refine, kSmallThreads,
                                                     lds_bytes) != hipSuccess ||
        per_cu <= 0)
        return 0;
    return per_cu * device_cus;
}

void launch_small_refine(const SmallJob *jobs, uint32_t njobs, uint32_t groups, uint32_t lds_bytes,
                         uint32_t *next_job, uint32_t *out_blocks, SmallResult *results,
                         uint32_t max_rounds, uint32_t *err, hipStream_t s) {
    launch_kernel(k_small_counter_reset, dim3(1), dim3(64), 0, s, next_job, err);
    launch_kernel(k_small_refine, dim3(groups), dim3(kSmallThreads), lds_bytes, s, jobs, njobs,
                  next_job, out_blocks, results, max_rounds, err);
}

}  // namespace dfamin
