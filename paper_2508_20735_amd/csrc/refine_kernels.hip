// HIP kernels of the partition-refinement path for gfx950 (wave64).
//
// One refinement round (the signature rounds of Section 3.3, Algorithm 4,
// with grouping by hashing instead of sorting):
//   k_mark       bookkeeping of the states to refine: a block with one member
//                never splits again (singleton bits); once a round changed
//                few ids, only blocks with a member whose successor changed
//                id can split, and those blocks are marked ("touched").
//   k_signature  every refined state q writes its signature
//                  ( block[q], block[col_0[q]], ..., block[col_{k_eff-1}[q]] )
//                into a row of `sig` and a 64-bit hash of it.  Column reads are
//                coalesced (symbol-major layout); the block ids are gathers.
//                The other states keep their id.
//   k_insert     groups equal signatures.  A member whose key equals the key
//                of the state that holds its block's id keeps that id (a
//                direct compare, no table).  The others go through a
//                lock-free open-addressing table in HBM: the hash only picks
//                the slot and a 24-bit tag, keys are always compared in full,
//                so grouping is exact; the first state to claim a slot
//                becomes the id of every state with that signature.  The LDS
//                variant first groups the 256 states of a workgroup in an LDS
//                table, so only one state per distinct signature and
//                workgroup touches the HBM table.
//   k_round_end  one workgroup: the block count of the round (the states
//                that hold their block's id); an unchanged count means the
//                partition is stable (the block id leads the signature, so
//                each round refines the previous one).
// Rounds 0 and 1 can group by exact labels without a table (acceptance bit
// patterns, then packed pattern labels).  Block ids during the rounds are
// member states chosen by the hardware's atomic order; the final partition
// is renumbered canonically (smallest state of each block) once, by
// k_canon_min / k_canon_apply.
#include <hip/hip_cooperative_groups.h>

#include "device_common.h"

namespace dfamin {
namespace {

constexpr unsigned long long kEmptyPair = ~0ull;

// ---------------------------------------------------------------- ingest

// One thread per state: reads its row of delta, writes one entry per column.
__global__ __launch_bounds__(kBlock) void k_ingest(const uint32_t *__restrict__ delta, uint32_t n,
                                                    uint32_t k, uint32_t *__restrict__ cols,
                                                    size_t N, uint32_t offset, uint32_t toff,
                                                    uint32_t *err, uint32_t *nonid) {
    bool bad = false;
    unsigned long long moves = 0;  // letters 0..63 that move some state
    auto put = [&](size_t q, uint32_t a, uint32_t t) {
        bad |= t >= n;
        if (t != q) {
            if (a < 64)
                moves |= 1ull << a;
            else if (nonid[a] == 0u)
                nonid[a] = 1u;
        }
        cols[static_cast<size_t>(a) * N + offset + q] = t + toff;
    };
    // rows of a multiple of 4 letters at a 16-byte aligned address are read
    // 16 bytes at a time (uniform over the grid)
    if (k % 4 == 0 && (reinterpret_cast<uintptr_t>(delta) & 15u) == 0) {
        for (size_t q = global_tid(); q < n; q += grid_stride()) {
            const uint4 *row = reinterpret_cast<const uint4 *>(delta + q * k);
            for (uint32_t a = 0; a < k; a += 4) {
                const uint4 v = row[a / 4];
                put(q, a, v.x);
                put(q, a + 1, v.y);
                put(q, a + 2, v.z);
                put(q, a + 3, v.w);
            }
        }
    } else {
        for (size_t q = global_tid(); q < n; q += grid_stride()) {
            const uint32_t *row = delta + q * k;
            for (uint32_t a = 0; a < k; ++a) put(q, a, row[a]);
        }
    }
    wave_set_flag(err, bad);
    moves = wave_or64(moves);
    if (lane_id() == 0) {
        while (moves) {
            const int a = __ffsll(moves) - 1;
            moves &= moves - 1;
            if (nonid[a] == 0u) nonid[a] = 1u;
        }
    }
}

// Initial labels (accepting ? 1 : 0), packed acceptance bits, class flags.
__global__ __launch_bounds__(kBlock) void k_init_blocks(const uint8_t *__restrict__ acc, uint32_t n,
                                                         uint32_t offset,
                                                         uint32_t *__restrict__ block,
                                                         unsigned long long *accbits,
                                                         uint32_t *class_flags) {
    bool any_acc = false, any_rej = false;
    const bool aligned = (offset & 63u) == 0;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kBlock; base < n;
         base += static_cast<size_t>(gridDim.x) * kBlock) {
        const size_t q = base + threadIdx.x;
        const bool valid = q < n;
        const bool f = valid && acc[q] != 0;
        if (valid) block[offset + q] = f ? 1u : 0u;
        any_acc |= f;
        any_rej |= valid && !f;
        if (aligned) {
            const unsigned long long m = __ballot(f);
            const size_t first = base + (threadIdx.x & ~63u);
            if (lane_id() == 0 && first < n && m) accbits[(offset + first) >> 6] = m;
        } else if (f) {
            const size_t g = offset + q;
            atomicOr(accbits + (g >> 6), 1ull << (g & 63));
        }
    }
    wave_set_flag(class_flags + 0, any_acc);
    wave_set_flag(class_flags + 1, any_rej);
}

__global__ void k_ctl_reset(RoundCtl *ctl, const uint32_t *class_flags, uint32_t max_rounds,
                            uint32_t check_eq, uint32_t eq_a, uint32_t eq_b,
                            uint32_t pattern_first, uint32_t packed_second,
                            const uint32_t *init_count) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    RoundCtl c{};
    c.prev_count = init_count ? *init_count
                              : (class_flags[0] ? 1u : 0u) + (class_flags[1] ? 1u : 0u);
    c.max_rounds = max_rounds;
    c.check_eq = check_eq;
    c.eq_a = eq_a;
    c.eq_b = eq_b;
    c.pattern_first = pattern_first;
    c.packed_second = packed_second;
    // ids produced by label rounds are not state indices: the round after
    // them refines every state
    c.all_active_until = pattern_first + packed_second;
    c.full_until = c.all_active_until;
    *ctl = c;
}

__global__ void k_ctl_resume(RoundCtl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->done = 0;
}

__global__ void k_ctl_full(RoundCtl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->full_until = ctl->round;
}

// ---------------------------------------------------------------- round kernels

__device__ __forceinline__ unsigned long long load_entry(const unsigned long long *p, bool cached) {
    return cached ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT)
                  : __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Finds the slot holding q's signature or claims an empty one for it.
// Entry = (epoch:8 | tag:24) << 32 | representative; entries of older
// epochs count as empty.  Lock-free: a slot only ever changes from "empty" to
// a final value within an epoch, and every decision is confirmed by a CAS or
// by reading such a final value.  A cached read may show an older "empty"
// value; the CAS then fails and returns the value actually stored, which is
// examined next without reading the cache again.  The load factor stays
// <= 1/2, so the probe always reaches an empty slot.
__device__ __forceinline__ uint32_t find_or_claim(unsigned long long *table, uint64_t mask,
                                                  uint32_t epoch, uint64_t h, uint32_t self,
                                                  const uint32_t *sig, size_t W, bool cached,
                                                  bool &claimed) {
    const uint32_t tag = (epoch << 24) | static_cast<uint32_t>(h >> 40);
    const unsigned long long want = (static_cast<unsigned long long>(tag) << 32) | self;
    uint64_t s = h & mask;
    unsigned long long e = load_entry(table + s, cached);
    for (;;) {
        if (static_cast<uint32_t>(e >> 56) != epoch) {
            const unsigned long long prev = atomicCAS(table + s, e, want);
            if (prev == e) {
                claimed = true;
                return self;
            }
            e = prev;
            continue;
        }
        if (static_cast<uint32_t>(e >> 32) == tag) {
            const uint32_t rep = static_cast<uint32_t>(e);
            if (rows_equal(sig, W, self, rep)) {
                claimed = false;
                return rep;
            }
        }
        s = (s + 1) & mask;
        e = load_entry(table + s, cached);
    }
}

// Rounds after the first table round skip the blocks that cannot split:
// once a round changed the ids of few states, a block is refined only if a
// member has a successor whose id changed (the block is "touched").  Members
// of one block had equal keys in the round that formed it; if no successor
// id changed, their new keys are equal again.  Uniform over the grid.
__device__ __forceinline__ bool incremental_round(const RoundCtl &c, size_t N, uint32_t r) {
    return r > c.full_until && static_cast<uint64_t>(c.last_changed) * 8 < N;
}


// Whether this round's successor-id gathers go through the LDS slices
// (edges bucketed for this refinement): the rounds that refine nearly every
// state, i.e. the first table round, and non-incremental rounds with at most
// three blocks per four states (fewer singletons than that leave too few
// states to refine for a full pass over the edges).  Uniform over the grid.
__device__ __forceinline__ bool pb_round(const PbArgs &pb, const RoundCtl &c, size_t N) {
    if (!pb.nb || c.done) return false;
    const uint32_t r = c.round;
    if (r <= c.all_active_until) return true;
    if (incremental_round(c, N, r)) return false;
    return 4ull * c.prev_count < 3ull * N;
}

struct SigParams {
    const uint32_t *cols;
    const uint32_t *colmap;
    size_t N;
    uint32_t k_eff;
    uint32_t *blockA, *blockB;
    uint32_t *sig;
    uint64_t *hash;
    unsigned long long *table;
    uint64_t table_cap;
    const uint32_t *multi;
    unsigned long long *active;
    const unsigned long long *accbits;
    uint32_t *presence;
    uint32_t *presence_packed;
    uint8_t *lab8;
    uint32_t *counters;
    const RoundCtl *ctl;
    uint32_t cached_probe;
    unsigned long long *chg;
    unsigned long long *single;
    unsigned long long *touched;
    unsigned long long *chg_sum;
    uint32_t grouping;  // 1: sort grouping (no claims in the signature kernel)
    uint32_t hash_bits;  // 0: full key hashes; else only the low bits
    // segmented refinements: the parts, so that a wave inside parts with
    // fewer letters than k_eff skips the padding letters (nparts 0: none)
    const Part *parts;
    const uint32_t *tile_part;
    uint32_t nparts;
    PbArgs pb;  // nb > 0: dense rounds gather through LDS slices
    // segmented refinements: decided tiles and their holders (else null)
    const uint8_t *tile_dead;
    const uint16_t *tile_lead;
};

// Segmented refinements: whether every kBlock-state tile of [base, base + n)
// (base a multiple of kBlock, base < N) holds only decided segments.  Their
// ids never change again and both block buffers hold them, so every round
// kernel skips them.  Uniform across the workgroup.
__device__ __forceinline__ bool tiles_dead(const uint8_t *dead, size_t N, size_t base,
                                           uint32_t n) {
    if (!dead) return false;
    const size_t end = base + n < N ? base + n : N;
    for (size_t t = base / kBlock; t * kBlock < end; ++t)
        if (!dead[t]) return false;
    return true;
}

// The states of those tiles that hold their block's id (the block count
// includes them every round).
__device__ __forceinline__ uint32_t dead_holders(const uint16_t *lead, size_t N, size_t base,
                                                 uint32_t n) {
    const size_t end = base + n < N ? base + n : N;
    uint32_t h = 0;
    for (size_t t = base / kBlock; t * kBlock < end; ++t) h += lead[t];
    return h;
}

__device__ __forceinline__ uint32_t states_in(size_t N, size_t base, uint32_t n) {
    return static_cast<uint32_t>((base + n < N ? base + n : N) - base);
}

// Letters a wave must read: in a segmented refinement, letters at or above
// the largest alphabet of the parts that hold the wave's states are padding
// (the identity, whose successor id is the state's own id, the leading
// component of its key); k_eff otherwise.  Uniform across the wave.
__device__ __forceinline__ uint32_t wave_letters(const SigParams &p, size_t first, uint32_t keff) {
    if (!p.nparts || first >= p.N) return keff;
    const size_t last = first + 63 < p.N ? first + 63 : p.N - 1;
    uint32_t pi = p.tile_part[first / kBlock];
    while (static_cast<size_t>(p.parts[pi].off) + p.parts[pi].n <= first) ++pi;
    uint32_t k = 0;
    for (; pi < p.nparts && p.parts[pi].off <= last; ++pi) k = k > p.parts[pi].k ? k : p.parts[pi].k;
    return k < keff ? k : keff;
}

__device__ __forceinline__ uint64_t limit_hash(uint64_t h, uint32_t bits) {
    return bits ? (h & ((1ull << bits) - 1ull)) : h;
}

__device__ __forceinline__ uint32_t acc_bit(const unsigned long long *accbits, uint32_t t) {
    return static_cast<uint32_t>(accbits[t >> 6] >> (t & 63)) & 1u;
}

// Round 0 when k_eff + 1 <= kPatternMaxBits: the signature of q is the bit
// pattern (q accepting, successor 0 accepting, ...), which is itself an exact
// label of q's new block; no table is needed.  Distinct patterns are counted
// by the workgroups that set a bit first in a presence bitmap (deduplicated
// in LDS per workgroup, then OR-ed into HBM).
template <int KC>
__global__ __launch_bounds__(kBlock) void k_pattern_round(SigParams p) {
    __shared__ uint32_t pres[(1u << kPatternMaxBits) / 32];
    if (p.ctl->done) return;
    const uint32_t keff = KC > 0 ? static_cast<uint32_t>(KC) : p.k_eff;
    const uint32_t bits = keff + 1;
    const uint32_t words = bits >= 5 ? (1u << bits) / 32 : 1u;
    // up to 64 patterns: each thread keeps the patterns it saw in a register
    const bool in_reg = bits <= 6;
    for (uint32_t i = threadIdx.x; i < words; i += kBlock) pres[i] = 0;
    __syncthreads();
    uint32_t *__restrict__ out = p.blockB;
    unsigned long long seen_reg = 0;
    const ColPtrs<KC> colp(p.cols, p.colmap, p.N);
    auto emit = [&](size_t q, uint32_t label) {
        out[q] = label;
        if (p.lab8) p.lab8[q] = static_cast<uint8_t>(label);
        if (in_reg)
            seen_reg |= 1ull << label;
        else
            atomicOr(pres + (label >> 5), 1u << (label & 31));
    };
    if constexpr (KC > 0) {
        // S states per thread and iteration, every load of one kind issued
        // for all of them before any value is used (the round is bound by
        // the latency of the column reads and the dependent bit gathers)
        constexpr int S = 4;
        for (size_t base = static_cast<size_t>(blockIdx.x) * (S * kBlock); base < p.N;
             base += static_cast<size_t>(gridDim.x) * (S * kBlock)) {
            size_t q[S];
            uint32_t t[S][KC], label[S];
#pragma unroll
            for (int i = 0; i < S; ++i) q[i] = base + i * kBlock + threadIdx.x;
#pragma unroll
            for (int i = 0; i < S; ++i)
#pragma unroll
                for (int j = 0; j < KC; ++j) t[i][j] = q[i] < p.N ? colp.c[j][q[i]] : 0u;
#pragma unroll
            for (int i = 0; i < S; ++i) {
                label[i] = q[i] < p.N ? acc_bit(p.accbits, static_cast<uint32_t>(q[i])) : 0u;
#pragma unroll
                for (int j = 0; j < KC; ++j) label[i] |= acc_bit(p.accbits, t[i][j]) << (j + 1);
            }
#pragma unroll
            for (int i = 0; i < S; ++i)
                if (q[i] < p.N) emit(q[i], label[i]);
        }
    } else {
        for (size_t q = global_tid(); q < p.N; q += grid_stride()) {
            uint32_t label = acc_bit(p.accbits, static_cast<uint32_t>(q));
            for (uint32_t j = 0; j < keff; ++j) {
                const uint32_t t = p.cols[static_cast<size_t>(p.colmap[j]) * p.N + q];
                label |= acc_bit(p.accbits, t) << (j + 1);
            }
            emit(q, label);
        }
    }
    if (in_reg) {
        seen_reg = wave_or64(seen_reg);
        if (lane_id() == 0 && seen_reg) {
            atomicOr(pres + 0, static_cast<uint32_t>(seen_reg));
            if (words > 1) atomicOr(pres + 1, static_cast<uint32_t>(seen_reg >> 32));
        }
    }
    __syncthreads();
    uint32_t fresh = 0;
    for (uint32_t i = threadIdx.x; i < words; i += kBlock) {
        const uint32_t m = pres[i];
        if (m == 0) continue;
        const uint32_t seen =
            __hip_atomic_load(p.presence + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (m & ~seen) fresh += __popc(m & ~atomicOr(p.presence + i, m));
    }
    wg_add_spread(p.counters, 0, fresh);
    wg_add_spread(p.counters, 3, fresh);
}

// Round 1 after a pattern round when (k_eff + 1)^2 <= kPackedMaxBits: the
// signature (label of q, labels of its successors) packs exactly into one
// word, which becomes the new label.  Labels are gathered from the byte copy
// written by round 0 (small enough to stay in L2).  Distinct labels are
// marked in a map of one byte per label and counted by a pass over it; a
// workgroup first removes the duplicates among the tiles it handles in an
// LDS set, so a frequent label costs about one store per workgroup, not one
// per state.
constexpr uint32_t kLdsSlots = 2 * kBlock;
// labels a workgroup remembers across its tiles; the set is emptied before a
// tile once it is half full, so a tile (at most kBlock new labels) always
// finds empty slots
constexpr uint32_t kLabelSlots = 16 * kBlock;

// The packed round marks each label present in a map of one byte per label
// (the first time a workgroup meets it) with a plain store, and a pass over
// the map counts the labels afterwards.  Measured on MI355X, reading the
// label's bit first and setting it with an atomic whose old value counts
// it made the 2^22-state round 141 us instead of 69 + 10 us, and atomics
// that return nothing on a bit map made it slower still: a store waits on
// nothing, and several workgroups storing the same byte agree on its value.
__device__ __forceinline__ void label_present(uint32_t *map, uint32_t key) {
    reinterpret_cast<uint8_t *>(map)[key] = 1;
}

// Labels present in the map: the block count after the packed round.
__global__ __launch_bounds__(kBlock) void k_count_labels(SigParams p) {
    if (p.ctl->done) return;
    const uint4 *__restrict__ m = reinterpret_cast<const uint4 *>(p.presence_packed);
    constexpr size_t n = kLabelMapBytes / 16;
    uint32_t c = 0;
    for (size_t i = global_tid(); i < n; i += grid_stride()) {
        const uint4 v = m[i];
        // (bytes are 0 or 1)
        c += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
    }
    wg_add_spread(p.counters, 0, c);
    wg_add_spread(p.counters, 3, c);
}

template <int KC>
__global__ __launch_bounds__(kBlock) void k_packed_round(SigParams p) {
    __shared__ uint32_t lset[kLabelSlots];
    __shared__ uint32_t lfill;
    if (p.ctl->done) return;
    const uint32_t r = p.ctl->round;
    uint32_t *__restrict__ Y = (r & 1u) ? p.blockA : p.blockB;
    const uint32_t keff = KC > 0 ? static_cast<uint32_t>(KC) : p.k_eff;
    const uint32_t bits = keff + 1;
    const uint32_t tx = threadIdx.x;
    const ColPtrs<KC> colp(p.cols, p.colmap, p.N);
    for (uint32_t i = tx; i < kLabelSlots; i += kBlock) lset[i] = ~0u;
    if (tx == 0) lfill = 0;
    __syncthreads();
    // XCD-sliced tiles: in a union each XCD gathers the labels of one
    // operand only, a footprint its own L2 holds.  A tile has 2 * kBlock
    // states, two per thread, so that each thread has the loads of two
    // states in flight (the round is bound by load latency).
    constexpr int S = 2;
    const TileRange tr = xcd_tiles(p.N, S * kBlock);
    for (size_t t = tr.first; t < tr.end; t += tr.step) {
        const size_t base = t * (S * kBlock);
        // every thread reads the fill before any thread of this tile
        // inserts; a tile adds at most S * kBlock labels, so a set at most
        // half full always has empty slots for them
        const bool half_full = lfill > kLabelSlots / 2;
        __syncthreads();
        if (half_full) {
            for (uint32_t i = tx; i < kLabelSlots; i += kBlock) lset[i] = ~0u;
            if (tx == 0) lfill = 0;
            __syncthreads();
        }
        size_t q[S];
        uint32_t key[S];
#pragma unroll
        for (int i = 0; i < S; ++i) q[i] = base + i * kBlock + tx;
        if constexpr (KC > 0) {
            // all column entries first, then all byte labels
            uint32_t tt[S][KC];
#pragma unroll
            for (int i = 0; i < S; ++i)
#pragma unroll
                for (int j = 0; j < KC; ++j) tt[i][j] = q[i] < p.N ? colp.c[j][q[i]] : 0u;
#pragma unroll
            for (int i = 0; i < S; ++i) {
                key[i] = q[i] < p.N ? p.lab8[q[i]] : 0u;
#pragma unroll
                for (int j = 0; j < KC; ++j)
                    key[i] |= static_cast<uint32_t>(p.lab8[tt[i][j]]) << (bits * (j + 1));
            }
        } else {
#pragma unroll
            for (int i = 0; i < S; ++i) {
                key[i] = 0;
                if (q[i] >= p.N) continue;
                key[i] = p.lab8[q[i]];
                for (uint32_t j = 0; j < keff; ++j) {
                    const uint32_t tj = p.cols[static_cast<size_t>(p.colmap[j]) * p.N + q[i]];
                    key[i] |= static_cast<uint32_t>(p.lab8[tj]) << (bits * (j + 1));
                }
            }
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (q[i] >= p.N) continue;
            Y[q[i]] = key[i];
            // keys are < 2^kPackedMaxBits, so ~0u marks an empty LDS slot
            uint32_t slot = (key[i] * 0x9E3779B1u) >> 20;  // 12 bits
            bool first = false;
            for (;;) {
                const uint32_t e =
                    __hip_atomic_load(lset + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (e == key[i]) break;
                if (e == ~0u) {
                    const uint32_t prev = atomicCAS(lset + slot, ~0u, key[i]);
                    if (prev == ~0u) {
                        first = true;
                        atomicAdd(&lfill, 1u);
                        break;
                    }
                    if (prev == key[i]) break;
                }
                slot = (slot + 1) & (kLabelSlots - 1);
            }
            if (first) label_present(p.presence_packed, key[i]);
        }
        __syncthreads();
    }
}

// First kernel of a round: clears the table every kEpochs rounds; in
// incremental rounds it records, for the states refined last round, whether
// their block is now a singleton, and marks the blocks with a member whose
// successor changed id in the last round.  It also clears the touched bitmap
// of the next round.
// Sets bit xi of the bitmap T for the lanes with `want` (every lane of the
// wave calls it).  Lanes whose bits share a word are merged into one atomic:
// in id order (chains, twins laid out in the same order) a wave's 64 marks
// often fall into one word, and 64 atomics on one address serialise.  At most
// two merges (the second only if the first merged several lanes); the lanes
// left set their bits one by one.
__device__ __forceinline__ void wave_mark_bit(unsigned long long *T, uint32_t xi, bool want) {
    const uint32_t w = xi >> 6;
    const unsigned long long bit = 1ull << (xi & 63);
    unsigned long long pending = __ballot(want);
    for (int pass = 0; pass < 2 && pending; ++pass) {
        const int lead = __ffsll(pending) - 1;
        const uint32_t lw = __shfl(w, lead, 64);
        const bool mine = ((pending >> lane_id()) & 1ull) && w == lw;
        const unsigned long long grp = __ballot(mine);
        const unsigned long long v = wave_or64(mine ? bit : 0ull);
        if (static_cast<int>(lane_id()) == lead) atomicOr(T + lw, v);
        pending &= ~grp;
        if (__popcll(grp) < 2) break;
    }
    if ((pending >> lane_id()) & 1ull) atomicOr(T + w, bit);
}

template <int KC>
__device__ __forceinline__ void mark_body(const SigParams &p) {
    if (p.ctl->done) return;
    const uint32_t r = p.ctl->round;
    // the table is cleared every kEpochs rounds (its entries carry the epoch)
    if (r > 0 && r % kEpochs == 0) {
        for (size_t i = global_tid(); i < p.table_cap; i += grid_stride()) p.table[i] = 0ull;
    }
    const size_t words = (p.N + 63) / 64;
    unsigned long long *__restrict__ Tn = p.touched + ((r + 1) & 1u) * words;
    for (size_t i = global_tid(); i < words; i += grid_stride()) Tn[i] = 0ull;
    // this round's changed-wave summary starts empty (the grouping kernels
    // fill it)
    const size_t sum_words = summary_words(p.N);
    unsigned long long *__restrict__ Sn = p.chg_sum + (r & 1u) * sum_words;
    for (size_t i = global_tid(); i < sum_words; i += grid_stride()) Sn[i] = 0ull;
    if (r <= p.ctl->all_active_until || !incremental_round(*p.ctl, p.N, r)) return;
    unsigned long long *__restrict__ T = p.touched + (r & 1u) * words;
    const uint32_t *__restrict__ X = (r & 1u) ? p.blockB : p.blockA;
    const unsigned long long *__restrict__ chg = p.chg;
    // last round's summary in LDS: a successor's changed-id word is read
    // only when its group of states changed an id (the few groups of an
    // incremental round), instead of one random gather per transition
    __shared__ unsigned long long lsum[kSumLdsWords];
    const bool filter = sum_words <= kSumLdsWords;
    if (filter) {
        const unsigned long long *__restrict__ Sp = p.chg_sum + ((r - 1) & 1u) * sum_words;
        for (size_t i = threadIdx.x; i < sum_words; i += kBlock) lsum[i] = Sp[i];
        __syncthreads();
    }
    auto changed = [&](uint32_t t) -> bool {
        if (filter && !summary_bit(lsum, t)) return false;
        return ((chg[t >> 6] >> (t & 63)) & 1ull) != 0;
    };
    const uint32_t keff = KC > 0 ? static_cast<uint32_t>(KC) : p.k_eff;
    const ColPtrs<KC> colp(p.cols, p.colmap, p.N);
    // S states per thread; each kind of load is issued for all of them before
    // any of its values is used (the kernel is bound by load latency)
    constexpr int S = 4;
    for (size_t base = static_cast<size_t>(blockIdx.x) * (S * kBlock); base < p.N;
         base += static_cast<size_t>(gridDim.x) * (S * kBlock)) {
        if (tiles_dead(p.tile_dead, p.N, base, S * kBlock)) continue;
        size_t q[S];
        unsigned long long sw[S], aw[S];
        bool s[S], was_active[S];
        uint32_t x[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            q[i] = base + i * kBlock + threadIdx.x;
            const size_t first = q[i] - lane_id();
            sw[i] = first < p.N ? p.single[first >> 6] : ~0ull;
            aw[i] = first < p.N ? p.active[first >> 6] : 0ull;
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
            s[i] = q[i] >= p.N || ((sw[i] >> lane_id()) & 1ull);
            // a block formed last round with one member stays a singleton
            was_active[i] = !s[i] && ((aw[i] >> lane_id()) & 1ull);
            x[i] = was_active[i] ? X[q[i]] : 0u;
        }
        // a block id is one of the block's states, so a state whose id is
        // another state's index shares its block; a state holding its own
        // index learns from its own mark (a coalesced read)
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (was_active[i]) s[i] = x[i] == q[i] && p.multi[q[i]] != r;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const unsigned long long nsw = __ballot(s[i]);
            const size_t first = q[i] - lane_id();
            if (lane_id() == 0 && first < p.N && nsw != sw[i]) p.single[first >> 6] = nsw;
        }
        bool dirty[S];
        if constexpr (KC > 0) {
            // unconditional, straight-line loads (a state that needs none
            // reads state 0's): conditional loads sit in branches, across
            // which the compiler waits for every load in flight.  Padding
            // letters of a segmented refinement (the identity) never make
            // members of a block differ, so they are not read (kw is uniform
            // across the wave).
            uint32_t t[S][KC], kw[S];
            // a wave whose states are all singletons (or frozen) marks
            // nothing: it reads no letter (uniform across the wave)
#pragma unroll
            for (int i = 0; i < S; ++i)
                kw[i] = __ballot(!s[i]) ? wave_letters(p, q[i] - lane_id(), KC) : 0u;
#pragma unroll
            for (int i = 0; i < S; ++i)
#pragma unroll
                for (int j = 0; j < KC; ++j) t[i][j] = j < kw[i] ? colp.c[j][s[i] ? 0 : q[i]] : 0u;
#pragma unroll
            for (int i = 0; i < S; ++i) {
                bool any = false;
#pragma unroll
                for (int j = 0; j < KC; ++j)
                    if (j < kw[i]) any |= changed(t[i][j]);
                dirty[i] = !s[i] && any;
            }
        } else {
#pragma unroll
            for (int i = 0; i < S; ++i) {
                dirty[i] = false;
                for (uint32_t j0 = 0; j0 < keff && !s[i] && !dirty[i]; j0 += 8) {
                    const uint32_t m = keff - j0 < 8 ? keff - j0 : 8;
                    uint32_t t[8];
#pragma unroll
                    for (uint32_t j = 0; j < 8; ++j)
                        if (j < m) t[j] = p.cols[static_cast<size_t>(p.colmap[j0 + j]) * p.N + q[i]];
#pragma unroll
                    for (uint32_t j = 0; j < 8; ++j)
                        if (j < m) dirty[i] |= changed(t[j]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const uint32_t xi = dirty[i] ? (was_active[i] ? x[i] : X[q[i]]) : 0u;
            wave_mark_bit(T, xi, dirty[i]);
        }
    }
}

// Whether state q is refined this round (selective rounds), with the
// bookkeeping of the selection: in full rounds the states refined last round
// learn whether their block is now a singleton (the marking kernel does this
// in incremental rounds), and the wave's mask of refined states is stored.
// Every lane of the wave must call it (ballots).
// was_active: the state was refined in the previous round.  A state that is
// refined in neither round already has its id in both block buffers (the
// round that skipped it first copied it), so it needs no copy now.
// sw, aw: the wave's singleton and refined-state words (as loaded here);
// mq: multi[q] when the caller loaded it ahead (else ~0u: loaded here when
// needed).
__device__ __forceinline__ bool select_state_words(const SigParams &p, size_t q, uint32_t w0,
                                                   uint32_t r, bool inc,
                                                   const unsigned long long *T,
                                                   unsigned long long sw, unsigned long long aw,
                                                   uint32_t mq, bool &was_active) {
    const bool valid = q < p.N;
    const size_t first = q - lane_id();
    const size_t wd = first >> 6;
    was_active = ((aw >> lane_id()) & 1ull) != 0;
    bool s = !valid || ((sw >> lane_id()) & 1ull);
    if (!inc) {
        // (a state whose id is another state's index shares its block)
        if (!s && was_active) s = w0 == q && (mq != ~0u ? mq : p.multi[q]) != r;
        const unsigned long long nsw = __ballot(s);
        if (lane_id() == 0 && first < p.N && nsw != sw) p.single[wd] = nsw;
    }
    const bool act = !s && (!inc || ((T[w0 >> 6] >> (w0 & 63)) & 1ull));
    const unsigned long long am = __ballot(act);
    if (lane_id() == 0 && first < p.N) p.active[wd] = am;
    return act;
}

__device__ __forceinline__ bool select_state(const SigParams &p, size_t q, uint32_t w0, uint32_t r,
                                             bool inc, const unsigned long long *T,
                                             bool &was_active) {
    const size_t first = q - lane_id();
    const unsigned long long sw = first < p.N ? p.single[first >> 6] : ~0ull;
    const unsigned long long aw = first < p.N ? p.active[first >> 6] : 0ull;
    return select_state_words(p, q, w0, r, inc, T, sw, aw, ~0u, was_active);
}

// Writes the key row and hash of a refined state; a state that holds its
// block's id (selective rounds) keeps it and counts as its block.
__device__ __forceinline__ void emit_key(const SigParams &p, uint32_t *__restrict__ Y, size_t q,
                                         uint32_t w0, const uint32_t *w, uint32_t keff, size_t W,
                                         bool holder_keeps, uint32_t &claims) {
    uint32_t *__restrict__ row = p.sig + q * W;
    row[0] = w0;
    uint64_t h = mix_step(kHashSeed, w0);
    for (uint32_t j = 0; j < keff; ++j) {
        row[1 + j] = w[j];
        h = mix_step(h, w[j]);
    }
    h = limit_hash(mix_final(h), p.hash_bits);
    p.hash[q] = h;
    if (holder_keeps && w0 == q) {
        // the state that holds its block's id keeps it: the members with
        // its key join it without the table (grouping kernels), so a block
        // that does not split keeps its id
        Y[q] = w0;
        ++claims;
    }
}

// Signatures of the states refined this round.  A state is refined if the
// round refines everything (the first rounds), or if its block is not a
// singleton and, in incremental rounds, is touched; the others keep their id
// and are copied to the output buffer.  A refined state that holds its
// block's id keeps it (its block survives with that id).
// KC > 0: k_eff known at compile time (fully unrolled gathers, two states per
// thread);
// KC == 0: runtime k_eff, gathers issued in batches of 8.
template <int KC>
__device__ __forceinline__ void signature_body(const SigParams &p) {
    if (p.ctl->done || pb_round(p.pb, *p.ctl, p.N)) return;
    const uint32_t r = p.ctl->round;
    const uint32_t *__restrict__ X = (r & 1u) ? p.blockB : p.blockA;
    uint32_t *__restrict__ Y = (r & 1u) ? p.blockA : p.blockB;
    const bool all = r <= p.ctl->all_active_until;
    const uint32_t keff = KC > 0 ? static_cast<uint32_t>(KC) : p.k_eff;
    const size_t W = keff + 1;
    const bool inc = !all && incremental_round(*p.ctl, p.N, r);
    const size_t words = (p.N + 63) / 64;
    const unsigned long long *__restrict__ T = p.touched + (r & 1u) * words;
    uint32_t leaders = 0, claims = 0;

    if constexpr (KC > 0) {
        const ColPtrs<KC> colp(p.cols, p.colmap, p.N);
        // two states per thread, all independent loads of both issued before
        // their values are used
        // XCD-sliced tiles of two kBlock-state halves (a union's successor
        // ids are gathered from one operand per XCD)
        const TileRange tr = xcd_tiles(p.N, 2 * kBlock);
        for (size_t tile = tr.first; tile < tr.end; tile += tr.step) {
            const size_t base = tile * (2 * kBlock);
            if (tiles_dead(p.tile_dead, p.N, base, 2 * kBlock)) {
                if (threadIdx.x == 0) leaders += dead_holders(p.tile_lead, p.N, base, 2 * kBlock);
                continue;
            }
            const size_t q[2] = {base + threadIdx.x, base + kBlock + threadIdx.x};
            bool act[2];
            uint32_t w0[2], t[2][KC], w[2][KC];
#pragma unroll
            for (int i = 0; i < 2; ++i) w0[i] = q[i] < p.N ? X[q[i]] : 0u;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                if (all) {
                    act[i] = q[i] < p.N;
                    const size_t first = q[i] - lane_id();
                    const unsigned long long am = __ballot(act[i]);
                    if (lane_id() == 0 && first < p.N) p.active[first >> 6] = am;
                } else {
                    bool was;
                    act[i] = select_state(p, q[i], w0[i], r, inc, T, was);
                    if (q[i] < p.N && !act[i]) {
                        if (was) Y[q[i]] = w0[i];
                        leaders += w0[i] == q[i] ? 1u : 0u;
                    }
                }
            }
            // waves where most lanes are refined load unconditionally (the
            // others reread the wave's first refined state, lines the wave
            // fetches anyway); sparse waves load per lane
            const unsigned long long am[2] = {__ballot(act[0]), __ballot(act[1])};
            // letters this wave reads for each of its two states (padding
            // letters of a segmented refinement are the state's own id; a
            // wave with no refined state reads none)
            const uint32_t kw[2] = {am[0] ? wave_letters(p, q[0] - lane_id(), KC) : 0u,
                                    am[1] ? wave_letters(p, q[1] - lane_id(), KC) : 0u};
            const uint32_t nact = static_cast<uint32_t>(__popcll(am[0])) +
                                  static_cast<uint32_t>(__popcll(am[1]));
            if (nact >= 64) {
                // a slot with no refined lane borrows the other slot's (which
                // then has all 64)
                size_t qs[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const int src = am[i] ? i : (i ^ 1);
                    const size_t borrow =
                        q[src] - lane_id() +
                        static_cast<size_t>(__ffsll(static_cast<unsigned long long>(am[src])) - 1);
                    qs[i] = act[i] ? q[i] : borrow;
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < KC; ++j) t[i][j] = j < kw[i] ? colp.c[j][qs[i]] : 0u;
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < KC; ++j) w[i][j] = j < kw[i] ? X[t[i][j]] : w0[i];
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < KC; ++j)
                        t[i][j] = act[i] && j < kw[i] ? colp.c[j][q[i]] : 0u;
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < KC; ++j)
                        w[i][j] = act[i] ? (j < kw[i] ? X[t[i][j]] : w0[i]) : 0u;
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
                if (act[i])
                    emit_key(p, Y, q[i], w0[i], w[i], KC, W, !all && p.grouping == 0, claims);
        }
    } else {
        const TileRange tr = xcd_tiles(p.N, kBlock);
        for (size_t tile = tr.first; tile < tr.end; tile += tr.step) {
            if (tiles_dead(p.tile_dead, p.N, tile * kBlock, kBlock)) {
                if (threadIdx.x == 0) leaders += dead_holders(p.tile_lead, p.N, tile * kBlock, kBlock);
                continue;
            }
            const size_t q = tile * kBlock + threadIdx.x;
            const bool valid = q < p.N;
            const uint32_t w0 = valid ? X[q] : 0u;
            bool act = valid;
            if (all) {
                const size_t first = q - lane_id();
                const unsigned long long am = __ballot(act);
                if (lane_id() == 0 && first < p.N) p.active[first >> 6] = am;
            } else {
                bool was;
                act = select_state(p, q, w0, r, inc, T, was);
                if (valid && !act) {
                    if (was) Y[q] = w0;
                    leaders += w0 == q ? 1u : 0u;
                }
            }
            if (!act) continue;
            uint32_t *__restrict__ row = p.sig + q * W;
            row[0] = w0;
            uint64_t h = mix_step(kHashSeed, w0);
            // runtime k_eff: gathers issued in batches of 8
            for (uint32_t j0 = 0; j0 < keff; j0 += 8) {
                const uint32_t m = keff - j0 < 8 ? keff - j0 : 8;
                uint32_t t[8], w[8];
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j)
                    if (j < m) t[j] = p.cols[static_cast<size_t>(p.colmap[j0 + j]) * p.N + q];
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j)
                    if (j < m) w[j] = X[t[j]];
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j)
                    if (j < m) {
                        row[1 + j0 + j] = w[j];
                        h = mix_step(h, w[j]);
                    }
            }
            h = limit_hash(mix_final(h), p.hash_bits);
            p.hash[q] = h;
            if (!all && p.grouping == 0 && w0 == q) {
                Y[q] = w0;
                ++claims;
            }
        }
    }
    wg_add_spread(p.counters, 0, leaders + claims);
    wg_add_spread(p.counters, 3, claims);
}

// ---------------------------------------------------------------- gathers through LDS slices
//
// A dense round gathers k_eff block ids per state at random over the whole
// id array, which runs at the device's random-gather rate (HBM / Infinity
// Cache lines).  Here the gathers go through LDS instead.  Once per
// refinement the edges (q, letter) are bucketed by the slice of their target
// (2^kPbSliceLog states, whose ids fill 64 KB of LDS), and inside a bucket
// by source tile.  In a dense round, pass A gives each bucket a workgroup
// that loads its slice of the round's ids into LDS and streams the bucket's
// edges, writing the gathered id of each edge next to it (coalesced).  Pass B
// gives each source tile a workgroup that reads its runs from every bucket,
// places the ids into the tile's keys in LDS, and then does what the
// signature kernel does with them.  Both passes stream; the only random
// accesses are to LDS.

// States per thread whose successors are loaded together in the bucketing
// kernels (a tile holds kPbTile / kBlock = 8 per thread).
template <int KC>
constexpr int kPbBatch = KC <= 4 ? 8 : (KC <= 8 ? 4 : 2);
// The scatter's workgroups are twice as wide: its LDS (the tile's edges)
// allows two per CU, which then hold 16 waves instead of 8.
constexpr uint32_t kPbScatterThreads = 2 * kBlock;
template <int KC>
constexpr int kPbScatterBatch = kPbBatch<KC> / 2;

// Edge counts per (tile, bucket), tile-major: cnt[t * nb + b] is the length
// of tile t's run in bucket b (one coalesced row per tile).
template <int KC>
__global__ __launch_bounds__(kBlock) void k_pb_count(const uint32_t *cols, const uint32_t *colmap,
                                                      size_t N, uint32_t nb, uint32_t ntiles,
                                                      uint32_t *cnt) {
    __shared__ uint32_t hist[kPbMaxBuckets];
    const ColPtrs<KC> colp(cols, colmap, N);
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        for (uint32_t b = threadIdx.x; b < nb; b += kBlock) hist[b] = 0;
        __syncthreads();
        const size_t base = static_cast<size_t>(t) * kPbTile;
        // the loads of a batch of states go out before their atomics
        for (uint32_t i0 = 0; i0 < kPbTile; i0 += kPbBatch<KC> * kBlock) {
            uint32_t tg[kPbBatch<KC>][KC];
#pragma unroll
            for (int u = 0; u < kPbBatch<KC>; ++u) {
                const size_t q = base + i0 + u * kBlock + threadIdx.x;
#pragma unroll
                for (int a = 0; a < KC; ++a) tg[u][a] = q < N ? colp.c[a][q] : ~0u;
            }
#pragma unroll
            for (int u = 0; u < kPbBatch<KC>; ++u)
#pragma unroll
                for (int a = 0; a < KC; ++a)
                    if (tg[u][a] != ~0u) atomicAdd(hist + (tg[u][a] >> kPbSliceLog), 1u);
        }
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < nb; b += kBlock)
            cnt[static_cast<size_t>(t) * nb + b] = hist[b];
        __syncthreads();
    }
}

// The edge list is bucket-major (bucket b's edges are contiguous, tile by
// tile), while the counts are tile-major.  The run starts come from a scan
// down each column of the count matrix, in three coalesced steps: column
// sums over chunks of kPbChunk tiles, a scan of each column's chunk sums
// (one wave per bucket) with the bucket totals scanned after it, and the
// run starts of each chunk's tiles.
__global__ __launch_bounds__(kBlock) void k_pb_colsum(const uint32_t *cnt, uint32_t nb,
                                                       uint32_t ntiles, uint32_t *csum) {
    const uint32_t c = blockIdx.x;
    const uint32_t t0 = c * kPbChunk;
    const uint32_t t1 = t0 + kPbChunk < ntiles ? t0 + kPbChunk : ntiles;
    for (uint32_t b = threadIdx.x; b < nb; b += kBlock) {
        uint32_t sum = 0;
        for (uint32_t t = t0; t < t1; ++t) sum += cnt[static_cast<size_t>(t) * nb + b];
        csum[static_cast<size_t>(c) * nb + b] = sum;
    }
}

// One wave per bucket: exclusive scan of the column's chunk sums in place,
// and the bucket's edge count into btot[b].
__global__ __launch_bounds__(kBlock) void k_pb_colscan(uint32_t *csum, uint32_t nb,
                                                        uint32_t nchunks, uint32_t *btot) {
    const uint32_t b = blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
    if (b >= nb) return;  // (uniform across the wave)
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < nchunks; c0 += 64) {
        const uint32_t c = c0 + lane_id();
        const uint32_t v = c < nchunks ? csum[static_cast<size_t>(c) * nb + b] : 0u;
        uint32_t x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane_id() >= static_cast<uint32_t>(d)) x += y;
        }
        if (c < nchunks) csum[static_cast<size_t>(c) * nb + b] = carry + x - v;
        carry += __shfl(x, 63, 64);
    }
    if (lane_id() == 0) btot[b] = carry;
}

// One workgroup of 1024 threads (nb <= 1024): bucket starts, bstart[nb] =
// the edge count.
__global__ __launch_bounds__(1024) void k_pb_bscan(const uint32_t *btot, uint32_t nb,
                                                    uint32_t *bstart) {
    __shared__ uint32_t wsum[16];
    const uint32_t i = threadIdx.x;
    const uint32_t v = i < nb ? btot[i] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane_id() >= static_cast<uint32_t>(d)) x += y;
    }
    if (lane_id() == 63) wsum[i / 64] = x;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t w = 0; w < i / 64; ++w) before += wsum[w];
    if (i < nb) bstart[i] = before + x - v;
    if (i == 1023) bstart[nb] = before + x;
}

// Run starts, tile-major: off[t * nb + b] = bucket b's start + the chunk's
// scanned column sum + the runs of the chunk's earlier tiles in bucket b.
__global__ __launch_bounds__(kBlock) void k_pb_apply(const uint32_t *cnt, const uint32_t *csum,
                                                      const uint32_t *bstart, uint32_t nb,
                                                      uint32_t ntiles, uint32_t *off) {
    const uint32_t c = blockIdx.x;
    const uint32_t t0 = c * kPbChunk;
    const uint32_t t1 = t0 + kPbChunk < ntiles ? t0 + kPbChunk : ntiles;
    for (uint32_t b = threadIdx.x; b < nb; b += kBlock) {
        uint32_t run = bstart[b] + csum[static_cast<size_t>(c) * nb + b];
        for (uint32_t t = t0; t < t1; ++t) {
            const size_t k = static_cast<size_t>(t) * nb + b;
            off[k] = run;
            run += cnt[k];
        }
    }
}

// Tile t's runs into LDS: rbase[b] = the start of its run in bucket b (in
// the bucketed edge list), rstart[b] = the run's start in the tile's own edge
// order (the runs back to back, bucket by bucket), rstart[nb] = the tile's
// edge count.  Ends with a barrier.
template <uint32_t NT = kBlock>
__device__ __forceinline__ void pb_tile_runs(const PbArgs &pb, uint32_t t, uint32_t *rstart,
                                             uint32_t *rbase, uint32_t *wsum) {
    const uint32_t tx = threadIdx.x;
    const size_t row = static_cast<size_t>(t) * pb.nb;
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < pb.nb; b0 += NT) {
        const uint32_t b = b0 + tx;
        uint32_t len = 0;
        if (b < pb.nb) {
            rbase[b] = pb.off[row + b];
            len = pb.cnt[row + b];
        }
        uint32_t x = len;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane_id() >= static_cast<uint32_t>(d)) x += y;
        }
        if (lane_id() == 63) wsum[tx / 64] = x;
        __syncthreads();
        uint32_t before = carry;
        for (uint32_t w = 0; w < tx / 64; ++w) before += wsum[w];
        if (b < pb.nb) rstart[b] = before + x - len;
        uint32_t total = carry;
        for (uint32_t w = 0; w < NT / 64; ++w) total += wsum[w];
        __syncthreads();
        carry = total;
    }
    if (tx == 0) rstart[pb.nb] = carry;
    __syncthreads();
}

// Small alphabets (k_eff <= 4: the ids fit beside the tile's keys in LDS):
// tile t's runs as one id per edge position instead of run starts to search.
// rid[j] = the run (bucket) holding position j of the tile's edge order,
// delta[b] = the start of run b in the edge list minus its start in the
// tile's order (so position j sits at j + delta[rid[j]], modulo 2^32); if
// lpos is given, lpos[b] = the run's start in the tile's order.  Each run is
// filled by the thread that scans its length.  Returns the tile's edge
// count; ends with a barrier.
template <uint32_t NT = kBlock>
__device__ __forceinline__ uint32_t pb_tile_run_ids(const PbArgs &pb, uint32_t t, uint16_t *rid,
                                                    uint32_t *delta, uint32_t *lpos,
                                                    uint32_t *wsum, uint32_t *tot) {
    const uint32_t tx = threadIdx.x;
    const size_t row = static_cast<size_t>(t) * pb.nb;
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < pb.nb; b0 += NT) {
        const uint32_t b = b0 + tx;
        uint32_t len = 0, at = 0;
        if (b < pb.nb) {
            at = pb.off[row + b];
            len = pb.cnt[row + b];
        }
        uint32_t x = len;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane_id() >= static_cast<uint32_t>(d)) x += y;
        }
        if (lane_id() == 63) wsum[tx / 64] = x;
        __syncthreads();
        uint32_t before = carry;
        for (uint32_t w = 0; w < tx / 64; ++w) before += wsum[w];
        if (b < pb.nb) {
            const uint32_t start = before + x - len;
            delta[b] = at - start;
            if (lpos) lpos[b] = start;
            for (uint32_t l = 0; l < len; ++l) rid[start + l] = static_cast<uint16_t>(b);
        }
        uint32_t total = carry;
        for (uint32_t w = 0; w < NT / 64; ++w) total += wsum[w];
        __syncthreads();
        carry = total;
    }
    if (tx == 0) *tot = carry;
    __syncthreads();
    return *tot;
}

// The run holding position j of a tile's edge order (rstart[lo] <= j <
// rstart[lo + 1]; empty runs are never chosen).
__device__ __forceinline__ uint32_t pb_run_of(const uint32_t *rstart, uint32_t nb, uint32_t j) {
    uint32_t lo = 0, hi = nb;  // rstart[lo] <= j < rstart[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (rstart[mid] <= j)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Places every edge of a tile into its run (order inside a run is free: an
// edge carries its own source slot).  The tile's edges are first sorted by
// bucket in LDS (its runs laid out back to back), then each run is written
// out contiguously, so the stores coalesce instead of landing two bytes at a
// time in hundreds of runs.
template <int KC>
__global__ __launch_bounds__(kPbScatterThreads) void k_pb_scatter(const uint32_t *cols, const uint32_t *colmap,
                                                        size_t N, PbArgs pb) {
    constexpr bool kIds = KC <= 4;
    __shared__ uint32_t rs[kPbMaxBuckets + 1];           // run starts, or deltas
    __shared__ uint32_t rb[kIds ? 1 : kPbMaxBuckets];    // run bases (search)
    __shared__ uint16_t rid[kIds ? kPbTile * KC : 2];    // run ids (small alphabets)
    __shared__ uint32_t lpos[kPbMaxBuckets];
    __shared__ uint32_t wsum[kPbScatterThreads / 64];
    __shared__ uint32_t tot;
    __shared__ uint16_t ltl[kPbTile * KC];
    __shared__ uint16_t lsrc[kPbTile * KC];
    const uint32_t tx = threadIdx.x;
    const ColPtrs<KC> colp(cols, colmap, N);
    for (uint32_t t = blockIdx.x; t < pb.ntiles; t += gridDim.x) {
        uint32_t total;
        if constexpr (kIds) {
            total = pb_tile_run_ids<kPbScatterThreads>(pb, t, rid, rs, lpos, wsum, &tot);
        } else {
            pb_tile_runs<kPbScatterThreads>(pb, t, rs, rb, wsum);
            for (uint32_t b = tx; b < pb.nb; b += kPbScatterThreads) lpos[b] = rs[b];
            total = rs[pb.nb];
            __syncthreads();
        }
        const size_t base = static_cast<size_t>(t) * kPbTile;
        // the loads of a batch of states go out before their atomics
        for (uint32_t i0 = 0; i0 < kPbTile; i0 += kPbScatterBatch<KC> * kPbScatterThreads) {
            uint32_t tg[kPbScatterBatch<KC>][KC];
#pragma unroll
            for (int u = 0; u < kPbScatterBatch<KC>; ++u) {
                const size_t q = base + i0 + u * kPbScatterThreads + tx;
#pragma unroll
                for (int a = 0; a < KC; ++a) tg[u][a] = q < N ? colp.c[a][q] : ~0u;
            }
#pragma unroll
            for (int u = 0; u < kPbScatterBatch<KC>; ++u) {
                const uint32_t i = i0 + u * kPbScatterThreads + tx;
#pragma unroll
                for (int a = 0; a < KC; ++a) {
                    if (tg[u][a] == ~0u) continue;
                    const uint32_t e = atomicAdd(lpos + (tg[u][a] >> kPbSliceLog), 1u);
                    ltl[e] = static_cast<uint16_t>(tg[u][a] & ((1u << kPbSliceLog) - 1u));
                    lsrc[e] = static_cast<uint16_t>(i * KC + a);
                }
            }
        }
        __syncthreads();
        for (uint32_t j = tx; j < total; j += kPbScatterThreads) {
            uint32_t e;
            if constexpr (kIds) {
                e = j + rs[rid[j]];
            } else {
                const uint32_t lo = pb_run_of(rs, pb.nb, j);
                e = rb[lo] + (j - rs[lo]);
            }
            pb.tl[e] = ltl[j];
            pb.src[e] = lsrc[j];
        }
        __syncthreads();
    }
}

// Pass A: one or more workgroups per bucket; each loads the bucket's slice of
// the round's ids into LDS and writes the gathered id of its share of the
// bucket's edges.
constexpr uint32_t kPbGatherThreads = 1024;  // one workgroup of 16 waves per bucket
// pass B: threads of a tile's workgroup (measured on MI355X, bench step:
// 512 threads 6.97 ms, 256 7.03, 1024 7.28: three workgroups per CU by LDS,
// so 24 waves instead of 12, while 1,024 threads leave two states per thread)
constexpr uint32_t kPbSigThreads = 512;
// the packed round's pass B (bench step 6.96 -> 6.88 ms against 256 threads)
constexpr uint32_t kPbPackedThreads = 512;

__global__ __launch_bounds__(kPbGatherThreads) void k_pb_gather(SigParams p, uint32_t per_bucket) {
    extern __shared__ uint32_t slice[];
    if (!pb_round(p.pb, *p.ctl, p.N)) return;
    const uint32_t r = p.ctl->round;
    const uint32_t *__restrict__ X = (r & 1u) ? p.blockB : p.blockA;
    const PbArgs &pb = p.pb;
    constexpr uint32_t S = 1u << kPbSliceLog;
    // (the round end reads the record only after this kernel has finished)
    if (blockIdx.x == 0 && threadIdx.x == 0)
        const_cast<RoundCtl *>(p.ctl)->pb_rounds |= 1ull << (r % 64);
    for (uint32_t job = blockIdx.x; job < pb.nb * per_bucket; job += gridDim.x) {
        const uint32_t b = job / per_bucket, part = job % per_bucket;
        const size_t s0 = static_cast<size_t>(b) * S;
        const uint32_t len = static_cast<uint32_t>(p.N - s0 < S ? p.N - s0 : S);
        __syncthreads();  // the previous job's gathers are done with the slice
        for (uint32_t i = threadIdx.x; i < len; i += kPbGatherThreads) slice[i] = X[s0 + i];
        __syncthreads();
        const uint32_t lo = pb.bstart[b], hi = pb.bstart[b + 1];
        const uint32_t chunk = (hi - lo + per_bucket - 1) / per_bucket;
        const uint32_t a0 = lo + part * chunk;
        const uint32_t a1 = a0 + chunk < hi ? a0 + chunk : hi;
        // four edges per thread with 8-byte target and 16-byte value accesses,
        // after a scalar head up to a multiple of four
        const uint32_t al = (a0 + 3u) & ~3u;
        const uint32_t v0 = al < a1 ? al : a1;
        for (uint32_t e = a0 + threadIdx.x; e < v0; e += kPbGatherThreads) pb.val[e] = slice[pb.tl[e]];
        for (uint32_t e = v0 + 4 * threadIdx.x; e < a1; e += 4 * kPbGatherThreads) {
            if (e + 4 <= a1) {
                const uint2 tv = *reinterpret_cast<const uint2 *>(pb.tl + e);
                uint4 v;
                v.x = slice[tv.x & 0xFFFFu];
                v.y = slice[tv.x >> 16];
                v.z = slice[tv.y & 0xFFFFu];
                v.w = slice[tv.y >> 16];
                *reinterpret_cast<uint4 *>(pb.val + e) = v;
            } else {
                for (uint32_t f = e; f < a1; ++f) pb.val[f] = slice[pb.tl[f]];
            }
        }
    }
}

// Reads tile t's runs from every bucket (one flattened list, each edge's
// run found by its id, or for wider alphabets by binary search over the run
// starts) and places the gathered values into key[(state - tile start) * KC
// + letter].  Ends with a barrier.
template <int KC, uint32_t NT = kBlock>  // NT: threads of the workgroup
struct PbRunsLds {
    static constexpr bool kIds = KC <= 4;
    uint32_t rs[kPbMaxBuckets + 1];         // run starts, or deltas
    uint32_t rb[kIds ? 1 : kPbMaxBuckets];  // run bases (search)
    uint16_t rid[kIds ? kPbTile * KC : 2];  // run ids (small alphabets)
    uint32_t wsum[NT / 64];
    uint32_t tot;
};

template <int KC, uint32_t NT = kBlock>
__device__ __forceinline__ void pb_tile_keys(const PbArgs &pb, uint32_t t, uint32_t *key,
                                             PbRunsLds<KC, NT> &L) {
    const uint32_t tx = threadIdx.x;
    uint32_t total;
    if constexpr (PbRunsLds<KC, NT>::kIds) {
        total = pb_tile_run_ids<NT>(pb, t, L.rid, L.rs, nullptr, L.wsum, &L.tot);
    } else {
        pb_tile_runs<NT>(pb, t, L.rs, L.rb, L.wsum);
        total = L.rs[pb.nb];
    }
    // eight edges per thread at a time: every run lookup first, then all
    // their loads in flight together, then the LDS stores
    constexpr int B = 8;
    for (uint32_t j0 = 0; j0 < total; j0 += B * NT) {
        uint32_t e[B];
        bool ok[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t j = j0 + u * NT + tx;
            ok[u] = j < total;
            if constexpr (PbRunsLds<KC, NT>::kIds) {
                e[u] = ok[u] ? j + L.rs[L.rid[j]] : 0u;
            } else {
                const uint32_t lo = pb_run_of(L.rs, pb.nb, j);
                e[u] = ok[u] ? L.rb[lo] + (j - L.rs[lo]) : 0u;
            }
        }
        uint32_t sv[B], vv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            sv[u] = ok[u] ? pb.src[e[u]] : 0u;
            vv[u] = ok[u] ? pb.val[e[u]] : 0u;
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (ok[u]) key[sv[u]] = vv[u];
    }
    __syncthreads();
}

// Round 1 (packed labels) through the slices.  Pass A: the bucket's slice
// of round-0 byte labels (16 KB) into LDS, one byte per edge written next to
// it (the id array pb.val read as bytes).
__global__ __launch_bounds__(kPbGatherThreads) void k_pb_gather8(SigParams p) {
    __shared__ uint8_t slice[1u << kPbSliceLog];
    if (p.ctl->done) return;
    const PbArgs &pb = p.pb;
    uint8_t *__restrict__ val8 = reinterpret_cast<uint8_t *>(pb.val);
    constexpr uint32_t S = 1u << kPbSliceLog;
    const uint32_t tx = threadIdx.x;
    for (uint32_t b = blockIdx.x; b < pb.nb; b += gridDim.x) {
        const size_t s0 = static_cast<size_t>(b) * S;
        const uint32_t len = static_cast<uint32_t>(p.N - s0 < S ? p.N - s0 : S);
        __syncthreads();  // the previous bucket's gathers are done with the slice
        // (s0 is a multiple of 2^kPbSliceLog: four labels per aligned word)
        for (uint32_t i = 4 * tx; i < len; i += 4 * kPbGatherThreads) {
            if (i + 4 <= len) {
                *reinterpret_cast<uint32_t *>(slice + i) =
                    *reinterpret_cast<const uint32_t *>(p.lab8 + s0 + i);
            } else {
                for (uint32_t f = i; f < len; ++f) slice[f] = p.lab8[s0 + f];
            }
        }
        __syncthreads();
        const uint32_t lo = pb.bstart[b], hi = pb.bstart[b + 1];
        const uint32_t al = (lo + 3u) & ~3u;
        const uint32_t v0 = al < hi ? al : hi;
        for (uint32_t e = lo + tx; e < v0; e += kPbGatherThreads) val8[e] = slice[pb.tl[e]];
        for (uint32_t e = v0 + 4 * tx; e < hi; e += 4 * kPbGatherThreads) {
            if (e + 4 <= hi) {
                const uint2 tv = *reinterpret_cast<const uint2 *>(pb.tl + e);
                const uint32_t v = static_cast<uint32_t>(slice[tv.x & 0xFFFFu]) |
                                   static_cast<uint32_t>(slice[tv.x >> 16]) << 8 |
                                   static_cast<uint32_t>(slice[tv.y & 0xFFFFu]) << 16 |
                                   static_cast<uint32_t>(slice[tv.y >> 16]) << 24;
                *reinterpret_cast<uint32_t *>(val8 + e) = v;
            } else {
                for (uint32_t f = e; f < hi; ++f) val8[f] = slice[pb.tl[f]];
            }
        }
    }
}

// Pass B of round 1: tile t's byte labels from every bucket into
// key8[(state - tile start) * KC + letter], as pb_tile_keys does with ids.
// Ends with a barrier.
template <int KC, uint32_t NT = kBlock>
__device__ __forceinline__ void pb_tile_keys8(const PbArgs &pb, uint32_t t, uint8_t *key8,
                                              PbRunsLds<KC, NT> &L) {
    const uint32_t tx = threadIdx.x;
    const uint8_t *__restrict__ val8 = reinterpret_cast<const uint8_t *>(pb.val);
    uint32_t total;
    if constexpr (PbRunsLds<KC, NT>::kIds) {
        total = pb_tile_run_ids<NT>(pb, t, L.rid, L.rs, nullptr, L.wsum, &L.tot);
    } else {
        pb_tile_runs<NT>(pb, t, L.rs, L.rb, L.wsum);
        total = L.rs[pb.nb];
    }
    constexpr int B = 8;
    for (uint32_t j0 = 0; j0 < total; j0 += B * NT) {
        uint32_t e[B];
        bool ok[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t j = j0 + u * NT + tx;
            ok[u] = j < total;
            if constexpr (PbRunsLds<KC, NT>::kIds) {
                e[u] = ok[u] ? j + L.rs[L.rid[j]] : 0u;
            } else {
                const uint32_t lo = pb_run_of(L.rs, pb.nb, j);
                e[u] = ok[u] ? L.rb[lo] + (j - L.rs[lo]) : 0u;
            }
        }
        uint32_t sv[B], vv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            sv[u] = ok[u] ? pb.src[e[u]] : 0u;
            vv[u] = ok[u] ? val8[e[u]] : 0u;
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (ok[u]) key8[sv[u]] = static_cast<uint8_t>(vv[u]);
    }
    __syncthreads();
}

// Pass B of round 1 (packed labels, k_eff <= 4): one workgroup per source
// tile; the keys and the distinct-label count as k_packed_round computes
// them, the tile's states taken 2 * kBlock at a time so that the LDS label
// set (emptied when half full) always has room.
template <int KC, uint32_t NT>
__global__ __launch_bounds__(NT) void k_packed_pb(SigParams p) {
    __shared__ uint8_t key8[kPbTile * KC];
    __shared__ PbRunsLds<KC, NT> runs;
    __shared__ uint32_t lset[kLabelSlots];
    __shared__ uint32_t lfill;
    if (p.ctl->done) return;
    const PbArgs &pb = p.pb;
    const uint32_t r = p.ctl->round;
    uint32_t *__restrict__ Y = (r & 1u) ? p.blockA : p.blockB;
    constexpr uint32_t bits = KC + 1;
    constexpr int EP = kPbTile / NT;
    static_assert(2 * NT <= kLabelSlots / 2, "a step's labels must fit a half-empty label set");
    const uint32_t tx = threadIdx.x;
    for (uint32_t i = tx; i < kLabelSlots; i += NT) lset[i] = ~0u;
    if (tx == 0) lfill = 0;
    __syncthreads();
    for (uint32_t t = blockIdx.x; t < pb.ntiles; t += gridDim.x) {
        const size_t base = static_cast<size_t>(t) * kPbTile;
        uint32_t own[EP];
#pragma unroll
        for (int e = 0; e < EP; ++e) {
            const size_t q = base + e * NT + tx;
            own[e] = q < p.N ? p.lab8[q] : 0u;
        }
        pb_tile_keys8<KC, NT>(pb, t, key8, runs);
#pragma unroll
        for (int e0 = 0; e0 < EP; e0 += 2) {
            // every thread reads the same fill (the last step ended with a
            // barrier, and so did the key assembly) before any thread
            // inserts; a step adds at most 2 * NT labels to a set at
            // most half full
            const bool half_full = lfill > kLabelSlots / 2;
            __syncthreads();
            if (half_full) {
                for (uint32_t i = tx; i < kLabelSlots; i += NT) lset[i] = ~0u;
                if (tx == 0) lfill = 0;
                __syncthreads();
            }
#pragma unroll
            for (int e = e0; e < e0 + 2; ++e) {
                const uint32_t i = e * NT + tx;
                const size_t q = base + i;
                if (q >= p.N) continue;
                uint32_t key = own[e];
#pragma unroll
                for (int j = 0; j < KC; ++j)
                    key |= static_cast<uint32_t>(key8[i * KC + j]) << (bits * (j + 1));
                Y[q] = key;
                uint32_t slot = (key * 0x9E3779B1u) >> 20;  // 12 bits: kLabelSlots
                bool first = false;
                for (;;) {
                    const uint32_t v = __hip_atomic_load(lset + slot, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (v == key) break;
                    if (v == ~0u) {
                        const uint32_t prev = atomicCAS(lset + slot, ~0u, key);
                        if (prev == ~0u) {
                            first = true;
                            atomicAdd(&lfill, 1u);
                            break;
                        }
                        if (prev == key) break;
                    }
                    slot = (slot + 1) & (kLabelSlots - 1);
                }
                if (first) label_present(p.presence_packed, key);
            }
            // the step's inserts are done before any thread reads the fill
            // for the next step (every thread must see the same fill: the
            // emptying branch holds a barrier)
            __syncthreads();
        }
    }
}

// Pass B: one workgroup per source tile of kPbTile states: the tile's keys
// from the buckets, then what the signature kernel does with each state.
template <int KC, uint32_t NT>
__global__ __launch_bounds__(NT) void k_signature_pb(SigParams p) {
    __shared__ uint32_t key[kPbTile * KC];
    __shared__ PbRunsLds<KC, NT> runs;
    if (!pb_round(p.pb, *p.ctl, p.N)) return;
    const PbArgs &pb = p.pb;
    const uint32_t r = p.ctl->round;
    const uint32_t *__restrict__ X = (r & 1u) ? p.blockB : p.blockA;
    uint32_t *__restrict__ Y = (r & 1u) ? p.blockA : p.blockB;
    const bool all = r <= p.ctl->all_active_until;
    const bool inc = !all && incremental_round(*p.ctl, p.N, r);
    const size_t words = (p.N + 63) / 64;
    const unsigned long long *__restrict__ T = p.touched + (r & 1u) * words;
    constexpr size_t W = KC + 1;
    uint32_t leaders = 0, claims = 0;
    const uint32_t tx = threadIdx.x;
    constexpr int EP = kPbTile / NT;  // states per thread in a tile
    for (uint32_t t = blockIdx.x; t < pb.ntiles; t += gridDim.x) {
        const size_t base = static_cast<size_t>(t) * kPbTile;
        // the tile's own ids are loaded before its keys are assembled, so
        // their latency overlaps that work instead of following it
        uint32_t w0s[EP], mqs[EP];
        unsigned long long sws[EP], aws[EP];
#pragma unroll
        for (int e = 0; e < EP; ++e) {
            const size_t q = base + e * NT + tx;
            const size_t first = q - lane_id();
            w0s[e] = q < p.N ? X[q] : 0u;
            sws[e] = (!all && first < p.N) ? p.single[first >> 6] : ~0ull;
            aws[e] = (!all && first < p.N) ? p.active[first >> 6] : 0ull;
            mqs[e] = (!all && !inc && q < p.N) ? p.multi[q] : ~0u;
        }
        pb_tile_keys<KC, NT>(pb, t, key, runs);
#pragma unroll
        for (int e = 0; e < EP; ++e) {
            const uint32_t i = e * NT + tx;
            const size_t q = base + i;
            // (the whole wave takes part in the ballots below)
            const uint32_t w0 = w0s[e];
            bool act;
            if (all) {
                act = q < p.N;
                const size_t first = q - lane_id();
                const unsigned long long am = __ballot(act);
                if (lane_id() == 0 && first < p.N) p.active[first >> 6] = am;
            } else {
                bool was;
                act = select_state_words(p, q, w0, r, inc, T, sws[e], aws[e], mqs[e], was);
                if (q < p.N && !act) {
                    if (was) Y[q] = w0;
                    leaders += w0 == q ? 1u : 0u;
                }
            }
            if (act) {
                uint32_t w[KC];
#pragma unroll
                for (int a = 0; a < KC; ++a) w[a] = key[i * KC + a];
                emit_key(p, Y, q, w0, w, KC, W, !all && p.grouping == 0, claims);
            }
        }
        __syncthreads();  // the keys are done with before the next tile
    }
    wg_add_spread<NT>(p.counters, 0, leaders + claims);
    wg_add_spread<NT>(p.counters, 3, claims);
}

// ---------------------------------------------------------------- grouping

struct InsParams {
    const uint32_t *sig;
    const uint64_t *hash;
    size_t N;
    uint32_t W;
    unsigned long long *table;
    uint64_t mask;
    uint32_t *blockA, *blockB;
    uint32_t *multi;
    const unsigned long long *active;
    uint32_t *counters;
    const RoundCtl *ctl;
    uint32_t cached_probe;
    int lds_stage;
    unsigned long long *chg;
    unsigned long long *chg_sum;
    const uint8_t *tile_dead;  // segmented refinements: decided tiles (else null)
};

// Stores a wave's changed-id mask and sets the summary bits of its groups
// with a changed state (lane 0 only).
__device__ __forceinline__ void store_changed(unsigned long long *chg, unsigned long long *chg_sum,
                                              size_t N, uint32_t r, size_t first,
                                              unsigned long long cm) {
    if (lane_id() != 0 || first >= N) return;
    chg[first >> 6] = cm;
    set_summary(chg_sum + (r & 1u) * summary_words(N), first, cm);
}

// Whether this round stages keys in LDS (uniform across the grid).
__device__ __forceinline__ bool stage_in_lds(const InsParams &p) {
    // 1 (and the automatic mode 2): every round pre-groups in LDS.  Measured
    // on MI355X, staging every round was as fast as grouping directly on
    // random DFAs (within 1-4%) and up to 2.2x faster on chains,
    // bit-splitters and Fibonacci words, whose block members share tiles;
    // choosing by the previous round's duplicate rate lost up to 10% there.
    return p.lds_stage != 0;
}

// Counter words: [0] blocks after the round, [1] states not refined,
// [2] states whose id changed, [3] blocks formed by claims.  The signature
// kernel adds the unrefined block holders and its own claims.
__device__ __forceinline__ void insert_body(const InsParams &p) {
    if (p.ctl->done || stage_in_lds(p)) return;
    const uint32_t r = p.ctl->round;
    const uint32_t epoch = r % kEpochs + 1;
    const bool all = r <= p.ctl->all_active_until;
    const uint32_t *__restrict__ X = (r & 1u) ? p.blockB : p.blockA;
    uint32_t *__restrict__ Y = (r & 1u) ? p.blockA : p.blockB;
    uint32_t blocks = 0, idle = 0, changed = 0;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kBlock; base < p.N;
         base += static_cast<size_t>(gridDim.x) * kBlock) {
        if (tiles_dead(p.tile_dead, p.N, base, kBlock)) {
            if (threadIdx.x == 0) idle += states_in(p.N, base, kBlock);
            continue;
        }
        const size_t q = base + threadIdx.x;
        const size_t first = base + (threadIdx.x & ~63u);
        const unsigned long long am = first < p.N ? p.active[first >> 6] : 0ull;
        const bool valid = q < p.N;
        const bool act = valid && ((am >> lane_id()) & 1ull);
        idle += (valid && !act) ? 1u : 0u;
        bool ch = false;
        if (act) {
            const uint32_t x = X[q];
            // the state holding its block's id kept it in the signature
            // kernel; a member with the same key joins it directly
            if (!all && x != q && rows_equal(p.sig, p.W, q, x)) {
                Y[q] = x;
                mark_multi(p.multi, x, r + 1);
            } else if (all || x != q) {
                bool claimed = false;
                const uint32_t id = find_or_claim(p.table, p.mask, epoch, p.hash[q],
                                                  static_cast<uint32_t>(q), p.sig, p.W,
                                                  p.cached_probe != 0, claimed);
                Y[q] = id;
                if (claimed)
                    ++blocks;
                else
                    mark_multi(p.multi, id, r + 1);
                ch = id != x;
            }
        }
        const unsigned long long cm = __ballot(ch);
        store_changed(p.chg, p.chg_sum, p.N, r, first, cm);
        changed += ch ? 1u : 0u;
    }
    wg_add_spread(p.counters, 0, blocks);
    wg_add_spread(p.counters, 1, idle);
    wg_add_spread(p.counters, 2, changed);
    wg_add_spread(p.counters, 3, blocks);
}

// LDS-staged grouping: a workgroup first groups the refined states of its
// tile of kBlock states in an LDS table (full-key compare), then only the
// first state of each local group goes to the HBM table; the others copy its
// result through LDS.

__device__ __forceinline__ void insert_lds_body(const InsParams &p) {
    __shared__ unsigned long long ltab[kLdsSlots];
    __shared__ uint32_t gid[kBlock];
    __shared__ uint32_t lsize[kBlock];
    if (p.ctl->done || !stage_in_lds(p)) return;
    const uint32_t r = p.ctl->round;
    const uint32_t epoch = r % kEpochs + 1;
    const bool all = r <= p.ctl->all_active_until;
    const uint32_t *__restrict__ X = (r & 1u) ? p.blockB : p.blockA;
    uint32_t *__restrict__ Y = (r & 1u) ? p.blockA : p.blockB;
    const uint32_t tx = threadIdx.x;
    uint32_t blocks = 0, idle = 0, changed = 0;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kBlock; base < p.N;
         base += static_cast<size_t>(gridDim.x) * kBlock) {
        if (tiles_dead(p.tile_dead, p.N, base, kBlock)) {
            if (tx == 0) idle += states_in(p.N, base, kBlock);
            continue;
        }
        const size_t q = base + tx;
        const size_t first = base + (tx & ~63u);
        const unsigned long long am = first < p.N ? p.active[first >> 6] : 0ull;
        const bool valid = q < p.N;
        const bool act = valid && ((am >> lane_id()) & 1ull);
        idle += (valid && !act) ? 1u : 0u;
        // whole tile idle: nothing to group (uniform across the workgroup)
        if (__syncthreads_or(act) == 0) {
            if (lane_id() == 0 && first < p.N) p.chg[first >> 6] = 0ull;
            continue;
        }
        const uint32_t x = act ? X[q] : 0u;
        // the state holding its block's id kept it in the signature kernel;
        // a member with the same key joins it directly, the others group in
        // LDS first
        const bool joins = act && !all && x != q && rows_equal(p.sig, p.W, q, x);
        if (joins) {
            Y[q] = x;
            mark_multi(p.multi, x, r + 1);
        }
        const bool grp = act && !joins && (all || x != q);
        for (uint32_t i = tx; i < kLdsSlots; i += kBlock) ltab[i] = kEmptyPair;
        lsize[tx] = 0;
        __syncthreads();
        const uint64_t h = grp ? p.hash[q] : 0;
        uint32_t lead = tx;
        if (grp) {
            const uint32_t ltag = static_cast<uint32_t>(h >> 32);
            uint32_t s = static_cast<uint32_t>(h) & (kLdsSlots - 1);
            for (;;) {
                unsigned long long e =
                    __hip_atomic_load(ltab + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (e == kEmptyPair) {
                    const unsigned long long want = (static_cast<unsigned long long>(ltag) << 32) | tx;
                    const unsigned long long prev = atomicCAS(ltab + s, kEmptyPair, want);
                    if (prev == kEmptyPair) {
                        lead = tx;
                        break;
                    }
                    e = prev;
                }
                if (static_cast<uint32_t>(e >> 32) == ltag) {
                    const uint32_t other = static_cast<uint32_t>(e);
                    if (rows_equal(p.sig, p.W, q, base + other)) {
                        lead = other;
                        break;
                    }
                }
                s = (s + 1) & (kLdsSlots - 1);
            }
            atomicAdd(lsize + lead, 1u);
        }
        __syncthreads();
        if (grp && lead == tx) {
            bool claimed = false;
            const uint32_t id = find_or_claim(p.table, p.mask, epoch, h, static_cast<uint32_t>(q),
                                              p.sig, p.W, p.cached_probe != 0, claimed);
            gid[tx] = id;
            if (claimed) ++blocks;
            if (!claimed || lsize[tx] > 1) mark_multi(p.multi, id, r + 1);
        }
        __syncthreads();
        bool ch = false;
        if (grp) {
            const uint32_t id = gid[lead];
            Y[q] = id;
            ch = id != x;
        }
        const unsigned long long cm = __ballot(ch);
        store_changed(p.chg, p.chg_sum, p.N, r, first, cm);
        changed += ch ? 1u : 0u;
        __syncthreads();
    }
    wg_add_spread(p.counters, 0, blocks);
    wg_add_spread(p.counters, 1, idle);
    wg_add_spread(p.counters, 2, changed);
    wg_add_spread(p.counters, 3, blocks);
}

// The same grouping with two states per thread (tiles of 2 * kBlock
// states) and the signature width known at compile time (KC = k_eff > 0):
// the reads of both states' rows, their holders' rows and their hashes are
// in flight together, and the probes of the two states' tile leaders are
// issued one after the other without waiting in between (the kernel is
// bound by the latency of these dependent random reads).
template <int KC>
__device__ __forceinline__ bool rows_equal_fixed(const uint32_t *__restrict__ sig, size_t a,
                                                 size_t b) {
    constexpr int W = KC + 1;
    const uint32_t *ra = sig + a * W;
    const uint32_t *rb = sig + b * W;
    uint32_t va[W], vb[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
        va[i] = ra[i];
        vb[i] = rb[i];
    }
    bool eq = true;
#pragma unroll
    for (int i = 0; i < W; ++i) eq &= va[i] == vb[i];
    return eq;
}

template <int KC>
__device__ __forceinline__ void insert_lds2_body(const InsParams &p) {
    constexpr int S = 2;
    constexpr uint32_t kTile = S * kBlock;
    constexpr uint32_t kSlots2 = 2 * kTile;
    __shared__ unsigned long long ltab[kSlots2];
    __shared__ uint32_t gid[kTile];
    __shared__ uint32_t lsize[kTile];
    if (p.ctl->done || !stage_in_lds(p)) return;
    const uint32_t r = p.ctl->round;
    const uint32_t epoch = r % kEpochs + 1;
    const bool all = r <= p.ctl->all_active_until;
    const uint32_t *__restrict__ X = (r & 1u) ? p.blockB : p.blockA;
    uint32_t *__restrict__ Y = (r & 1u) ? p.blockA : p.blockB;
    const uint32_t tx = threadIdx.x;
    uint32_t blocks = 0, idle = 0, changed = 0;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kTile; base < p.N;
         base += static_cast<size_t>(gridDim.x) * kTile) {
        if (tiles_dead(p.tile_dead, p.N, base, kTile)) {
            if (tx == 0) idle += states_in(p.N, base, kTile);
            continue;
        }
        size_t q[S], first[S];
        bool act[S];
        uint32_t loc[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            loc[i] = i * kBlock + tx;
            q[i] = base + loc[i];
            first[i] = q[i] - lane_id();
            const unsigned long long am = first[i] < p.N ? p.active[first[i] >> 6] : 0ull;
            act[i] = q[i] < p.N && ((am >> lane_id()) & 1ull);
            idle += (q[i] < p.N && !act[i]) ? 1u : 0u;
        }
        // whole tile idle: nothing to group (uniform across the workgroup)
        if (__syncthreads_or(act[0] || act[1]) == 0) {
#pragma unroll
            for (int i = 0; i < S; ++i)
                if (lane_id() == 0 && first[i] < p.N) p.chg[first[i] >> 6] = 0ull;
            continue;
        }
        uint32_t x[S];
#pragma unroll
        for (int i = 0; i < S; ++i) x[i] = act[i] ? X[q[i]] : 0u;
        // the state holding its block's id kept it in the signature kernel;
        // a member with the same key joins it directly, the others group in
        // LDS first
        bool joins[S], grp[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const bool cand = act[i] && !all && x[i] != q[i];
            joins[i] = cand && rows_equal_fixed<KC>(p.sig, q[i], x[i]);
        }
        uint64_t h[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (joins[i]) {
                Y[q[i]] = x[i];
                mark_multi(p.multi, x[i], r + 1);
            }
            grp[i] = act[i] && !joins[i] && (all || x[i] != q[i]);
            h[i] = grp[i] ? p.hash[q[i]] : 0;
        }
        for (uint32_t i = tx; i < kSlots2; i += kBlock) ltab[i] = kEmptyPair;
#pragma unroll
        for (int i = 0; i < S; ++i) lsize[loc[i]] = 0;
        __syncthreads();
        uint32_t lead[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            lead[i] = loc[i];
            if (!grp[i]) continue;
            const uint32_t ltag = static_cast<uint32_t>(h[i] >> 32);
            uint32_t sl = static_cast<uint32_t>(h[i]) & (kSlots2 - 1);
            for (;;) {
                unsigned long long e =
                    __hip_atomic_load(ltab + sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (e == kEmptyPair) {
                    const unsigned long long want =
                        (static_cast<unsigned long long>(ltag) << 32) | loc[i];
                    const unsigned long long prev = atomicCAS(ltab + sl, kEmptyPair, want);
                    if (prev == kEmptyPair) break;
                    e = prev;
                }
                if (static_cast<uint32_t>(e >> 32) == ltag) {
                    const uint32_t other = static_cast<uint32_t>(e);
                    if (rows_equal_fixed<KC>(p.sig, q[i], base + other)) {
                        lead[i] = other;
                        break;
                    }
                }
                sl = (sl + 1) & (kSlots2 - 1);
            }
            atomicAdd(lsize + lead[i], 1u);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (!grp[i] || lead[i] != loc[i]) continue;
            bool claimed = false;
            const uint32_t id = find_or_claim(p.table, p.mask, epoch, h[i],
                                              static_cast<uint32_t>(q[i]), p.sig, p.W,
                                              p.cached_probe != 0, claimed);
            gid[loc[i]] = id;
            if (claimed) ++blocks;
            if (!claimed || lsize[loc[i]] > 1) mark_multi(p.multi, id, r + 1);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < S; ++i) {
            bool ch = false;
            if (grp[i]) {
                const uint32_t id = gid[lead[i]];
                Y[q[i]] = id;
                ch = id != x[i];
            }
            const unsigned long long cm = __ballot(ch);
            store_changed(p.chg, p.chg_sum, p.N, r, first[i], cm);
            changed += ch ? 1u : 0u;
        }
        __syncthreads();
    }
    wg_add_spread(p.counters, 0, blocks);
    wg_add_spread(p.counters, 1, idle);
    wg_add_spread(p.counters, 2, changed);
    wg_add_spread(p.counters, 3, blocks);
}

// One workgroup: the round's block count (spread counters), the stop tests,
// and the counter reset.
__device__ __forceinline__ void round_end_body(RoundCtl *ctl, const uint32_t *blockA,
                                               const uint32_t *blockB, uint32_t *counters,
                                               uint32_t N) {
    constexpr int kWords = 4;  // blocks, idle states, changed ids, claims
    __shared__ uint32_t red[kWords][kBlock / 64];
    if (ctl->done) return;
    const uint32_t r = ctl->round;
    uint32_t v[kWords] = {0, 0, 0, 0};
    for (uint32_t i = threadIdx.x; i < kSpread; i += kBlock)
        for (int w = 0; w < kWords; ++w) {
            v[w] += counters[i * kSpreadStride + w];
            counters[i * kSpreadStride + w] = 0;
        }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        for (int w = 0; w < kWords; ++w) v[w] += __shfl_xor(v[w], d, 64);
    if (lane_id() == 0)
        for (int w = 0; w < kWords; ++w) red[w][threadIdx.x / 64] = v[w];
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 0; w < kWords; ++w) {
        v[w] = 0;
        for (int i = 0; i < kBlock / 64; ++i) v[w] += red[w][i];
    }
    const uint32_t c = v[0], idle = v[1];
    const uint32_t *out = (r & 1u) ? blockA : blockB;
    ctl->last_gain = c - ctl->prev_count;
    ctl->last_active = N - idle;
    ctl->last_claims = v[3];
    ctl->last_changed = v[2];
    ctl->active_sum += N - idle;
    ctl->active_hist[r % kActiveHist] = N - idle;
    ctl->gain_hist[r % kActiveHist] = c - ctl->prev_count;
    if (c == ctl->prev_count) {
        ctl->stable = 1;
        ctl->done = 1;
    } else {
        ctl->changing += 1;
        ctl->prev_count = c;
    }
    if (ctl->check_eq && out[ctl->eq_a] != out[ctl->eq_b]) {
        ctl->separated = 1;
        ctl->done = 1;
    }
    ctl->round = r + 1;
    if (!ctl->done && ctl->max_rounds && r + 1 >= ctl->max_rounds) {
        ctl->limit = 1;
        ctl->done = 1;
    }
}

// The round kernels: one launch per phase (host, chunk and graph loops).
template <int KC>
__global__ __launch_bounds__(kBlock) void k_mark(SigParams p) {
    mark_body<KC>(p);
}

template <int KC>
__global__ __launch_bounds__(kBlock) void k_signature(SigParams p) {
    signature_body<KC>(p);
}

__global__ __launch_bounds__(kBlock) void k_insert(InsParams p) { insert_body(p); }

__global__ __launch_bounds__(kBlock) void k_insert_lds(InsParams p) { insert_lds_body(p); }

template <int KC>
__global__ __launch_bounds__(kBlock) void k_insert_lds2(InsParams p) { insert_lds2_body<KC>(p); }

__global__ __launch_bounds__(kBlock) void k_round_end(RoundCtl *ctl, const uint32_t *blockA,
                                                       const uint32_t *blockB, uint32_t *counters,
                                                       uint32_t N) {
    round_end_body(ctl, blockA, blockB, counters, N);
}


// ---------------------------------------------------------------- segmented refinement

__device__ __forceinline__ uint32_t find_part(const SegArgs &g, size_t q) {
    uint32_t p = g.tile_part[q / kBlock];
    while (static_cast<size_t>(g.parts[p].off) + g.parts[p].n <= q) ++p;
    return p;
}

__global__ __launch_bounds__(kBlock) void k_ingest_parts(SegArgs g, size_t N, uint32_t k,
                                                          uint32_t *__restrict__ cols,
                                                          uint32_t *err, uint32_t *nonid) {
    bool bad = false;
    unsigned long long moves = 0;
    for (size_t q = global_tid(); q < N; q += grid_stride()) {
        const Part P = g.parts[find_part(g, q)];
        const size_t i = q - P.off;
        for (uint32_t a = 0; a < k; ++a) {
            uint32_t t = static_cast<uint32_t>(i);  // padding letters are the identity
            if (a < P.k) {
                t = P.delta[i * P.k + a];
                if (t >= P.n) {
                    bad = true;
                    t = 0;
                }
            }
            if (t != i) {
                if (a < 64)
                    moves |= 1ull << a;
                else if (nonid[a] == 0u)
                    nonid[a] = 1u;
            }
            cols[static_cast<size_t>(a) * N + q] = t + P.off;
        }
    }
    wave_set_flag(err, bad);
    moves = wave_or64(moves);
    if (lane_id() == 0) {
        while (moves) {
            const int a = __ffsll(moves) - 1;
            moves &= moves - 1;
            if (nonid[a] == 0u) nonid[a] = 1u;
        }
    }
}

// The classes present in each segment are gathered per tile in LDS (a tile
// spans at most kBlock segments), then OR-ed into seg_flags once per tile and
// segment: per-state atomics on one word per segment serialised.
__global__ __launch_bounds__(kBlock) void k_init_parts(SegArgs g, size_t N,
                                                        uint32_t *__restrict__ block,
                                                        unsigned long long *accbits) {
    __shared__ uint32_t lflag[kBlock];
    __shared__ uint32_t seg_first;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kBlock; base < N;
         base += static_cast<size_t>(gridDim.x) * kBlock) {
        lflag[threadIdx.x] = 0;
        if (threadIdx.x == 0) seg_first = g.parts[g.tile_part[base / kBlock]].seg;
        __syncthreads();
        const size_t q = base + threadIdx.x;
        bool f = false;
        if (q < N) {
            const Part P = g.parts[find_part(g, q)];
            f = P.accepting[q - P.off] != 0;
            block[q] = 2u * P.seg + (f ? 1u : 0u);
            atomicOr(lflag + (P.seg - seg_first), f ? 1u : 2u);
        }
        const unsigned long long fm = __ballot(f);
        if (lane_id() == 0 && q < N) accbits[q >> 6] = fm;
        __syncthreads();
        const uint32_t m = lflag[threadIdx.x];
        if (m) atomicOr(g.seg_flags + seg_first + threadIdx.x, m);
        __syncthreads();
    }
}

// Round 0 of a segmented refinement refines the initial labels 2 * segment
// + accepting, so a state's key is its segment and the acceptance of the
// state and of each successor (section 3.3, the first signature round): at
// most 2^(k_eff + 1) keys per segment.  They index a table of nseg <<
// (k_eff + 1) words in which each key keeps its smallest state (LDS minimum
// per workgroup, then one atomicMin per key present in the workgroup); that
// state becomes the block id of every state with the key.  The ids are then
// state indices with the same partition as a table round's, so the rounds
// after it run unchanged.  A padding letter of a part (the identity) gives
// the state's own acceptance without a load.
constexpr uint32_t kSegPatTile = 4 * kBlock;   // states per workgroup step
constexpr uint32_t kSegPatLds = 4096;          // keys kept in LDS per step

__global__ __launch_bounds__(kBlock) void k_segpat_min(SigParams p, SegArgs g,
                                                        uint32_t *table, uint16_t *pat,
                                                        uint32_t bits) {
    __shared__ uint32_t lmin[kSegPatLds];
    __shared__ uint32_t seg_first;
    if (p.ctl->done || p.ctl->round != 0) return;
    const size_t nkeys = static_cast<size_t>(g.nseg) << bits;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kSegPatTile; base < p.N;
         base += static_cast<size_t>(gridDim.x) * kSegPatTile) {
        for (uint32_t i = threadIdx.x; i < kSegPatLds; i += kBlock) lmin[i] = ~0u;
        if (threadIdx.x == 0) seg_first = g.parts[g.tile_part[base / kBlock]].seg;
        __syncthreads();
        for (uint32_t u = 0; u < kSegPatTile / kBlock; ++u) {
            const size_t q = base + u * kBlock + threadIdx.x;
            if (q >= p.N) break;
            const Part P = g.parts[find_part(g, q)];
            const uint32_t own = static_cast<uint32_t>((p.accbits[q >> 6] >> (q & 63)) & 1ull);
            uint32_t key = own;
            // eight letters' loads at a time, then their acceptance bits
            for (uint32_t a0 = 0; a0 < p.k_eff; a0 += 8) {
                uint32_t t[8];
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j) {
                    const uint32_t a = a0 + j;
                    t[j] = (a < p.k_eff && p.colmap[a] < P.k)
                               ? p.cols[static_cast<size_t>(p.colmap[a]) * p.N + q]
                               : static_cast<uint32_t>(q);
                }
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j) {
                    const uint32_t a = a0 + j;
                    if (a >= p.k_eff) break;
                    const uint32_t bit =
                        t[j] == q ? own
                                  : static_cast<uint32_t>((p.accbits[t[j] >> 6] >> (t[j] & 63)) & 1ull);
                    key |= bit << (a + 1);
                }
            }
            pat[q] = static_cast<uint16_t>(key);
            const size_t local = (static_cast<size_t>(P.seg - seg_first) << bits) | key;
            if (local < kSegPatLds)
                atomicMin(lmin + local, static_cast<uint32_t>(q));
            else
                atomicMin(table + ((static_cast<size_t>(P.seg) << bits) | key),
                          static_cast<uint32_t>(q));
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < kSegPatLds; i += kBlock) {
            const size_t k = (static_cast<size_t>(seg_first) << bits) + i;
            if (lmin[i] != ~0u && k < nkeys) atomicMin(table + k, lmin[i]);
        }
        __syncthreads();
    }
}

// Every state takes its key's smallest state as its block id; the round's
// bookkeeping as the grouping kernels do it (refined-state masks, block
// marks, changed-id bits and summary, the spread counters).
__global__ __launch_bounds__(kBlock) void k_segpat_assign(SigParams p, SegArgs g,
                                                           const uint32_t *table,
                                                           const uint16_t *pat, uint32_t bits,
                                                           uint32_t *multi) {
    if (p.ctl->done || p.ctl->round != 0) return;
    const uint32_t r = 0;
    const uint32_t *__restrict__ X = p.blockA;
    uint32_t *__restrict__ Y = p.blockB;
    uint32_t blocks = 0, changed = 0;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kBlock; base < p.N;
         base += static_cast<size_t>(gridDim.x) * kBlock) {
        const size_t q = base + threadIdx.x;
        const bool valid = q < p.N;
        bool ch = false;
        if (valid) {
            const uint32_t seg = g.parts[find_part(g, q)].seg;
            const uint32_t id = table[(static_cast<size_t>(seg) << bits) | pat[q]];
            Y[q] = id;
            if (id == q)
                ++blocks;
            else
                mark_multi(multi, id, r + 1);
            ch = id != X[q];
            changed += ch ? 1u : 0u;
        }
        const size_t first = q - lane_id();
        const unsigned long long am = __ballot(valid);
        if (lane_id() == 0 && first < p.N) p.active[first >> 6] = am;
        const unsigned long long cm = __ballot(ch);
        store_changed(p.chg, p.chg_sum, p.N, r, first, cm);
    }
    wg_add_spread(p.counters, 0, blocks);
    wg_add_spread(p.counters, 2, changed);
    wg_add_spread(p.counters, 3, blocks);
}

// seg_prev[s] = classes of segment s; *init_count = their sum.
__global__ __launch_bounds__(kBlock) void k_seg_init(SegArgs g) {
    uint32_t sum = 0;
    for (size_t s = global_tid(); s < g.nseg; s += grid_stride()) {
        const uint32_t c = __popc(g.seg_flags[s]);
        g.seg_prev[s] = c;
        g.seg_changing[s] = 0;
        g.seg_cnt[s] = 0;
        sum += c;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
    if (lane_id() == 0 && sum) atomicAdd(g.init_count, sum);
}

// Blocks per segment after the round: the states that are their block's id
// (a block's id is the state that first claimed its signature).  Counts are
// aggregated per tile in LDS (a tile spans at most kBlock segments).
__device__ __forceinline__ void seg_count_body(const SegArgs &g, size_t N, const RoundCtl *ctl,
                                               const uint32_t *blockA, const uint32_t *blockB) {
    __shared__ uint32_t lcnt[kBlock];
    __shared__ uint32_t seg_first, tile_live, tile_dies, holders;
    if (ctl->done) return;
    const uint32_t r = ctl->round;
    const uint32_t *__restrict__ Y = (r & 1u) ? blockA : blockB;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kBlock; base < N;
         base += static_cast<size_t>(gridDim.x) * kBlock) {
        lcnt[threadIdx.x] = 0;
        if (threadIdx.x == 0) {
            // a tile whose segments are all decided has nothing to count (and
            // never has again: a decided segment stays decided)
            const size_t t = base / kBlock;
            uint32_t live = 0, dies = 0;
            if (!g.tile_dead[t]) {
                uint32_t p = g.tile_part[t];
                seg_first = g.parts[p].seg;
                const size_t end = base + kBlock < N ? base + kBlock : N;
                for (; p < g.nparts && g.parts[p].off < end; ++p)
                    live |= g.seg_done[g.parts[p].seg] == 0u;
                dies = !live;
            }
            tile_live = live;
            tile_dies = dies;
            holders = 0;
        }
        __syncthreads();
        if (!tile_live) {
            if (tile_dies) {
                // the round kernels skip the tile from the next round on and
                // count its block holders from here: the states of its
                // segments were refined for the last time two rounds ago, and
                // the round after that copied their ids into both buffers
                const size_t q = base + threadIdx.x;
                const unsigned long long hm = __ballot(q < N && Y[q] == q);
                if (lane_id() == 0 && hm) atomicAdd(&holders, static_cast<uint32_t>(__popcll(hm)));
                __syncthreads();
                if (threadIdx.x == 0) {
                    g.tile_lead[base / kBlock] = static_cast<uint16_t>(holders);
                    g.tile_dead[base / kBlock] = 1;
                }
            }
            __syncthreads();  // every thread has read tile_live
            continue;
        }
        const size_t q = base + threadIdx.x;
        if (q < N && Y[q] == q) {
            const uint32_t seg = g.parts[find_part(g, q)].seg;
            if (g.seg_done[seg] == 0u) atomicAdd(lcnt + (seg - seg_first), 1u);
        }
        __syncthreads();
        const uint32_t c = lcnt[threadIdx.x];
        if (c) atomicAdd(g.seg_cnt + seg_first + threadIdx.x, c);
        __syncthreads();
    }
}

// Per-segment end of round: a segment whose block count did not change is
// stable (its partition never changes again: the segments are disjoint), and
// a pair whose start states got different ids is separated; either way the
// segment is decided in this round.
__device__ __forceinline__ void seg_end_body(const SegArgs &g, const RoundCtl *ctl,
                                             const uint32_t *blockA, const uint32_t *blockB) {
    if (ctl->done) return;
    const uint32_t r = ctl->round;
    const uint32_t *__restrict__ Y = (r & 1u) ? blockA : blockB;
    for (size_t s = global_tid(); s < g.nseg; s += grid_stride()) {
        if (g.seg_done[s]) continue;
        const uint32_t c = g.seg_cnt[s];
        g.seg_cnt[s] = 0;
        if (c == g.seg_prev[s]) {
            g.seg_done[s] = r + 1;
            continue;
        }
        g.seg_changing[s] += 1;
        g.seg_prev[s] = c;
        if (g.pairs) {
            const Part A = g.parts[2 * s], B = g.parts[2 * s + 1];
            if (Y[A.off + A.start] != Y[B.off + B.start]) g.seg_done[s] = r + 1;
        }
    }
}

// The states of the segments decided in this round are marked as skipped in
// the singleton bits (one workgroup per segment; the bits of a word shared
// with a neighbouring segment are set atomically).
__device__ __forceinline__ void seg_freeze_body(const SegArgs &g, const RoundCtl *ctl,
                                                unsigned long long *single) {
    if (ctl->done) return;
    const uint32_t r = ctl->round;
    for (size_t s = blockIdx.x; s < g.nseg; s += gridDim.x) {
        if (g.seg_done[s] != r + 1) continue;
        const Part first = g.parts[g.pairs ? 2 * s : s];
        const Part last = g.parts[g.pairs ? 2 * s + 1 : s];
        const size_t lo = first.off, hi = static_cast<size_t>(last.off) + last.n;
        for (size_t w = (lo >> 6) + threadIdx.x; w <= ((hi - 1) >> 6); w += kBlock) {
            const size_t b0 = w << 6;
            unsigned long long m = ~0ull;
            if (b0 < lo) m &= ~0ull << (lo - b0);
            if (b0 + 64 > hi) m &= ~0ull >> (b0 + 64 - hi);
            if (m == ~0ull)
                single[w] = m;
            else
                atomicOr(single + w, m);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_seg_count(SegArgs g, size_t N, const RoundCtl *ctl,
                                                       const uint32_t *blockA,
                                                       const uint32_t *blockB) {
    seg_count_body(g, N, ctl, blockA, blockB);
}

__global__ __launch_bounds__(kBlock) void k_seg_end(SegArgs g, const RoundCtl *ctl,
                                                     const uint32_t *blockA,
                                                     const uint32_t *blockB) {
    seg_end_body(g, ctl, blockA, blockB);
}

__global__ __launch_bounds__(kBlock) void k_seg_freeze(SegArgs g, const RoundCtl *ctl,
                                                        unsigned long long *single) {
    seg_freeze_body(g, ctl, single);
}

// Persistent loop: up to `rounds` rounds inside one cooperative launch, the
// phases of a round separated by grid barriers instead of kernel boundaries
// (the barrier's release and acquire make each phase's writes visible to
// every workgroup, on every XCD, before the next phase reads them).  Every
// workgroup takes the same barriers: the stop flag is read right after a
// barrier and written only by the round's last phase, between two barriers.
// The grid must fit on the device at once (the cooperative launch refuses
// more workgroups than can be resident together).
template <int KC>
__global__ __launch_bounds__(kBlock) void k_rounds_persistent(SigParams sp, InsParams ip,
                                                               SegArgs g, RoundCtl *ctl,
                                                               uint32_t rounds) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    for (uint32_t i = 0; i < rounds; ++i) {
        if (__hip_atomic_load(&ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        mark_body<KC>(sp);
        grid.sync();
        signature_body<KC>(sp);
        grid.sync();
        insert_lds_body(ip);
        insert_body(ip);
        grid.sync();
        if (g.nseg) {  // (uniform) the per-segment bookkeeping of the round
            seg_count_body(g, ip.N, ctl, ip.blockA, ip.blockB);
            grid.sync();
            seg_end_body(g, ctl, ip.blockA, ip.blockB);
            grid.sync();
            seg_freeze_body(g, ctl, sp.single);
            grid.sync();
        }
        if (blockIdx.x == 0)
            round_end_body(ctl, ip.blockA, ip.blockB, ip.counters, static_cast<uint32_t>(ip.N));
        grid.sync();
    }
}

__global__ __launch_bounds__(kBlock) void k_part_output(SegArgs g, size_t N,
                                                         const uint32_t *__restrict__ canon,
                                                         uint32_t *__restrict__ out) {
    for (size_t q = global_tid(); q < N; q += grid_stride()) {
        const Part P = g.parts[find_part(g, q)];
        out[P.out + (q - P.off)] = canon[q] - P.off;
    }
}

__global__ __launch_bounds__(kBlock) void k_pair_verdicts(SegArgs g,
                                                           const uint32_t *__restrict__ block,
                                                           int32_t *verdicts) {
    for (size_t s = global_tid(); s < g.nseg; s += grid_stride()) {
        const Part A = g.parts[2 * s], B = g.parts[2 * s + 1];
        verdicts[s] = block[A.off + A.start] == block[B.off + B.start] ? 1 : 0;
    }
}

// ---------------------------------------------------------------- pointer jumping

__global__ __launch_bounds__(kBlock) void k_jump(uint32_t *__restrict__ cols, size_t N,
                                                  uint32_t k, uint32_t level,
                                                  uint32_t *diff, uint32_t *nonid) {
    const uint32_t a = blockIdx.y;
    const uint32_t *__restrict__ prev = cols + (static_cast<size_t>(level - 1) * k + a) * N;
    uint32_t *__restrict__ cur = cols + (static_cast<size_t>(level) * k + a) * N;
    bool d = false, moves = false;
    for (size_t q = global_tid(); q < N; q += grid_stride()) {
        const uint32_t m = prev[q];
        const uint32_t t = prev[m];
        cur[q] = t;
        d |= t != m;
        moves |= t != q;
    }
    wave_set_flag(diff + static_cast<size_t>(level) * k + a, d);
    wave_set_flag(nonid + static_cast<size_t>(level) * k + a, moves);
}

// Flags of the closure columns over the states outside singleton blocks:
// nonid[c] when column c moves such a state, diff[c] when it differs from
// the previous level of its letter on such a state (level 0: unused).
// Singletons never split, so a column that is the identity, or repeats its
// previous level, on every other state only repeats a key component there.
__global__ __launch_bounds__(kBlock) void k_col_flags(const uint32_t *__restrict__ cols, size_t N,
                                                      uint32_t k,
                                                      const unsigned long long *__restrict__ single,
                                                      uint32_t *diff, uint32_t *nonid) {
    const uint32_t c = blockIdx.y;
    const uint32_t *__restrict__ col = cols + static_cast<size_t>(c) * N;
    const uint32_t *__restrict__ prev = c >= k ? cols + static_cast<size_t>(c - k) * N : col;
    bool d = false, moves = false;
    for (size_t q = global_tid(); q < N; q += grid_stride()) {
        if ((single[q >> 6] >> (q & 63)) & 1ull) continue;
        const uint32_t t = col[q];
        d |= t != prev[q];
        moves |= t != q;
    }
    wave_set_flag(diff + c, d);
    wave_set_flag(nonid + c, moves);
}

// ---------------------------------------------------------------- canonical ids

__global__ __launch_bounds__(kBlock) void k_zero(ZeroList z) {
    for (int r = 0; r < z.count; ++r) {
        unsigned long long *__restrict__ p = z.p[r];
        for (size_t i = global_tid(); i < z.words[r]; i += grid_stride()) p[i] = 0ull;
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, size_t n, uint32_t v) {
    for (size_t i = global_tid(); i < n; i += grid_stride()) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_canon_min(const uint32_t *__restrict__ ids, size_t N,
                                                       uint32_t *mins) {
    for (size_t q = global_tid(); q < N; q += grid_stride())
        atomicMin(mins + ids[q], static_cast<uint32_t>(q));
}

__global__ __launch_bounds__(kBlock) void k_canon_apply(const uint32_t *__restrict__ ids, size_t N,
                                                         const uint32_t *__restrict__ mins,
                                                         uint32_t *__restrict__ out) {
    for (size_t q = global_tid(); q < N; q += grid_stride()) out[q] = mins[ids[q]];
}

// ---------------------------------------------------------------- dense leader numbering

constexpr int kScanThreads = static_cast<int>(kScanTile);  // one element per thread

// Per-tile leader counts: ballot of "block[q] == q" and popcount per wave.
__global__ __launch_bounds__(kScanThreads) void k_leader_partials(const uint32_t *__restrict__ block,
                                                                   size_t N, uint32_t *partials) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    const size_t q = static_cast<size_t>(blockIdx.x) * kScanTile + threadIdx.x;
    const bool lead = q < N && block[q] == q;
    const unsigned long long m = __ballot(lead);
    if (lane_id() == 0) wsum[threadIdx.x / 64] = static_cast<uint32_t>(__popcll(m));
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) s += wsum[w];
        partials[blockIdx.x] = s;
    }
}

// Exclusive scan of the tile counts in one workgroup; partials[ntiles] and
// *total receive the sum.
__global__ __launch_bounds__(kScanThreads) void k_scan_partials(uint32_t *partials, uint32_t ntiles,
                                                                 uint32_t *total) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < ntiles; base += kScanThreads) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < ntiles ? partials[i] : 0u;
        // inclusive scan within the wave by shuffles
        uint32_t x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (static_cast<int>(lane_id()) >= d) x += y;
        }
        if (lane_id() == 63) wsum[threadIdx.x / 64] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t s = 0;
            for (int w = 0; w < kScanThreads / 64; ++w) {
                const uint32_t t = wsum[w];
                wsum[w] = s;
                s += t;
            }
        }
        __syncthreads();
        const uint32_t excl = carry + wsum[threadIdx.x / 64] + x - v;
        __syncthreads();
        if (i < ntiles) partials[i] = excl;
        if (threadIdx.x == kScanThreads - 1) carry = excl + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[ntiles] = carry;
        *total = carry;
    }
}

// dense[q] for leaders: tile offset + leaders before q in the tile (ballot
// rank within the wave + wave offsets).
__global__ __launch_bounds__(kScanThreads) void k_leader_rank(const uint32_t *__restrict__ block,
                                                               size_t N,
                                                               const uint32_t *__restrict__ partials,
                                                               uint32_t *__restrict__ dense,
                                                               uint32_t *__restrict__ leader_of) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    const size_t q = static_cast<size_t>(blockIdx.x) * kScanTile + threadIdx.x;
    const bool lead = q < N && block[q] == q;
    const unsigned long long m = __ballot(lead);
    const uint32_t lane = lane_id();
    if (lane == 0) wsum[threadIdx.x / 64] = static_cast<uint32_t>(__popcll(m));
    __syncthreads();
    uint32_t woff = 0;
    for (uint32_t w = 0; w < threadIdx.x / 64; ++w) woff += wsum[w];
    if (lead) {
        const unsigned long long below = lane ? (m & ((1ull << lane) - 1ull)) : 0ull;
        const uint32_t d = partials[blockIdx.x] + woff + static_cast<uint32_t>(__popcll(below));
        dense[q] = d;
        leader_of[d] = static_cast<uint32_t>(q);
    }
}

// dq[q] = dense id of q's block.
__global__ __launch_bounds__(kBlock) void k_dense_of_state(const uint32_t *__restrict__ block,
                                                            const uint32_t *__restrict__ dense,
                                                            size_t N, uint32_t *__restrict__ dq) {
    for (size_t q = global_tid(); q < N; q += grid_stride()) dq[q] = dense[block[q]];
}

// One thread per quotient transition (b, a): qdelta[b*k + a] = dq[delta(l, a)]
// with l the leader of block b; qacc[b] = accepting[l] as 0/1.
__global__ __launch_bounds__(kBlock) void k_quotient(const uint32_t *__restrict__ delta,
                                                      const uint8_t *__restrict__ acc, uint32_t k,
                                                      const uint32_t *__restrict__ dq,
                                                      const uint32_t *__restrict__ leader_of,
                                                      const uint32_t *num_blocks, uint32_t start,
                                                      uint32_t *__restrict__ qdelta,
                                                      uint8_t *__restrict__ qacc, uint32_t *qstart) {
    const size_t total = static_cast<size_t>(*num_blocks) * k;
    if (global_tid() == 0) *qstart = dq[start];
    for (size_t i = global_tid(); i < total; i += grid_stride()) {
        const size_t b = i / k;
        const uint32_t a = static_cast<uint32_t>(i - b * k);
        const size_t l = leader_of[b];
        qdelta[i] = dq[delta[l * k + a]];
        if (a == 0) qacc[b] = acc[l] ? 1 : 0;
    }
}

// Discrete partition (every block a single state): the quotient is the input.
__global__ __launch_bounds__(kBlock) void k_quotient_identity(const uint32_t *__restrict__ delta,
                                                               const uint8_t *__restrict__ acc,
                                                               size_t n, uint32_t k,
                                                               uint32_t start,
                                                               uint32_t *__restrict__ qdelta,
                                                               uint8_t *__restrict__ qacc,
                                                               uint32_t *qstart) {
    if (global_tid() == 0) *qstart = start;
    const size_t total = n * k;
    for (size_t i = global_tid(); i < total; i += grid_stride()) qdelta[i] = delta[i];
    for (size_t q = global_tid(); q < n; q += grid_stride()) qacc[q] = acc[q] ? 1 : 0;
}

unsigned grid_for(size_t work, unsigned cap = 1u << 20) {
    size_t g = (work + kBlock - 1) / kBlock;
    if (g == 0) g = 1;
    if (g > cap) g = cap;
    return static_cast<unsigned>(g);
}

}  // namespace

// ---------------------------------------------------------------- launchers

namespace {
constexpr unsigned kDefaultGridCap = 8192;

SigParams sig_params(const RoundArgs &a) {
    return SigParams{a.cols,     a.colmap,     a.N,        a.k_eff,    a.blockA,
                     a.blockB,   a.sig,        a.hash,     a.table,    a.table_cap,
                     a.multi,    a.active,     a.accbits,  a.presence, a.presence_packed,
                     a.lab8,     a.counters,   a.ctl,      a.cached_probe, a.chg,
                     a.single,   a.touched,    a.chg_sum,  a.grouping, a.hash_bits,
                     a.seg.nseg ? a.seg.parts : nullptr,      a.seg.nseg ? a.seg.tile_part : nullptr,
                     a.seg.nseg ? a.seg.nparts : 0u, a.pb,
                     a.seg.nseg ? a.seg.tile_dead : nullptr,
                     a.seg.nseg ? a.seg.tile_lead : nullptr};
}

// Workgroups of a round kernel whose workgroups take `tile` states at a
// time, at most cap (0: no cap).
unsigned round_grid(const RoundArgs &a, unsigned cap, size_t tile = kBlock) {
    size_t g = (a.N + tile - 1) / tile;
    if (g == 0) g = 1;
    const size_t c = cap ? cap : (1u << 30);
    return static_cast<unsigned>(g > c ? c : g);
}

InsParams ins_params(const RoundArgs &a) {
    return InsParams{a.sig,    a.hash,   a.N,     a.k_eff + 1, a.table,    a.table_cap - 1,
                     a.blockA, a.blockB, a.multi, a.active,    a.counters, a.ctl,
                     a.cached_probe, a.lds_stage, a.chg, a.chg_sum,
                     a.seg.nseg ? a.seg.tile_dead : nullptr};
}

// Workgroups of the persistent loop: no more than fit on the device at once.
hipError_t coresident_grid(const void *kernel, unsigned &grid) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0);
    if (e != hipSuccess) return e;
    if (cus <= 0 || per_cu <= 0) return hipErrorInvalidConfiguration;
    // at most one workgroup per CU: a grid barrier's cost grows with the
    // workgroups that arrive at it
    grid = static_cast<unsigned>(cus) * std::min(static_cast<unsigned>(per_cu), kPersistentGroupsPerCu);
    return hipSuccess;
}

}  // namespace

void launch_ingest(const uint32_t *delta, uint32_t n, uint32_t k, uint32_t *cols, size_t N,
                   uint32_t offset, uint32_t target_offset, uint32_t *err, uint32_t *nonid,
                   hipStream_t s) {
    launch_kernel(k_ingest, dim3(grid_for(n)), dim3(kBlock), 0, s, delta, n, k, cols, N,
                       offset, target_offset, err, nonid);
}

void launch_init_blocks(const uint8_t *acc, uint32_t n, uint32_t offset, uint32_t *block,
                        unsigned long long *accbits, uint32_t *class_flags, hipStream_t s) {
    launch_kernel(k_init_blocks, dim3(grid_for(n, kDefaultGridCap)), dim3(kBlock), 0, s, acc,
                       n, offset, block, accbits, class_flags);
}

void launch_ctl_reset(RoundCtl *ctl, const uint32_t *class_flags, uint32_t max_rounds,
                      uint32_t check_eq, uint32_t eq_a, uint32_t eq_b, uint32_t pattern_first,
                      uint32_t packed_second, const uint32_t *init_count, hipStream_t s) {
    launch_kernel(k_ctl_reset, dim3(1), dim3(64), 0, s, ctl, class_flags, max_rounds,
                       check_eq, eq_a, eq_b, pattern_first, packed_second, init_count);
}

void launch_ingest_parts(const SegArgs &g, size_t N, uint32_t k, uint32_t *cols, uint32_t *err,
                         uint32_t *nonid, hipStream_t s) {
    launch_kernel(k_ingest_parts, dim3(grid_for(N, kDefaultGridCap)), dim3(kBlock), 0, s, g,
                       N, k, cols, err, nonid);
}

void launch_init_parts(const SegArgs &g, size_t N, uint32_t *block, unsigned long long *accbits,
                       hipStream_t s) {
    launch_kernel(k_init_parts, dim3(grid_for(N, kDefaultGridCap)), dim3(kBlock), 0, s, g, N,
                  block, accbits);
    launch_kernel(k_seg_init, dim3(grid_for(g.nseg, kDefaultGridCap)), dim3(kBlock), 0, s, g);
}

void launch_seg_pattern(const RoundArgs &a, hipStream_t s) {
    if (!a.segpat_bits) return;
    const SigParams sp = sig_params(a);
    const size_t words = static_cast<size_t>(a.seg.nseg) << a.segpat_bits;
    launch_kernel(k_fill_u32, dim3(grid_for(words, kDefaultGridCap)), dim3(kBlock), 0, s,
                  a.segpat_table, words, ~0u);
    launch_kernel(k_segpat_min, dim3(grid_for((a.N + kSegPatTile - 1) / kSegPatTile * kBlock,
                                              kDefaultGridCap)),
                  dim3(kBlock), 0, s, sp, a.seg, a.segpat_table, a.segpat, a.segpat_bits);
    launch_kernel(k_segpat_assign, dim3(grid_for(a.N, kDefaultGridCap)), dim3(kBlock), 0, s, sp,
                  a.seg, static_cast<const uint32_t *>(a.segpat_table),
                  static_cast<const uint16_t *>(a.segpat), a.segpat_bits, a.multi);
}

void launch_seg_round(const RoundArgs &a, hipStream_t s) {
    launch_kernel(k_seg_count, dim3(grid_for(a.N, kDefaultGridCap)), dim3(kBlock), 0, s,
                       a.seg, a.N, a.ctl, a.blockA, a.blockB);
    launch_kernel(k_seg_end, dim3(grid_for(a.seg.nseg, kDefaultGridCap)), dim3(kBlock), 0, s,
                       a.seg, a.ctl, a.blockA, a.blockB);
    launch_kernel(k_seg_freeze, dim3(std::min<uint32_t>(a.seg.nseg, kDefaultGridCap)),
                  dim3(kBlock), 0, s, a.seg, a.ctl, a.single);
}

void launch_part_output(const SegArgs &g, size_t N, const uint32_t *canon, uint32_t *out,
                        hipStream_t s) {
    launch_kernel(k_part_output, dim3(grid_for(N, kDefaultGridCap)), dim3(kBlock), 0, s, g, N,
                       canon, out);
}

void launch_pair_verdicts(const SegArgs &g, const uint32_t *block, int32_t *verdicts,
                          hipStream_t s) {
    launch_kernel(k_pair_verdicts, dim3(grid_for(g.nseg, kDefaultGridCap)), dim3(kBlock), 0,
                       s, g, block, verdicts);
}

void launch_ctl_resume(RoundCtl *ctl, hipStream_t s) {
    launch_kernel(k_ctl_resume, dim3(1), dim3(64), 0, s, ctl);
}

void launch_round_end(const RoundArgs &a, hipStream_t s) {
    launch_kernel(k_round_end, dim3(1), dim3(kBlock), 0, s, a.ctl, a.blockA, a.blockB,
                       a.counters, static_cast<uint32_t>(a.N));
}

void launch_pattern_kernel(const RoundArgs &a, hipStream_t s) {
    const SigParams sp = sig_params(a);
    const dim3 grid(round_grid(a, a.pattern_grid_cap)), block(kBlock);
    switch (a.k_eff) {
        case 1: launch_kernel(k_pattern_round<1>, grid, block, 0, s, sp); break;
        case 2: launch_kernel(k_pattern_round<2>, grid, block, 0, s, sp); break;
        case 3: launch_kernel(k_pattern_round<3>, grid, block, 0, s, sp); break;
        case 4: launch_kernel(k_pattern_round<4>, grid, block, 0, s, sp); break;
        case 8: launch_kernel(k_pattern_round<8>, grid, block, 0, s, sp); break;
        default: launch_kernel(k_pattern_round<0>, grid, block, 0, s, sp); break;
    }
}

void launch_packed_kernel(const RoundArgs &a, hipStream_t s) {
    const SigParams sp = sig_params(a);
    const dim3 grid(round_grid(a, a.pattern_grid_cap)), block(kBlock);
    switch (a.k_eff) {
        case 1: launch_kernel(k_packed_round<1>, grid, block, 0, s, sp); break;
        case 2: launch_kernel(k_packed_round<2>, grid, block, 0, s, sp); break;
        case 3: launch_kernel(k_packed_round<3>, grid, block, 0, s, sp); break;
        case 4: launch_kernel(k_packed_round<4>, grid, block, 0, s, sp); break;
        default: launch_kernel(k_packed_round<0>, grid, block, 0, s, sp); break;
    }
    launch_kernel(k_count_labels, dim3(1024), block, 0, s, sp);
}

void launch_pattern_round(const RoundArgs &a, hipStream_t s) {
    launch_pattern_kernel(a, s);
    launch_round_end(a, s);
}

void launch_packed_round(const RoundArgs &a, hipStream_t s) {
    launch_packed_kernel(a, s);
    launch_round_end(a, s);
}

void launch_signature(const RoundArgs &a, hipStream_t s) {
    const SigParams sp = sig_params(a);
    const dim3 grid(round_grid(a, a.round_grid_cap)), block(kBlock);
    switch (a.k_eff) {
        case 1: launch_kernel(k_signature<1>, grid, block, 0, s, sp); break;
        case 2: launch_kernel(k_signature<2>, grid, block, 0, s, sp); break;
        case 3: launch_kernel(k_signature<3>, grid, block, 0, s, sp); break;
        case 4: launch_kernel(k_signature<4>, grid, block, 0, s, sp); break;
        case 5: launch_kernel(k_signature<5>, grid, block, 0, s, sp); break;
        case 6: launch_kernel(k_signature<6>, grid, block, 0, s, sp); break;
        case 7: launch_kernel(k_signature<7>, grid, block, 0, s, sp); break;
        case 8: launch_kernel(k_signature<8>, grid, block, 0, s, sp); break;
        case 16: launch_kernel(k_signature<16>, grid, block, 0, s, sp); break;
        default: launch_kernel(k_signature<0>, grid, block, 0, s, sp); break;
    }
}

// ---- gathers through LDS slices

uint64_t pb_chunk_words(uint32_t nb, uint32_t ntiles) {
    return static_cast<uint64_t>((ntiles + kPbChunk - 1) / kPbChunk) * nb;
}

namespace {

template <int KC>
void pb_build_k(const uint32_t *cols, const uint32_t *colmap, size_t N, const PbArgs &pb,
                uint32_t *csum, uint32_t *btot, hipStream_t s) {
    const dim3 tiles(std::min<uint32_t>(pb.ntiles, 8192u)), block(kBlock);
    const uint32_t nchunks = (pb.ntiles + kPbChunk - 1) / kPbChunk;
    launch_kernel(k_pb_count<KC>, tiles, block, 0, s, cols, colmap, N, pb.nb, pb.ntiles, pb.cnt);
    launch_kernel(k_pb_colsum, dim3(nchunks), block, 0, s, pb.cnt, pb.nb, pb.ntiles, csum);
    launch_kernel(k_pb_colscan, dim3((pb.nb + kBlock / 64 - 1) / (kBlock / 64)), block, 0, s,
                  csum, pb.nb, nchunks, btot);
    launch_kernel(k_pb_bscan, dim3(1), dim3(1024), 0, s, btot, pb.nb, pb.bstart);
    launch_kernel(k_pb_apply, dim3(nchunks), block, 0, s, pb.cnt, csum, pb.bstart, pb.nb,
                  pb.ntiles, pb.off);
    launch_kernel(k_pb_scatter<KC>, tiles, dim3(kPbScatterThreads), 0, s, cols, colmap, N, pb);
}

}  // namespace

void launch_pb_build(const uint32_t *cols, const uint32_t *colmap, size_t N, uint32_t k_eff,
                     const PbArgs &pb, uint32_t *csum, uint32_t *btot, hipStream_t s) {
    switch (k_eff) {
        case 1: pb_build_k<1>(cols, colmap, N, pb, csum, btot, s); break;
        case 2: pb_build_k<2>(cols, colmap, N, pb, csum, btot, s); break;
        case 3: pb_build_k<3>(cols, colmap, N, pb, csum, btot, s); break;
        case 4: pb_build_k<4>(cols, colmap, N, pb, csum, btot, s); break;
        case 5: pb_build_k<5>(cols, colmap, N, pb, csum, btot, s); break;
        case 6: pb_build_k<6>(cols, colmap, N, pb, csum, btot, s); break;
        case 7: pb_build_k<7>(cols, colmap, N, pb, csum, btot, s); break;
        case 8: pb_build_k<8>(cols, colmap, N, pb, csum, btot, s); break;
        case 16: pb_build_k<16>(cols, colmap, N, pb, csum, btot, s); break;
        default: break;  // the host only buckets these widths
    }
}

void launch_pb_gather(const RoundArgs &a, hipStream_t s) {
    if (!a.pb.nb) return;
    const SigParams sp = sig_params(a);
    // one workgroup per bucket (measured on MI355X with 2^23 states: one
    // 64 KB slice per workgroup gathered 364 G ids/s; two or four workgroups
    // per bucket, each loading the slice, 305 and 229; 128 KB slices 199),
    // of 1,024 threads: two per CU then hold 32 waves instead of 8 (a 2^23-
    // state union's dense round 87 -> 44 us)
    const uint32_t per_bucket = 1u;
    launch_kernel(k_pb_gather, dim3(a.pb.nb * per_bucket), dim3(kPbGatherThreads),
                  (1u << kPbSliceLog) * 4u, s, sp, per_bucket);
}

void launch_packed_pb(const RoundArgs &a, hipStream_t s) {
    if (!a.pb.nb) return;
    const SigParams sp = sig_params(a);
    launch_kernel(k_pb_gather8, dim3(a.pb.nb), dim3(kPbGatherThreads), 0, s, sp);
    // one workgroup per tile (the kernel also takes fewer, each then keeping
    // its label set over several tiles)
    constexpr uint32_t NT = kPbPackedThreads;
    const dim3 grid(a.pb.ntiles), block(NT);
    switch (a.k_eff) {
        case 1: launch_kernel(k_packed_pb<1, NT>, grid, block, 0, s, sp); break;
        case 2: launch_kernel(k_packed_pb<2, NT>, grid, block, 0, s, sp); break;
        case 3: launch_kernel(k_packed_pb<3, NT>, grid, block, 0, s, sp); break;
        case 4: launch_kernel(k_packed_pb<4, NT>, grid, block, 0, s, sp); break;
        default: break;  // packed labels only for k_eff <= 4
    }
    launch_kernel(k_count_labels, dim3(1024), dim3(kBlock), 0, s, sp);
}

void launch_signature_pb(const RoundArgs &a, hipStream_t s) {
    if (!a.pb.nb) return;
    const SigParams sp = sig_params(a);
    constexpr uint32_t NT = kPbSigThreads;
    const dim3 grid(a.pb.ntiles), block(NT);
    switch (a.k_eff) {
        case 1: launch_kernel(k_signature_pb<1, NT>, grid, block, 0, s, sp); break;
        case 2: launch_kernel(k_signature_pb<2, NT>, grid, block, 0, s, sp); break;
        case 3: launch_kernel(k_signature_pb<3, NT>, grid, block, 0, s, sp); break;
        case 4: launch_kernel(k_signature_pb<4, NT>, grid, block, 0, s, sp); break;
        case 5: launch_kernel(k_signature_pb<5, NT>, grid, block, 0, s, sp); break;
        case 6: launch_kernel(k_signature_pb<6, NT>, grid, block, 0, s, sp); break;
        case 7: launch_kernel(k_signature_pb<7, NT>, grid, block, 0, s, sp); break;
        case 8: launch_kernel(k_signature_pb<8, NT>, grid, block, 0, s, sp); break;
        case 16: launch_kernel(k_signature_pb<16, NT>, grid, block, 0, s, sp); break;
        default: break;
    }
}

void launch_insert(const RoundArgs &a, hipStream_t s) {
    const dim3 grid(round_grid(a, a.round_grid_cap)), block(kBlock);
    const InsParams ip = ins_params(a);
    // the LDS-staged variants (lds_stage 1, and 2, which stages every round)
    // or the direct one (0)
    if (a.lds_stage != 0) {
        // two states per thread for the specialised signature widths
        const dim3 grid2(round_grid(a, a.round_grid_cap, 2 * kBlock));
        switch (a.insert_pair ? a.k_eff : 0u) {
            case 1: launch_kernel(k_insert_lds2<1>, grid2, block, 0, s, ip); break;
            case 2: launch_kernel(k_insert_lds2<2>, grid2, block, 0, s, ip); break;
            case 3: launch_kernel(k_insert_lds2<3>, grid2, block, 0, s, ip); break;
            case 4: launch_kernel(k_insert_lds2<4>, grid2, block, 0, s, ip); break;
            case 8: launch_kernel(k_insert_lds2<8>, grid2, block, 0, s, ip); break;
            default: launch_kernel(k_insert_lds, grid, block, 0, s, ip); break;
        }
    } else {
        launch_kernel(k_insert, grid, block, 0, s, ip);
    }
}

void launch_mark(const RoundArgs &a, hipStream_t s) {
    const SigParams sp = sig_params(a);
    // every workgroup loads the changed-id summary into LDS, so the grid is
    // capped; without the summary (too large for LDS) the cap is the round
    // kernels'
    const bool summary = summary_words(a.N) <= kSumLdsWords;
    const unsigned cap = !summary ? a.round_grid_cap
                         : a.round_grid_cap ? std::min(a.round_grid_cap, kMarkGridCap)
                                            : kMarkGridCap;
    const dim3 grid(round_grid(a, cap)), block(kBlock);
    switch (a.k_eff) {
        case 1: launch_kernel(k_mark<1>, grid, block, 0, s, sp); break;
        case 2: launch_kernel(k_mark<2>, grid, block, 0, s, sp); break;
        case 3: launch_kernel(k_mark<3>, grid, block, 0, s, sp); break;
        case 4: launch_kernel(k_mark<4>, grid, block, 0, s, sp); break;
        case 8: launch_kernel(k_mark<8>, grid, block, 0, s, sp); break;
        case 16: launch_kernel(k_mark<16>, grid, block, 0, s, sp); break;
        default: launch_kernel(k_mark<0>, grid, block, 0, s, sp); break;
    }
}

void launch_ctl_full(RoundCtl *ctl, hipStream_t s) {
    launch_kernel(k_ctl_full, dim3(1), dim3(64), 0, s, ctl);
}

void launch_round(const RoundArgs &a, hipStream_t s) {
    launch_mark(a, s);
    launch_pb_gather(a, s);
    launch_signature_pb(a, s);
    launch_signature(a, s);
    if (a.grouping)
        launch_sort_group(a, s);
    else
        launch_insert(a, s);
    if (a.seg.nseg) launch_seg_round(a, s);
    launch_round_end(a, s);
}

hipError_t launch_rounds_persistent(const RoundArgs &a, uint32_t rounds, hipStream_t s) {
    if (a.grouping) return hipErrorInvalidValue;
    const void *kernel;
    switch (a.k_eff) {
        case 1: kernel = reinterpret_cast<const void *>(&k_rounds_persistent<1>); break;
        case 2: kernel = reinterpret_cast<const void *>(&k_rounds_persistent<2>); break;
        case 3: kernel = reinterpret_cast<const void *>(&k_rounds_persistent<3>); break;
        case 4: kernel = reinterpret_cast<const void *>(&k_rounds_persistent<4>); break;
        case 8: kernel = reinterpret_cast<const void *>(&k_rounds_persistent<8>); break;
        default: kernel = reinterpret_cast<const void *>(&k_rounds_persistent<0>); break;
    }
    unsigned fit = 0;
    hipError_t e = coresident_grid(kernel, fit);
    if (e != hipSuccess) return e;
    const unsigned grid = std::min(round_grid(a, a.round_grid_cap), fit);
    SigParams sp = sig_params(a);
    InsParams ip = ins_params(a);
    SegArgs g = a.seg;
    RoundCtl *ctl = a.ctl;
    void *args[] = {&sp, &ip, &g, &ctl, &rounds};
    return hipLaunchCooperativeKernel(kernel, dim3(grid), dim3(kBlock), args, 0, s);
}

void launch_column_flags(const uint32_t *cols, size_t N, uint32_t k, uint32_t ncols,
                         const unsigned long long *single, uint32_t *diff, uint32_t *nonid,
                         hipStream_t s) {
    dim3 grid(grid_for(N, kDefaultGridCap / 4), ncols);
    launch_kernel(k_col_flags, grid, dim3(kBlock), 0, s, cols, N, k, single, diff, nonid);
}

void launch_jump(uint32_t *cols, size_t N, uint32_t k, uint32_t level, uint32_t *diff,
                 uint32_t *nonid, hipStream_t s) {
    dim3 grid(grid_for(N, kDefaultGridCap), k);
    launch_kernel(k_jump, grid, dim3(kBlock), 0, s, cols, N, k, level, diff, nonid);
}

void launch_zero(const ZeroList &z, hipStream_t s) {
    size_t most = 0;
    for (int r = 0; r < z.count; ++r) most = std::max(most, z.words[r]);
    if (most == 0) return;
    launch_kernel(k_zero, dim3(grid_for(most, kDefaultGridCap)), dim3(kBlock), 0, s, z);
}

void launch_canonicalise(const uint32_t *ids, size_t N, size_t id_range, uint32_t *scratch_min,
                         uint32_t *out, hipStream_t s) {
    const dim3 grid(grid_for(N)), block(kBlock);
    launch_kernel(k_fill_u32, dim3(grid_for(id_range, kDefaultGridCap)), block, 0, s,
                       scratch_min, id_range, ~0u);
    launch_kernel(k_canon_min, grid, block, 0, s, ids, N, scratch_min);
    launch_kernel(k_canon_apply, grid, block, 0, s, ids, N, scratch_min, out);
}

void launch_dense_leaders(const uint32_t *block, size_t N, uint32_t *partials, uint32_t *dense,
                          uint32_t *leader_of, uint32_t *num_blocks, hipStream_t s) {
    const uint32_t ntiles = static_cast<uint32_t>((N + kScanTile - 1) / kScanTile);
    launch_kernel(k_leader_partials, dim3(ntiles), dim3(kScanThreads), 0, s, block, N,
                       partials);
    launch_kernel(k_scan_partials, dim3(1), dim3(kScanThreads), 0, s, partials, ntiles,
                       num_blocks);
    launch_kernel(k_leader_rank, dim3(ntiles), dim3(kScanThreads), 0, s, block, N, partials,
                       dense, leader_of);
}

void launch_quotient(const uint32_t *delta, const uint8_t *acc, uint32_t k,
                     const uint32_t *block, const uint32_t *dense, const uint32_t *leader_of,
                     const uint32_t *num_blocks, uint32_t n, uint32_t start, uint32_t *dq,
                     uint32_t *qdelta, uint8_t *qacc, uint32_t *qstart, hipStream_t s) {
    launch_kernel(k_dense_of_state, dim3(grid_for(n, kDefaultGridCap)), dim3(kBlock), 0, s,
                       block, dense, static_cast<size_t>(n), dq);
    launch_kernel(k_quotient, dim3(grid_for(static_cast<size_t>(n) * k, kDefaultGridCap)),
                       dim3(kBlock), 0, s, delta, acc, k, dq, leader_of, num_blocks, start, qdelta,
                       qacc, qstart);
}

void launch_quotient_identity(const uint32_t *delta, const uint8_t *acc, uint32_t n, uint32_t k,
                              uint32_t start, uint32_t *qdelta, uint8_t *qacc, uint32_t *qstart,
                              hipStream_t s) {
    launch_kernel(k_quotient_identity,
                       dim3(grid_for(static_cast<size_t>(n) * k, kDefaultGridCap)), dim3(kBlock),
                       0, s, delta, acc, static_cast<size_t>(n), k, start, qdelta, qacc, qstart);
}

}  // namespace dfamin
