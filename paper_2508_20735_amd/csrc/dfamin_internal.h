// Internal declarations of libdfamin (not part of the public ABI).
//
// Device data layout (one refinement over N states, N = n or nA + nB):
//   cols     uint32 [ncols][N]   symbol-major transition columns; column c,
//                                state q -> cols[c*N + q].  Plain refinement
//                                uses the k input letters; the closure adds
//                                the letters a^(2^i) at column i*k + a.
//   colmap   uint32 [k_eff]      the columns that enter the signature
//   blockA/B uint32 [N]          block ids, double-buffered by round parity
//   sig      uint32 [N][k_eff+1] the signature of every state (row-major)
//   hash     uint64 [N]          64-bit hash of each signature
//   table    uint64 [cap]        lock-free open-addressing table
//                                (epoch:8 | tag:24 | representative:32)
//   multi    uint32 [N]          multi[b] = r + 1 when block b had two or more
//                                members after round r (singleton blocks
//                                never split again and are skipped)
//   active   uint64 [N/64]       per-wave bitmask of the states refined in
//                                the current round
//   accbits  uint64 [N/64]       acceptance, one bit per state (first round)
//   chg      uint64 [N/64]       state's block id changed in the last round
//   single   uint64 [N/64]       state's block is known to be a singleton
//   touched  uint64 [2][N/64]    per block id (bit b): the block has a member
//                                with a successor whose id changed; one
//                                bitmap per round parity
//   ctl      RoundCtl            round counter / stop flag on the device
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "launch.h"

namespace dfamin {

constexpr int kBlock = 256;        // threads per workgroup
constexpr uint32_t kEpochs = 255;  // table epochs before it is cleared
constexpr int kSpread = 64;        // per-round counters, one per 128-byte line
constexpr int kSpreadStride = 32;  // uint32 words between two counters
constexpr uint32_t kPatternMaxBits = 17;  // first round by bit patterns if k_eff + 1 <= 17
constexpr uint32_t kPackedMaxBits = 25;   // round 1 by packed labels if (k_eff + 1)^2 <= 25
// the packed round's label map: one byte per possible label
constexpr size_t kLabelMapBytes = size_t(1) << kPackedMaxBits;
// Changed-id summary: one bit per group of 2^kSumShift consecutive states,
// set when a state of the group changed its id in the round; 64 groups per
// word.  Incremental marking holds up to kSumLdsWords words in LDS.
constexpr uint32_t kSumShift = 5;
constexpr uint32_t kSumWordShift = kSumShift + 6;
constexpr uint32_t kSumLdsWords = 4096;  // 32 KB: N <= 2^23 with 32-state groups
// workgroups of the marking kernel: each loads the summary into LDS, so fewer
// and longer-lived workgroups load less
constexpr uint32_t kMarkGridCap = 1024;
__host__ __device__ inline size_t summary_words(size_t N) {
    return (N + (size_t(1) << kSumWordShift) - 1) >> kSumWordShift;
}
constexpr uint32_t kPersistentGroupsPerCu = 1;  // workgroups per CU in the persistent loops
constexpr uint32_t kActiveHist = 64;      // rounds of refined-state counts kept in RoundCtl

// Round-loop state kept on the device so that rounds can be enqueued (or
// replayed from a graph) without the host in the loop.
struct RoundCtl {
    uint32_t round;       // rounds completed
    uint32_t done;        // stop flag: stable, decided or limit reached
    uint32_t prev_count;  // blocks before the current round
    uint32_t last_gain;   // blocks added by the last round
    uint32_t changing;    // rounds that added blocks
    uint32_t stable;      // 1 once a round added no block
    uint32_t separated;   // equivalence: the two start states were split
    uint32_t limit;       // max_rounds reached
    uint32_t max_rounds;  // 0 = unbounded
    uint32_t eq_a, eq_b;  // equivalence: states whose blocks are compared
    uint32_t check_eq;    // 1 = stop as soon as eq_a and eq_b separate
    uint32_t pattern_first;  // round 0 grouped by acceptance bit patterns
    uint32_t packed_second;  // round 1 grouped by packed round-0 labels
    uint32_t all_active_until;  // rounds <= this refine every state
    uint32_t full_until;     // rounds <= this refine every state of a multi-state block
    uint32_t last_changed;   // states whose block id changed in the last round
    uint32_t last_active;    // states refined by the last round
    unsigned long long active_sum;  // states refined, summed over rounds
    uint32_t active_hist[kActiveHist];  // states refined by round r, at r % kActiveHist
    uint32_t gain_hist[kActiveHist];    // blocks added by round r, at r % kActiveHist
    uint32_t last_claims;               // blocks formed among the refined states
    unsigned long long pb_rounds;       // bit r % 64: round r gathered through LDS slices
};

// ---- launchers (defined in refine_kernels.hip); all enqueue on `s` ----

// Transpose row-major delta (n x k, targets < n) into cols[a*N + offset + q]
// adding `target_offset` to every target; sets *err = 1 on a target >= n and
// nonid[a] = 1 when letter a is not the identity on these states.
void launch_ingest(const uint32_t *delta, uint32_t n, uint32_t k, uint32_t *cols, size_t N,
                   uint32_t offset, uint32_t target_offset, uint32_t *err, uint32_t *nonid,
                   hipStream_t s);

// block[q] = accepting[q] ? 1 : 0 for q in [offset, offset + n), the
// acceptance bits (accbits, zeroed beforehand), and class_flags[0] / [1] = 1
// if some state accepts / rejects.
void launch_init_blocks(const uint8_t *acc, uint32_t n, uint32_t offset, uint32_t *block,
                        unsigned long long *accbits, uint32_t *class_flags, hipStream_t s);

// ctl := fresh state with prev_count = initial class count (read from
// class_flags on the device).
// With init_count != nullptr the initial block count is read from it
// instead of the two class flags.
void launch_ctl_reset(RoundCtl *ctl, const uint32_t *class_flags, uint32_t max_rounds,
                      uint32_t check_eq, uint32_t eq_a, uint32_t eq_b, uint32_t pattern_first,
                      uint32_t packed_second, const uint32_t *init_count, hipStream_t s);
// Clears the stop flag so that one more round can run (relabelling).
void launch_ctl_resume(RoundCtl *ctl, hipStream_t s);

// ---- segmented refinement (many DFAs in one refinement) ----
//
// The DFAs ("parts") are laid out back to back over the N states; a
// "segment" is a set of consecutive parts refined as one automaton (one DFA
// for batched minimisation, the two operands for batched equivalence).
// Initial labels are 2 * segment + accepting, so no block ever spans two
// segments; parts with fewer letters than the refinement are padded with
// identity letters, which do not change the partition.
struct Part {
    const uint32_t *delta;    // device, row-major n x k
    const uint8_t *accepting; // device, n
    uint32_t n, k;            // states, letters of this part
    uint32_t off;             // first state of the part in the union
    uint32_t seg;             // segment of the part
    uint32_t start;           // start state (local index)
    uint32_t pad;
    uint64_t out;             // output offset of the part's block ids
};

struct SegArgs {
    const Part *parts;        // nparts entries, ordered by off
    const uint32_t *tile_part;  // first part of every tile of kBlock states
    uint32_t nparts, nseg;
    uint32_t *seg_cnt;        // blocks per segment in the current round
    uint32_t *seg_prev;       // blocks per segment after the last round
    uint32_t *seg_changing;   // rounds that split a block of the segment
    uint32_t *seg_flags;      // acceptance classes per segment (bit 0/1)
    uint32_t *seg_done;       // r + 1 once the segment is decided in round r (0 before):
                              // its partition is stable, or (pairs) its two start states
                              // were separated; its states are skipped from then on
    uint32_t *init_count;     // sum over segments of their class counts
    uint32_t pairs;           // 1: segment s is the union of parts 2s and 2s + 1
    uint8_t *tile_dead;       // per tile of kBlock states: 1 once all its segments are decided
    uint16_t *tile_lead;      // per tile: states holding their block's id, written when the
                              // tile is found decided (its ids never change again)
};

// Transposes every part into cols (targets offset by the part's first
// state; letters >= part.k become the identity); err / nonid as launch_ingest.
void launch_ingest_parts(const SegArgs &g, size_t N, uint32_t k, uint32_t *cols, uint32_t *err,
                         uint32_t *nonid, hipStream_t s);
// Initial labels 2 * seg + accepting, acceptance bits (accbits, N/64 words),
// per-segment classes, their total.
void launch_init_parts(const SegArgs &g, size_t N, uint32_t *block, unsigned long long *accbits,
                       hipStream_t s);
// Writes every part's canonical block ids (local: global id - part offset)
// to out + part.out.
void launch_part_output(const SegArgs &g, size_t N, const uint32_t *canon, uint32_t *out,
                        hipStream_t s);
// verdict[s] = 1 iff the start states of parts 2s and 2s+1 share a block.
void launch_pair_verdicts(const SegArgs &g, const uint32_t *block, int32_t *verdicts,
                          hipStream_t s);

// Buffers of the sort-based grouping (sort_kernels.hip); N = states.
struct SortBuffers {
    unsigned long long *keys[2];  // N hashes, ping-pong
    uint32_t *vals[2];            // N states, ping-pong
    uint32_t *hist;               // 256 * sort_tiles digit counts
    uint32_t *partials;           // scan partials (partial_words)
    uint32_t *runhead;            // N: run head position of each sorted element
    uint32_t *m;                  // refined states this round (device)
};
// Successor-id gathers by target slices (a full round's gathers, served
// from LDS).  Edges (state q, letter a) are bucketed once per refinement by
// the slice of their target (kPbSliceLog bits: a slice's block ids fill a
// workgroup's LDS); inside bucket b they sit by source tile (kPbTile states),
// run (b, t) from off[t * nb + b], cnt[t * nb + b] edges long.
constexpr uint32_t kPbSliceLog = 14;   // 16,384 states: 64 KB of ids in LDS (two workgroups per CU)
constexpr uint32_t kPbTile = 2048;     // states of a source tile
constexpr uint32_t kPbMaxBuckets = 1024;  // N <= 2^24
constexpr uint32_t kPbChunk = 16;      // tiles per step of the run-start scan
struct PbArgs {
    uint16_t *tl;    // E: target within its slice
    uint16_t *src;   // E: (source state - tile start) * k_eff + letter
    uint32_t *val;   // E: the gathered block ids of the round
    uint32_t *cnt;     // ntiles * nb run lengths, tile-major
    uint32_t *off;     // ntiles * nb run starts in the edge list, tile-major
    uint32_t *bstart;  // nb + 1 bucket starts (the edge list is bucket-major)
    uint32_t nb, ntiles;  // nb == 0: gathers go directly to HBM
};
struct SortPlan {
    uint32_t sort_tiles, compact_tiles, hist_blocks, run_blocks;
    uint64_t hist_words, partial_words;
};
SortPlan sort_plan(size_t N);

// One signature round: signatures + hashes (and the periodic table clear),
// then grouping through the table, then the round-end bookkeeping.
struct RoundArgs {
    const uint32_t *cols;
    const uint32_t *colmap;
    size_t N;
    uint32_t k_eff;
    uint32_t *blockA, *blockB;
    uint32_t *sig;
    uint64_t *hash;
    unsigned long long *table;
    uint64_t table_cap;  // power of two
    uint32_t *multi;
    unsigned long long *active;
    const unsigned long long *accbits;
    uint32_t *counters;  // kSpread * kSpreadStride words, zero between rounds
    uint32_t *presence;  // 2^kPatternMaxBits bits, zero between calls
    uint32_t *presence_packed;  // label map, kLabelMapBytes bytes, zero when a refinement starts
    uint8_t *lab8;       // round-0 labels as bytes (packed round 1 only)
    RoundCtl *ctl;
    int lds_stage;              // 0 never, 1 and 2 (automatic) every round
    uint32_t round_grid_cap;    // workgroups of the round kernels (0 = one per 256 states)
    uint32_t pattern_grid_cap;  // workgroups of the label rounds
    uint32_t cached_probe;      // probe the table with cached loads first
    uint32_t insert_pair;       // 1: LDS-staged grouping with two states per thread
    unsigned long long *chg;      // N/64 words
    unsigned long long *single;   // N/64 words, zero before the first round
    unsigned long long *touched;  // 2 * (N/64) words, zero before the first round
    // 2 * summary_words(N) words: in the words of parity r & 1, bit g is set
    // when a state of group g (2^kSumShift states) changed its id in round r
    unsigned long long *chg_sum;
    uint32_t grouping;          // 0: hash table; 1: sort (radix sort of the key hashes)
    uint32_t hash_bits;         // 0: full hashes; else only the low bits (collision tests)
    SortBuffers sort;           // grouping == 1
    SegArgs seg;                // nseg == 0: a single automaton
    PbArgs pb;                  // nb > 0: dense rounds gather through slices in LDS
    // segmented refinements: round 0 by acceptance patterns (segpat_bits =
    // k_eff + 1 > 0), with a table of nseg << segpat_bits words and one
    // pattern per state
    uint32_t *segpat_table;
    uint16_t *segpat;
    uint32_t segpat_bits;
};
// Largest pattern width (bits) and table (words) of the segmented pattern
// round.
constexpr uint32_t kSegPatMaxBits = 16;
constexpr uint64_t kSegPatMaxWords = 1ull << 24;
// Round 0 of a segmented refinement without the table: every state's key is
// its segment and the acceptance of itself and its successors, and each key
// takes its smallest state as the block id (segpat_bits > 0).
void launch_seg_pattern(const RoundArgs &a, hipStream_t s);
// Builds the buckets of PbArgs for the k_eff columns of `cols` (colmap):
// needs pb.tl / pb.src (E = N * k_eff entries), pb.cnt and pb.off (ntiles *
// nb each), pb.bstart (nb + 1), and scratch: `csum` (pb_chunk_words(nb,
// ntiles) words) and `btot` (nb words); k_eff must be 1 to 8 or 16 and
// N <= kPbMaxBuckets << kPbSliceLog.
uint64_t pb_chunk_words(uint32_t nb, uint32_t ntiles);
void launch_pb_build(const uint32_t *cols, const uint32_t *colmap, size_t N, uint32_t k_eff,
                     const PbArgs &pb, uint32_t *csum, uint32_t *btot, hipStream_t s);
// Grouping of the round by sorting (grouping == 1), in place of the table
// kernels.
void launch_sort_group(const RoundArgs &a, hipStream_t s);
// One round: marking of the blocks to refine, signatures, grouping, the
// round end.
void launch_round(const RoundArgs &a, hipStream_t s);
// Up to `rounds` rounds (table grouping; one DFA, or the segments of a batch
// with their per-segment bookkeeping) in one cooperative launch of at most as
// many workgroups as fit on the device together; stops early once the
// partition is stable.  hipErrorInvalidValue for sort-grouped rounds.
hipError_t launch_rounds_persistent(const RoundArgs &a, uint32_t rounds, hipStream_t s);
// The marking kernel alone (also clears the table every kEpochs rounds).
void launch_mark(const RoundArgs &a, hipStream_t s);
// The next round refines every state of a multi-state block (used after the
// signature letters change).
void launch_ctl_full(RoundCtl *ctl, hipStream_t s);
// Per-segment block counts of the round, then the per-segment bookkeeping
// (all no-ops once the refinement has stopped); run before the round end.
// A segment whose partition did not change, or a pair whose start states
// separated, is decided: its states are marked as skipped (singleton bits)
// and it takes part in no later round.
void launch_seg_round(const RoundArgs &a, hipStream_t s);
// The launches of launch_round, separately (for kernel timing); the two
// slice passes launch nothing without bucketed edges (pb.nb == 0) and do
// nothing in rounds that gather directly.
void launch_pb_gather(const RoundArgs &a, hipStream_t s);
void launch_signature_pb(const RoundArgs &a, hipStream_t s);
// Round 1 (packed labels, k_eff <= 4) through the slices: the byte labels'
// pass A, then the keys and the label count per source tile.
void launch_packed_pb(const RoundArgs &a, hipStream_t s);
void launch_signature(const RoundArgs &a, hipStream_t s);
void launch_insert(const RoundArgs &a, hipStream_t s);
void launch_round_end(const RoundArgs &a, hipStream_t s);
// The label-round kernels without their round end.
void launch_pattern_kernel(const RoundArgs &a, hipStream_t s);
void launch_packed_kernel(const RoundArgs &a, hipStream_t s);
// Round 0 from acceptance bit patterns (requires k_eff + 1 <= kPatternMaxBits).
void launch_pattern_round(const RoundArgs &a, hipStream_t s);
// Round 1 from the packed round-0 labels of q and its successors (requires
// (k_eff + 1)^2 <= kPackedMaxBits and lab8 written by the pattern round).
void launch_packed_round(const RoundArgs &a, hipStream_t s);

// ---- leader-based refinement (naivePR; leader_kernels.hip) ----
//
//   block       uint32 [N]          leader (smallest member) of q's block,
//                                   updated in place by the move kernel
//   new_leader  uint64 [N]          election slot of block b: (tag << 32) | q
//                                   with tag = 2^32 - 1 - round; all ones
//                                   before the first round of a call
//   moved       uint64 [ceil(N/64)] states separated in the current round
struct LeaderArgs {
    const uint32_t *cols;
    const uint32_t *colmap;
    size_t N;
    uint32_t k_eff;
    uint32_t pad;
    uint32_t *block;
    unsigned long long *new_leader;
    unsigned long long *moved;
    uint32_t *counters;  // kSpread * kSpreadStride words, zero between rounds
    RoundCtl *ctl;
};
// Initial leaders: block[q] = smallest accepting or smallest rejecting state
// of q's class, from the acceptance bits; lead: 2 words preset to all ones.
void launch_leader_init(const unsigned long long *accbits, size_t N, uint32_t *lead,
                        uint32_t *block, hipStream_t s);
// One round (elect, move, end); the three launches separately for timing.
void launch_leader_round(const LeaderArgs &a, hipStream_t s);
// Up to `rounds` leader rounds in one cooperative launch (co-resident grid);
// stops early once no state moves.
hipError_t launch_leader_persistent(const LeaderArgs &a, uint32_t rounds, hipStream_t s);
void launch_leader_elect(const LeaderArgs &a, hipStream_t s);
void launch_leader_move(const LeaderArgs &a, hipStream_t s);
void launch_leader_end(const LeaderArgs &a, hipStream_t s);

// ---- reachability and the reachable sub-automaton (reach_kernels.hip) ----
struct ReachArgs {
    const uint32_t *delta;           // row-major n x k, targets < n (checked first)
    uint32_t n, k;
    unsigned long long *visited;     // n/64 words, zero before the search
    uint8_t *mark;                   // n: 0 unvisited, 1 settled, 2 / 3 dense frontier
    uint32_t *qa;                    // frontier queue, n entries
    uint32_t *sizes;                 // [0] entries in qa, [1] marks stored by a dense level
};
// *err = 1 if a target is >= n.
void launch_check_targets(const uint32_t *delta, uint64_t total, uint32_t n, uint32_t *err,
                          hipStream_t s);
void launch_bfs_init(const ReachArgs &a, uint32_t start, hipStream_t s);
// Expands levels in one workgroup while sizes[0] * k <= bfs_narrow_cap().
void launch_bfs_narrow(const ReachArgs &a, hipStream_t s);
uint32_t bfs_narrow_cap();
// The count listed states of qa become the frontier mark f.
void launch_bfs_list_to_marks(const ReachArgs &a, uint32_t count, uint8_t f, hipStream_t s);
// One dense level: frontier f expands into nf; sizes[1] = marks stored
// (0 iff no new state).
void launch_bfs_dense(const ReachArgs &a, uint8_t f, uint8_t nf, hipStream_t s);
// The states marked f settle and are listed in qa; sizes[0] = their number.
void launch_bfs_marks_to_list(const ReachArgs &a, uint8_t f, hipStream_t s);
// flags[q] = q if marked (reached), all ones otherwise.
void launch_reach_flags(const uint8_t *mark, size_t n, uint32_t *flags, hipStream_t s);
// sub_delta[i][a] = dense[delta[orig[i]][a]], sub_acc[i] = acc[orig[i]], i < *m_dev.
void launch_sub_dfa(const uint32_t *delta, const uint8_t *acc, uint32_t k, const uint32_t *orig,
                    const uint32_t *dense, const uint32_t *m_dev, uint32_t m_host,
                    uint32_t *sub_delta, uint8_t *sub_acc, hipStream_t s);
// block_out[q] = orig[sub_block[dense[q]]] if marked, all ones otherwise.
void launch_reach_expand(const uint8_t *mark, size_t n, const uint32_t *dense,
                         const uint32_t *orig, const uint32_t *sub_block, uint32_t *block_out,
                         hipStream_t s);

// Pointer jumping, level i >= 1, all k letters:
// cols[(i*k+a)*N + q] = cols[((i-1)*k+a)*N + cols[((i-1)*k+a)*N + q]];
// diff[i*k+a] = 1 if the level differs from level i-1 somewhere,
// nonid[i*k+a] = 1 if it is not the identity.
// Identity / previous-level flags of ncols closure columns (k letters per
// level) over the states whose bit in `single` is clear; diff and nonid must
// be zero.
void launch_column_flags(const uint32_t *cols, size_t N, uint32_t k, uint32_t ncols,
                         const unsigned long long *single, uint32_t *diff, uint32_t *nonid,
                         hipStream_t s);
void launch_jump(uint32_t *cols, size_t N, uint32_t k, uint32_t level, uint32_t *diff,
                 uint32_t *nonid, hipStream_t s);

// Canonical renumbering: out[q] = min{ q' : ids[q'] == ids[q] } for ids <
// id_range; scratch_min holds id_range words.
// Zeroes up to kZeroRegions byte regions (8-byte aligned, sizes multiples of
// 8) in one launch.
constexpr int kZeroRegions = 8;
struct ZeroList {
    unsigned long long *p[kZeroRegions];
    size_t words[kZeroRegions];  // 8-byte words
    int count;
};
void launch_zero(const ZeroList &z, hipStream_t s);
void launch_canonicalise(const uint32_t *ids, size_t N, size_t id_range, uint32_t *scratch_min,
                         uint32_t *out, hipStream_t s);

// Dense quotient numbering of a canonical partition: dense[l] for every
// leader l (block[l] == l) in increasing order; leader_of[b] = l;
// *num_blocks = B.  partials needs ceil(N / kScanTile) + 1 words.
constexpr uint32_t kScanTile = 1024;
void launch_dense_leaders(const uint32_t *block, size_t N, uint32_t *partials, uint32_t *dense,
                          uint32_t *leader_of, uint32_t *num_blocks, hipStream_t s);

// qdelta[b*k + a] = dense[block[delta[l*k + a]]], qacc[b] = acc[l] for
// l = leader_of[b]; *qstart = dense[block[start]].  dq: n words of scratch.
void launch_quotient(const uint32_t *delta, const uint8_t *acc, uint32_t k,
                     const uint32_t *block, const uint32_t *dense, const uint32_t *leader_of,
                     const uint32_t *num_blocks, uint32_t n, uint32_t start, uint32_t *dq,
                     uint32_t *qdelta, uint8_t *qacc, uint32_t *qstart, hipStream_t s);
// Quotient of a discrete partition (num_blocks == n): a copy of the input.
void launch_quotient_identity(const uint32_t *delta, const uint8_t *acc, uint32_t n, uint32_t k,
                              uint32_t start, uint32_t *qdelta, uint8_t *qacc, uint32_t *qstart,
                              hipStream_t s);

// ---- small DFAs, one workgroup each (batch_kernels.hip) ----
// A job: one DFA (nb == 0: minimisation, block ids to out_blocks + out) or
// the disjoint union of two DFAs with the same k (equivalence: the verdict).
// States are local: DFA a's are 0 .. na-1, DFA b's follow.
constexpr uint32_t kSmallThreads = 256;  // threads of a job's workgroup
constexpr uint32_t kSmallMaxK = 16;      // letters of a job
constexpr uint32_t kSmallMaxStates = 16384;  // states of a job (ids are 16-bit)
struct SmallJob {
    const uint32_t *delta_a, *delta_b;  // device, row-major
    const uint8_t *acc_a, *acc_b;
    uint32_t na, nb, k, start_a, start_b;
    uint32_t index;  // DFA or pair index in the call (results[index])
    uint64_t out;    // minimisation: offset of the DFA's ids in out_blocks
};
struct SmallResult {
    uint32_t num_blocks, rounds, changing, verdict, limit;
};
// LDS bytes of a job of n states (table of 2^ceil(log2 2n) >= 64 words and
// two 16-bit id arrays).
uint32_t small_refine_lds_bytes(uint32_t n);
// Workgroups that fit on the device at once with that much LDS (0: none).
int small_refine_max_groups(uint32_t lds_bytes, int device_cus);
// Refines every job (largest first: jobs sorted by size, taken from a
// counter); *err = 1 if some target is out of range; results[job.index].
void launch_small_refine(const SmallJob *jobs, uint32_t njobs, uint32_t groups, uint32_t lds_bytes,
                         uint32_t *next_job, uint32_t *out_blocks, SmallResult *results,
                         uint32_t max_rounds, uint32_t *err, hipStream_t s);

// ---- product exploration (product_kernels.hip) ----
struct ProductArgs {
    const uint32_t *dA, *dB;   // row-major
    const uint8_t *accA, *accB;
    uint32_t k;
    int mode;                  // 0 inclusion, 1 equivalence
    const unsigned long long *frontier;
    uint32_t frontier_size;
    unsigned long long *next;  // capacity next_cap
    uint32_t next_cap;
    uint32_t *next_size;       // atomic counter
    unsigned long long *visited;
    uint64_t visited_cap;      // power of two
    uint32_t *bad;             // set to 1 when a refuting pair is reached
    uint32_t *overflow;        // set to 1 when `next` overflows
};
void launch_product_level(const ProductArgs &a, hipStream_t s);
// Narrow exploration inside one workgroup (LDS queues of kProductNarrowCap
// pairs): requires frontier_size * k <= kProductNarrowCap and room in the
// visited set for max_levels * kProductNarrowCap more pairs at half load;
// out[0..3] = (frontier size, pairs added, levels, refuted); out[3] must be
// zero on entry.  The frontier stays in a.frontier.
constexpr uint32_t kProductNarrowThreads = 1024;
constexpr uint32_t kProductNarrowCap = 8192;
void launch_product_narrow(const ProductArgs &a, uint32_t max_levels, uint32_t *out,
                           hipStream_t s);
void launch_visited_clear(unsigned long long *visited, uint64_t cap, hipStream_t s);
void launch_visited_insert_start(unsigned long long *visited, uint64_t cap,
                                 unsigned long long key, hipStream_t s);
void launch_rehash(const unsigned long long *old_tab, uint64_t old_cap,
                   unsigned long long *new_tab, uint64_t new_cap, hipStream_t s);

}  // namespace dfamin
