/*
 * dfamin.h -- C ABI of libdfamin, parallel partition refinement for DFA
 * minimisation, equivalence and inclusion checking on AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Heemstra, Martens, Wijs, "Evaluating Massively Parallel Algorithms
 * for DFA Minimisation, Equivalence Checking and Inclusion Checking".
 *
 *   - A DFA is the 5-tuple (Q, Sigma, delta, F, q0) of Section 2 (Definition
 *     "Deterministic Finite Automaton"); states and letters are dense indices
 *     (Section 2, "Representation").
 *   - Minimisation computes the coarsest partition of Q that refines
 *     {F, Q\F} and is stable under every letter (Section 2; Section 3.3,
 *     Algorithm 4 computes it by signature rounds).  No unreachable states
 *     are removed: every one of the n states is partitioned (Section 2 treats
 *     reachability pruning as a separate pre-processing step).
 *   - Equivalence decides L(A) = L(B) (Section 4, Algorithm 6; here decided by
 *     refining the disjoint union, which Section 4 names as the alternative).
 *   - Inclusion decides L(A) <= L(B) (Section 4: the Hopcroft-Karp loop with
 *     the acceptance test changed to "q_A in F_A and q_B not in F_B", over the
 *     plain set of reached pairs).
 *
 * Conventions shared by every call:
 *   - delta is row-major: delta[q*k + a] = delta(q, a), uint32, every target
 *     < n.  (The paper stores |Sigma| arrays delta[a][q]; the library
 *     re-lays the table out itself.)
 *   - accepting[q] != 0 iff q is in F.
 *   - Block ids are canonical: block_out[q] = the smallest state index in q's
 *     block, so results do not depend on thread scheduling.
 *   - Indices are uint32 (n < 2^32 - 1); sizes of n*k are 64-bit internally.
 *   - Every call returns DFA_OK (0) or a negative status; nothing is thrown
 *     across the ABI.  dfa_last_error() describes the last failure on the
 *     calling thread.
 *   - Calls block until their results are ready.  Calls on one device are
 *     serialised inside the library (it keeps one grow-only device workspace
 *     per device).
 *   - Calls may come from several host threads.  The graph loop builds its
 *     round graphs node by node and captures no stream, so nothing another
 *     thread does can disturb it.  During a call, the calling thread's
 *     stream-capture interaction mode is relaxed, so the library's
 *     allocations never invalidate a capture that another thread (of the
 *     caller, or another library) has in progress.
 *   - The caller owns every buffer it passes; the library keeps no pointer
 *     after a call returns.
 *   - Host-pointer calls (dfa_minimise, dfa_equivalent, dfa_included) copy the
 *     inputs to the device and the results back.  The *_device variants take
 *     device pointers (memory of the current HIP device) and a hipStream_t
 *     (passed as void*, NULL = the library's own stream); their inputs must
 *     stay unchanged until the call returns.
 */
#ifndef DFAMIN_H
#define DFAMIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define DFA_OK 0
#define DFA_EINVAL (-1)  /* bad argument: n == 0, k == 0, target >= n, start >= n,
                            k mismatch, NULL required pointer */
#define DFA_ENOMEM (-2)  /* device allocation failed / request exceeds the budget */
#define DFA_EDEVICE (-3) /* a HIP runtime error */
#define DFA_EAGAIN (-4)  /* served request not finished yet */
#define DFA_ELIMIT (-5)  /* options.max_rounds reached before the partition was stable */
#define DFA_ECANCELED (-6) /* served request cancelled when its server was destroyed */

/* ---- partial transitive closure (Section 3.4, Algorithm 5) ---- */
#define DFA_TC_OFF 0  /* refine on the input letters only */
#define DFA_TC_ON 1   /* add the letters a^(2^i), i = 1..floor(log2 n), first */
#define DFA_TC_AUTO 2 /* start plain; switch to the closure when splitting stalls */

/* ---- refinement algorithm ---- */
#define DFA_ALGO_SIGNATURE 0 /* signature rounds with hashing: every block splits into
                                all its classes at once (Section 3.3, Algorithm 4) */
#define DFA_ALGO_SORT 2      /* signature rounds grouped by a stable radix sort of the
                                signature hashes instead of the hash table (the grouping of
                                sortPR, Section 3.3, Algorithm 4); same partitions and rounds
                                as DFA_ALGO_SIGNATURE.  Single-DFA calls only. */
#define DFA_ALGO_LEADER 1    /* leader rounds, naivePR (Section 3.2, Algorithm 2): the
                                states that differ from their block's leader leave it
                                together; with DFA_TC_ON this is transPR (Algorithm 5
                                followed by naivePR).  Same partition, more rounds,
                                no hash table.  Single-DFA calls only. */

/* ---- round-loop driver ---- */
#define DFA_LOOP_HOST 0  /* the host reads the block count after every round */
#define DFA_LOOP_CHUNK 1 /* rounds are enqueued in chunks; kernels turn into no-ops
                            on the device once the partition is stable; the host
                            checks once per chunk */
#define DFA_LOOP_GRAPH 2 /* like CHUNK, each chunk replayed from a hipGraph (built once per chunk shape) */
#define DFA_LOOP_PERSISTENT 3 /* each chunk is one cooperative launch that loops over
                                 the rounds on the device, its phases separated by grid
                                 barriers, and stops as soon as the partition is stable
                                 (the while-loop of Algorithms 2 and 4, Section 3, kept
                                 on the device).  Calls with DFA_ALGO_SIGNATURE
                                 (single and batched) or DFA_ALGO_LEADER; DFA_EINVAL
                                 with DFA_ALGO_SORT */

typedef struct dfa_options {
    int32_t tc_mode;      /* DFA_TC_*, default DFA_TC_AUTO */
    int32_t loop_mode;    /* DFA_LOOP_*, default DFA_LOOP_GRAPH */
    uint32_t start;       /* start state used for the quotient's start (default 0) */
    uint32_t max_rounds;  /* 0 = until stable */
    uint32_t chunk;       /* rounds per chunk in CHUNK/GRAPH mode; 0 = automatic: the
                             tuned start length (dfa_tuning.chunk), doubled after each
                             chunk that did not finish, up to 256 rounds (8 while
                             TC AUTO may still switch the closure on) */
    int32_t lds_stage;    /* 1 = pre-group keys in LDS before the global table,
                             0 = insert every key into the global table,
                             2 = automatic (default): currently as 1, which measured
                                 fastest or within 4% of 0 on every workload tried */
    int32_t algorithm;    /* DFA_ALGO_*, default DFA_ALGO_SIGNATURE; the batched calls
                             and the server accept only DFA_ALGO_SIGNATURE */
    int32_t prune;        /* dfa_minimise only: 0 = partition all n states (default, the
                             paper's convention, Section 2); 1 = only the states reachable
                             from `start` (breadth-first search first): block_out[q] =
                             DFA_UNREACHABLE for the others, ids are the smallest
                             reachable state of each block, and the quotient is the usual
                             minimal DFA.  The batched calls and the server accept only 0 */
    int32_t equiv_method; /* dfa_equivalent only: DFA_EQ_UNION (default) refines the
                             disjoint union; DFA_EQ_PRODUCT explores the synchronous
                             product breadth-first from (start_a, start_b) and stops at
                             the first pair with exactly one accepting side (Section 4's
                             Hopcroft-Karp over the plain set of reached pairs; the
                             refinement options are then ignored).  The batched calls
                             and the server accept only DFA_EQ_UNION */
    int32_t reserved;
} dfa_options;

#define DFA_EQ_UNION 0
#define DFA_EQ_PRODUCT 1

#define DFA_UNREACHABLE 0xFFFFFFFFu /* block_out value of a pruned state */

typedef struct dfa_stats {
    uint32_t rounds;          /* refinement rounds executed (signature or leader rounds);
                                 the last one confirms stability */
    uint32_t changing_rounds; /* rounds that split at least one block */
    uint32_t num_blocks;      /* blocks of the final partition */
    uint32_t k_eff;           /* letters per signature in the last round (k, or closure letters) */
    uint32_t tc_used;         /* 1 if the closure letters were built */
    uint32_t tc_levels;       /* floor(log2 n) when tc_used */
    uint32_t plain_rounds;    /* rounds run on the input letters before switching to the closure */
    uint32_t reachable;       /* states partitioned: n, or the reachable ones with prune;
                                 product exploration (dfa_included, DFA_EQ_PRODUCT): the
                                 pairs visited, saturating at 2^32 - 1, with `rounds` =
                                 the breadth-first levels expanded */
    double h2d_ms;            /* host-pointer calls: copy of the inputs */
    double device_ms;         /* device work of the call (HIP events) */
    double d2h_ms;            /* host-pointer calls: copy of the results */
    uint64_t transitions_refined; /* sum over rounds of n * k_eff (nominal) */
    uint64_t algorithmic_bytes;   /* signature rounds: sum over rounds of the refined
                                     states * (8*k_eff + 8); leader rounds: n * 4 per
                                     round plus the compared states * 16*k_eff */
} dfa_stats;

/* Quotient DFA: caller-provided arrays of capacity n*k (delta) and n
 * (accepting); the library fills the first num_blocks rows.  Blocks are
 * numbered densely in increasing order of their smallest member;
 * start = the block of options.start. */
typedef struct dfa_quotient {
    uint32_t *delta;
    uint8_t *accepting;
    uint32_t num_blocks; /* out */
    uint32_t start;      /* out */
} dfa_quotient;

/* One DFA operand of a two-DFA call. */
typedef struct dfa_view {
    uint32_t n, k, start;
    const uint32_t *delta;    /* n*k, row-major */
    const uint8_t *accepting; /* n */
} dfa_view;

/* Fill *opt with the defaults (TC AUTO, graph loop, LDS staging, start 0). */
void dfa_options_default(dfa_options *opt);

/*
 * Kernel tuning of the current device (launch shapes and kernel variants; no
 * effect on results).  Set by hand or by the package's autotuner (which
 * measures candidate tunings on the caller's workload and keeps the fastest
 * per device and workload shape); read by every later call on that device.
 * dfa_set_tuning returns DFA_EINVAL for out-of-range values.
 */
typedef struct dfa_tuning {
    uint32_t round_grid_cap; /* workgroups of the signature/grouping kernels (grid-stride
                                beyond); 0 = one workgroup per 256 states */
    uint32_t label_grid_cap; /* workgroups of the label rounds; 0 = one per 256 states */
    uint32_t label_rounds;   /* 0: every round uses the table; 1: round 0 groups by the bit
                                pattern of acceptance of q and its successors when
                                k_eff + 1 <= 17; 2: round 1 then groups by the packed
                                round-0 labels when (k_eff + 1)^2 <= 25 */
    uint32_t cached_probe;   /* 1: probe the grouping table with cached loads first */
    uint32_t chunk;          /* first chunk's rounds when options.chunk is 0 (1..4096) */
    uint32_t hash_bits;      /* 0 = full 64-bit key hashes (default); 1..63 keep only the
                                low bits, so that distinct keys share hashes: slower, still
                                exact (keys are always compared in full); for testing the
                                collision paths of both groupings */
    uint32_t batch_lds_states; /* batched calls: DFAs (equivalence: pairs) of at most this many
                                  states and at most 16 letters are refined whole inside one
                                  workgroup, ids and table in LDS; the others go through the
                                  segmented refinement.  0 = never; at most 16384, and lowered
                                  to what one workgroup's LDS holds on the device */
    uint32_t insert_pair;      /* 1 (default): the LDS-staged grouping kernel takes two states
                                  per thread when k_eff is 1, 2, 3, 4 or 8; 0: one */
    uint32_t slice_min_states; /* single-DFA refinements of at least this many states (and at
                                  most 2^24, k_eff 1..8 or 16, no closure, not the persistent
                                  loop) bucket their edges by target slice once, and their
                                  dense rounds in the first chunk gather successor ids through
                                  slices held in LDS; 0 = never; default 2^20 */
    uint32_t reserved[7];
} dfa_tuning;

void dfa_tuning_default(dfa_tuning *t);
int dfa_get_tuning(dfa_tuning *t);
int dfa_set_tuning(const dfa_tuning *t);

/*
 * Kernel timing for benchmarks.  While enabled on the current device, every
 * launch of a round kernel (signature, grouping, round end, label rounds) is
 * bracketed by HIP events on the library's stream, and chunks are launched
 * without graphs.  dfa_profile_enable(1) also clears the totals.
 * dfa_profile_read copies up to cap entries and sets *count to the number of
 * kernels seen.  algorithmic_bytes sums, over the launches, the states the
 * launch refined times the kernel's bytes per refined state (k = k_eff):
 * signature 8k + 4, grouping 4, label rounds 5k + 5, round end 0 (a whole
 * signature round is 8k + 8, the figure dfa_stats.algorithmic_bytes uses).
 * states sums the refined states and state_letters the refined states times
 * k_eff (the signature kernel's successor-id gathers).
 */
typedef struct dfa_kernel_time {
    char name[32];
    uint64_t launches;
    double total_ms;
    uint64_t algorithmic_bytes;
    uint64_t states;
    uint64_t state_letters;
} dfa_kernel_time;

int dfa_profile_enable(int on);
int dfa_profile_read(dfa_kernel_time *out, int cap, int *count);
/* Restricts the timing to the round kernel of that name (as reported in
 * dfa_kernel_time.name, e.g. "k_signature"): the other kernels run without
 * events, so the timed region is barely disturbed.  NULL or "" times every
 * round kernel again.  Kept across dfa_profile_enable calls.  DFA_EINVAL for
 * a name of 32 characters or more. */
int dfa_profile_only(const char *name);

/*
 * Minimise one DFA (Section 2 problem statement; Section 3.3, Algorithm 4
 * signature rounds; Section 3.4, Algorithm 5 closure).
 *   n, k        states and letters (both >= 1)
 *   delta       host, n*k uint32, row-major, every entry < n
 *   accepting   host, n bytes
 *   block_out   host, n uint32: canonical block id per state
 *   q_out       optional quotient (host arrays), NULL to skip
 *   opt, stats  optional (NULL = defaults / not reported)
 * Errors: DFA_EINVAL (bad sizes, target >= n, start >= n, NULL required
 * pointer), DFA_ENOMEM, DFA_EDEVICE, DFA_ELIMIT (block_out then holds the
 * partition reached so far).
 */
int dfa_minimise(uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *accepting,
                 uint32_t *block_out, dfa_quotient *q_out, const dfa_options *opt,
                 dfa_stats *stats);

/* As dfa_minimise with device pointers (delta, accepting, block_out and the
 * quotient arrays) on `stream`. */
int dfa_minimise_device(uint32_t n, uint32_t k, const uint32_t *delta,
                        const uint8_t *accepting, uint32_t *block_out, dfa_quotient *q_out,
                        const dfa_options *opt, dfa_stats *stats, void *stream);

/*
 * dfa_minimise_device for callers that cannot allocate device memory (code
 * in tight serving loops, harnesses that forbid hipMalloc): the call makes no
 * device allocation and frees nothing.  Same arguments, results and errors
 * as dfa_minimise_device; the caller still passes the inputs and outputs.
 *   - Every buffer the call needs is carved from a fixed workspace of
 *     256 MiB, a static device array that each device running this entry
 *     point holds until the process ends.  A plain refinement needs about
 *     n*(8k + 41) bytes plus a hash table of 8 * 2^ceil(log2 2n) bytes and
 *     about 4.1 MiB of label bitmaps (e.g. n up to about 2^21 at k = 4).
 *   - DFA_ENOMEM, before any work, when that estimate exceeds the workspace;
 *     DFA_ENOMEM also when a later part of the call does not fit (closure
 *     letters with DFA_TC_ON, pruning).  With DFA_TC_AUTO a closure that does
 *     not fit is skipped and plain rounds continue (same partition).
 *   - DFA_LOOP_GRAPH runs as DFA_LOOP_CHUNK (instantiating a graph allocates);
 *     the kernel tuning is the default one (dfa_tuning_default).
 *   - Calls on one device share that device's workspace, which keeps the last
 *     call's contents; every call clears what must start at zero.  Calls
 *     that overlapped on one device would race on it, so the library runs
 *     them one at a time (a lock of their own, separate from the other
 *     entry points') and each returns only when its work on the device is
 *     done.
 */
int dfa_minimise_device_fixed(uint32_t n, uint32_t k, const uint32_t *delta,
                              const uint8_t *accepting, uint32_t *block_out,
                              dfa_quotient *q_out, const dfa_options *opt, dfa_stats *stats,
                              void *stream);

/*
 * Equivalence L(a) = L(b) (Section 4, Algorithm 6's result; decided by
 * minimising the disjoint union and comparing the blocks of the two start
 * states, with an early exit as soon as they separate).
 *   a, b     host views; a->k must equal b->k
 *   verdict  out: 1 if equivalent, 0 otherwise
 */
int dfa_equivalent(const dfa_view *a, const dfa_view *b, int *verdict,
                   const dfa_options *opt, dfa_stats *stats);
int dfa_equivalent_device(const dfa_view *a, const dfa_view *b, int *verdict,
                          const dfa_options *opt, dfa_stats *stats, void *stream);

/*
 * Inclusion L(a) <= L(b) (Section 4: breadth-first exploration of the pairs
 * reachable from (start_a, start_b) in the synchronous product, stopping at a
 * pair (p, q) with p accepting in a and q not accepting in b).
 *   verdict          out: 1 if included, 0 otherwise
 *   pairs_visited    optional out: distinct pairs reached (the whole
 *                    reachable product when the verdict is 1)
 */
int dfa_included(const dfa_view *a, const dfa_view *b, int *verdict, uint64_t *pairs_visited,
                 const dfa_options *opt, dfa_stats *stats);
int dfa_included_device(const dfa_view *a, const dfa_view *b, int *verdict,
                        uint64_t *pairs_visited, const dfa_options *opt, dfa_stats *stats,
                        void *stream);

/*
 * Batches: many independent DFAs refined together in one set of launches
 * (one refinement over their disjoint union; each DFA's states start in its
 * own two classes, so no block spans two DFAs; DFAs with fewer letters are
 * padded with identity letters, which change no partition).  Results are the
 * same as those of the single-DFA calls.  The closure is built only with
 * tc_mode ON (AUTO acts as OFF in batches).
 */
typedef struct dfa_batch_stats {
    uint32_t count;           /* DFAs (or pairs) in the batch */
    uint32_t rounds;          /* rounds of the joint refinement (max over DFAs) */
    uint32_t k_eff;           /* letters per signature of the joint refinement */
    uint32_t reserved0;
    double h2d_ms, device_ms, d2h_ms;
    uint64_t states;              /* states in the union */
    uint64_t transitions_refined; /* sum over DFAs of n * k * (their own rounds) */
    uint64_t algorithmic_bytes;   /* as dfa_stats, for the joint refinement */
} dfa_batch_stats;

/*
 * Minimise count DFAs (Section 3.3, Algorithm 4, per DFA).
 *   dfas           count host views (n, k, start, delta, accepting); start unused
 *   blocks_concat  host; DFA i's canonical block ids (local state indices) at
 *                  block_offsets[i] (NULL: packed back to back in order)
 *   num_blocks     optional, count entries: blocks of each DFA
 *   rounds         optional, count entries: each DFA's own rounds (as dfa_stats.rounds)
 * Errors as dfa_minimise; "dfas[i]: ..." names the offending DFA.
 */
int dfa_minimise_batch(uint32_t count, const dfa_view *dfas, uint32_t *blocks_concat,
                       const uint64_t *block_offsets, uint32_t *num_blocks, uint32_t *rounds,
                       const dfa_options *opt, dfa_batch_stats *stats);
/* Device variant: views and blocks_concat point to device memory;
 * block_offsets, num_blocks and rounds stay host arrays. */
int dfa_minimise_batch_device(uint32_t count, const dfa_view *dfas, uint32_t *blocks_concat,
                              const uint64_t *block_offsets, uint32_t *num_blocks,
                              uint32_t *rounds, const dfa_options *opt, dfa_batch_stats *stats,
                              void *stream);

/*
 * Decide count equivalences L(a[i]) = L(b[i]) (Section 4) in one refinement
 * of the union of all pairs.  verdicts: host, count entries, 1 = equivalent.
 * a[i].k must equal b[i].k.
 */
int dfa_equivalent_batch(uint32_t count, const dfa_view *a, const dfa_view *b, int32_t *verdicts,
                         const dfa_options *opt, dfa_batch_stats *stats);
int dfa_equivalent_batch_device(uint32_t count, const dfa_view *a, const dfa_view *b,
                                int32_t *verdicts, const dfa_options *opt,
                                dfa_batch_stats *stats, void *stream);

/*
 * Served requests (continuous batching).  A server runs `lanes` workers,
 * each with its own HIP stream and device workspace.  Submitted requests
 * wait in FIFO order and are admitted while their device-memory footprint
 * fits hbm_budget.  A free lane takes the head request: requests with more
 * than batch_max_states states run alone (closure per tc_mode); smaller ones
 * of the same kind are refined together (up to max_group, one segmented
 * refinement, at most batch_round_budget rounds), and any that are not stable
 * by then run again alone with the closure.  Lanes overlap on the device, so
 * requests arriving while others run start as soon as a lane and memory are
 * free.  Results are the same as the single-request calls and do not depend
 * on the other requests in the mix.
 */
#define DFA_REQ_MINIMISE 0
#define DFA_REQ_EQUIVALENT 1

typedef struct dfa_server dfa_server;

typedef struct dfa_server_config {
    size_t hbm_budget;           /* device bytes for admitted requests (0 = half the free memory) */
    uint32_t lanes;              /* concurrent workers / streams (1..16, default 4) */
    uint32_t max_group;          /* requests per batched refinement (default 512) */
    uint32_t batch_max_states;   /* larger requests run alone (default 2^18) */
    uint32_t batch_round_budget; /* rounds of a batched refinement (>= 3, default 12) */
    int32_t tc_mode;             /* closure for requests run alone (default DFA_TC_AUTO) */
    uint32_t paused;             /* 1: the lanes take no request until dfa_server_resume
                                    (requests are still accepted and queued); default 0 */
    uint32_t reserved[8];
} dfa_server_config;

typedef struct dfa_request {
    int32_t kind;      /* DFA_REQ_MINIMISE or DFA_REQ_EQUIVALENT */
    uint32_t reserved;
    dfa_view a;        /* host view; copied by dfa_server_submit */
    dfa_view b;        /* second operand of an equivalence request */
} dfa_request;

typedef struct dfa_result {
    int32_t status;           /* DFA_OK or the request's error */
    int32_t verdict;          /* equivalence: 1 if equivalent */
    uint32_t num_blocks;      /* minimise */
    uint32_t rounds;          /* rounds of the request's own refinement */
    const uint32_t *blocks;   /* minimise: n canonical block ids, owned by the server
                                 until dfa_result_release */
    uint32_t n;
    uint32_t batched;         /* 1 if it ran in a batched refinement */
    double queue_ms;          /* submit -> start */
    double service_ms;        /* start -> done (of its group) */
    double latency_ms;        /* submit -> done */
    /* parts of service_ms, for the work the request ran in (its group's when
     * batched): input copies to the device (HIP events), device work of the
     * refinements (HIP events; a re-run alone included), result copy back */
    double h2d_ms, device_ms, d2h_ms;
} dfa_result;

typedef struct dfa_server_stats {
    uint64_t submitted, completed, rejected, pending;
    uint64_t batched_groups, solo_runs;
    double p50_ms, p99_ms, mean_ms; /* latency of completed requests */
    double uptime_s, requests_per_s;
    uint64_t hbm_in_use, hbm_budget;
    uint64_t waiting_threads;       /* threads blocked in dfa_server_wait */
} dfa_server_stats;

void dfa_server_config_default(dfa_server_config *cfg);
/* NULL on failure (see dfa_last_error).  Uses the current HIP device. */
dfa_server *dfa_server_create(const dfa_server_config *cfg);
/* Device bytes the server charges against hbm_budget for running `req`
 * alone: its inputs and workspace, plus a fixed part for the lane's buffers.
 * Admission also counts the workspaces that idle lanes keep from earlier
 * requests; when the head request does not fit beside them, the idle lanes
 * free theirs first, so device memory held by the server stays within the
 * budget. */
int dfa_server_footprint(const dfa_server *s, const dfa_request *req, size_t *bytes);
/* Copies the request's arrays into page-locked host memory (pooled by the
 * server; large arrays are copied by several threads), so the caller may free
 * them on return; the lane that runs the request uploads them asynchronously.
 * DFA_ENOMEM if the request can never fit the budget. */
int dfa_server_submit(dfa_server *s, const dfa_request *req, uint64_t *ticket);
/* DFA_EAGAIN while the request runs or waits. */
int dfa_server_poll(dfa_server *s, uint64_t ticket, dfa_result *out);
/* Blocks until the request is done.  A thread may wait while another thread
 * destroys the server: a request that had not started then returns with
 * out->status = DFA_ECANCELED (and out->blocks = NULL), and
 * dfa_server_destroy returns only after every such waiter has left. */
int dfa_server_wait(dfa_server *s, uint64_t ticket, dfa_result *out);
/* Lets the lanes of a server created with cfg.paused = 1 take requests. */
int dfa_server_resume(dfa_server *s);
/* Frees a finished request's result (the blocks pointer becomes invalid). */
int dfa_result_release(dfa_server *s, uint64_t ticket);
int dfa_server_get_stats(dfa_server *s, dfa_server_stats *out);
/* Cancels waiting requests (status DFA_ECANCELED), waits for running ones,
 * frees the lanes' workspaces (their streams are kept by the library for
 * later servers).  Results not released are freed too.  Apart from threads
 * blocked in dfa_server_wait, no other call on the same server may run
 * concurrently with it or follow it. */
void dfa_server_destroy(dfa_server *s);

/* Description of the last failure on the calling thread ("" if none). */
const char *dfa_last_error(void);

/* Name, compute-unit count and memory of the current HIP device. */
int dfa_device_info(char *name, size_t name_cap, int *compute_units, size_t *hbm_bytes);

#ifdef __cplusplus
}
#endif

#endif /* DFAMIN_H */
