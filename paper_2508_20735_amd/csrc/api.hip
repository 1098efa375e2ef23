// C ABI of libdfamin: argument checks, device workspace, the round-loop
// drivers and the host/device copies.  All compute runs in the kernels of
// refine_kernels.hip and product_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <exception>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <string>
#include <vector>

#include "dfamin.h"
#include "dfamin_internal.h"

// Workspace of dfa_minimise_device_fixed, the entry point that allocates no
// device memory: every buffer of its calls is carved from this array.  Each
// device that runs that entry point holds its own copy until the process
// ends.  Host code never passes this name to a kernel or a copy (on the host
// it is a stand-in, not a device address); the device address comes from
// hipGetSymbolAddress, taken once per device.
static constexpr size_t kFixedScratchBytes = size_t(256) << 20;
static __device__ __align__(256) uint8_t scratch[kFixedScratchBytes];

namespace dfamin {

GraphRecorder *&graph_recorder() {
    thread_local GraphRecorder *recorder = nullptr;
    return recorder;
}

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    try {
        g_last_error = buf;
    } catch (...) {
        // the status still tells the caller what failed
    }
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(DFA_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define DFA_TRY(expr)              \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ != DFA_OK) return rc_; \
    } while (0)

// Grow-only device allocation.
// Every device allocation gets a new number, so that cached facts about a
// buffer's contents never outlive the allocation (a new one may reuse the
// address).
std::atomic<uint64_t> g_allocation_number{0};

// A fixed region of device memory that buffers are carved from instead of
// being allocated (the workspace of the allocation-free entry point); reset
// at the start of every call that uses it.
struct Arena {
    uint8_t *base = nullptr;
    size_t size = 0;
    size_t used = 0;
    uint64_t generation = 1;  // bumped by every reset: earlier carves are void
};

struct Buffer {
    void *p = nullptr;
    size_t cap = 0;
    uint64_t allocation = 0;  // number of the current allocation (0: none)
    Arena *arena = nullptr;   // carve from this region, never allocate
    uint64_t carved_in = 0;   // arena generation of the current carve
    int ensure(size_t bytes, const char *what) {
        if (arena && carved_in != arena->generation) {  // carved before the last reset
            p = nullptr;
            cap = 0;
        }
        if (p && bytes <= cap) return DFA_OK;
        if (arena) {
            // a region outgrown within a call is abandoned until the next reset
            const size_t want = (std::max<size_t>(bytes, 256) + 255) & ~static_cast<size_t>(255);
            if (want > arena->size - arena->used)
                return fail(DFA_ENOMEM,
                            "%s: %zu bytes do not fit the fixed workspace (%zu of %zu bytes "
                            "already in use)",
                            what, want, arena->used, arena->size);
            p = arena->base + arena->used;
            arena->used += want;
            cap = want;
            carved_in = arena->generation;
            allocation = ++g_allocation_number;
            return DFA_OK;
        }
        if (p) {
            (void)hipFree(p);
            p = nullptr;
            cap = 0;
        }
        size_t want = std::max<size_t>(bytes, 256);
        want = (want + (2u << 20) - 1) & ~static_cast<size_t>((2u << 20) - 1);
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(DFA_ENOMEM, "device allocation of %zu bytes for %s failed: %s", want, what,
                        hipGetErrorString(e));
        }
        cap = want;
        allocation = ++g_allocation_number;
        return DFA_OK;
    }
    template <class T>
    T *as() const {
        return static_cast<T *>(p);
    }
};

constexpr size_t kPinnedWords = 1u << 16;

// A chunk graph is reused while the round arguments and the chunk length
// are unchanged (RoundArgs / LeaderArgs values are built from zeroed storage,
// so they can be compared bytewise).
struct GraphKey {
    RoundArgs args;      // signature rounds (zero for leader rounds)
    LeaderArgs largs;    // leader rounds (zero for signature rounds)
    uint32_t chunk;
    uint32_t leader;
    bool operator==(const GraphKey &o) const { return std::memcmp(this, &o, sizeof *this) == 0; }
};

// Holds one device context's lock for the length of a library call, and for
// that long lets the calling thread allocate, free and synchronise without
// invalidating a graph capture that another thread (a server lane, another
// caller) has in progress: the thread's capture interaction mode is relaxed,
// and the caller's own mode comes back on return.
struct RelaxedCapture {
    hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
    RelaxedCapture() { (void)hipThreadExchangeStreamCaptureMode(&mode); }
    ~RelaxedCapture() { (void)hipThreadExchangeStreamCaptureMode(&mode); }
    RelaxedCapture(const RelaxedCapture &) = delete;
    RelaxedCapture &operator=(const RelaxedCapture &) = delete;
};

struct CallScope {
    RelaxedCapture relaxed;
    std::lock_guard<std::mutex> lock;
    explicit CallScope(std::mutex &m) : lock(m) {}
};

struct Ctx {
    std::mutex mu;
    bool inited = false;
    int device = -1;
    hipStream_t stream = nullptr;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_in = nullptr;
    uint32_t *pinned = nullptr;  // host staging for small transfers
    Buffer cols, tc_cols, colmap, blockA, blockB, sig, hash, table, ctl, flags, canon, dense,
        leader_of, partials, scalars, multi, active, accbits, counters, presence, presence_packed,
        lab8;
    dfa_tuning tune{};
    Buffer stage_delta, stage_acc, stage_block, stage_qdelta, stage_qacc, stage_delta_b,
        stage_acc_b;
    Buffer visited, visited2, front0, front1;
    Buffer new_leader, moved;
    Buffer chg, single, touched, chg_sum;
    // the column list last uploaded, and the allocation it went to
    std::vector<uint32_t> colmap_on_device;
    uint64_t colmap_on_device_in = 0;
    Buffer reach_visited, reach_qa, reach_qb, reach_flags, reach_dense, reach_orig, sub_delta,
        sub_acc, sub_block;
    Buffer sort_keys0, sort_keys1, sort_vals0, sort_vals1, sort_hist, sort_partials,
        sort_runhead, sort_m;
    Buffer serve_in;  // server lanes: device copies of the running requests' inputs
    hipEvent_t ev_p0 = nullptr, ev_p1 = nullptr;  // pruned minimisation, whole call
    hipEvent_t ev_up0 = nullptr, ev_up1 = nullptr;  // server lanes: a group's input copies
    // waits on the stream sleep instead of spinning (server lanes, so that
    // waiting lanes leave the host cores to submissions)
    bool blocking_sync = false;
    hipEvent_t ev_sync = nullptr;
    Buffer parts, tile_part, seg_words, batch_in, batch_out, tile_dead;
    Buffer small_jobs, small_results, small_ctl;  // batched small DFAs (one workgroup each)
    Buffer pb_tl, pb_src, pb_val, pb_off, pb_partials;  // edges bucketed by target slice
    Buffer segpat_table, segpat;  // round 0 of segmented refinements by acceptance patterns
    Arena arena;  // the allocation-free context's fixed workspace (unused elsewhere)
    uint8_t *pinned_batch = nullptr;  // host staging of batched inputs/outputs
    uint8_t *ring[2] = {nullptr, nullptr};  // page-locked chunks for large host copies
    hipEvent_t ring_ev[2] = {nullptr, nullptr};
    bool ring_recorded[2] = {false, false};  // ring_ev[i] has been recorded
    size_t pinned_batch_cap = 0;
    // chunk graphs, one per chunk length in use (automatic chunks grow
    // 4, 8, ..., 256 within one call), replaced round-robin
    static constexpr int kGraphSlots = 8;
    hipGraphExec_t graphs[kGraphSlots] = {};
    GraphKey graph_keys[kGraphSlots] = {};
    int graph_victim = 0;
    // kernel timing (dfa_profile_enable): event pairs around the round
    // kernels, folded into per-kernel totals after every readback
    bool profiling = false;
    std::string prof_only;  // time only this kernel ("" = every round kernel)
    struct KernelTime {
        uint64_t launches = 0;
        double ms = 0;
        uint64_t bytes = 0;
        uint64_t states = 0;         // refined states over the launches
        uint64_t state_letters = 0;  // refined states times k_eff
    };
    std::map<std::string, KernelTime> ktimes;
    struct Pending {
        const char *name;
        size_t ev0, ev1;
        uint32_t round;
        uint32_t bytes_per_state;
        uint32_t k_eff;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> evpool;
    size_t ev_used = 0;
};

constexpr int kMaxDevices = 64;
Ctx g_ctx[kMaxDevices];

int get_ctx(Ctx *&out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DFA_EDEVICE, "device index %d out of range", dev);
    out = &g_ctx[dev];
    return DFA_OK;
}

// Streams are never destroyed: a context that goes away (a server lane)
// returns its stream here and the next one takes it.  Destroying a stream
// while another thread of the process synchronises the whole device (which
// waits on every stream of the device) is a race the library cannot see
// from its side, so it never does it.
std::mutex g_stream_pool_mu;
std::vector<hipStream_t> g_stream_pool[kMaxDevices];

int take_stream(int dev, hipStream_t &out) {
    {
        std::lock_guard<std::mutex> g(g_stream_pool_mu);
        auto &pool = g_stream_pool[dev];
        if (!pool.empty()) {
            out = pool.back();
            pool.pop_back();
            return DFA_OK;
        }
    }
    // default priority; callers' streams are joined explicitly (join_stream)
    HIP_TRY(hipStreamCreateWithFlags(&out, hipStreamNonBlocking));
    return DFA_OK;
}

void give_stream(int dev, hipStream_t st) {
    if (!st || dev < 0 || dev >= kMaxDevices) return;
    try {
        std::lock_guard<std::mutex> g(g_stream_pool_mu);
        g_stream_pool[dev].push_back(st);
    } catch (...) {
        // not pooled: the stream stays allocated until the process ends
    }
}

int init_ctx(Ctx &c) {
    if (c.inited) return DFA_OK;
    HIP_TRY(hipGetDevice(&c.device));
    if (c.device < 0 || c.device >= kMaxDevices)
        return fail(DFA_EDEVICE, "device index %d out of range", c.device);
    DFA_TRY(take_stream(c.device, c.stream));
    HIP_TRY(hipEventCreate(&c.ev_start));
    HIP_TRY(hipEventCreate(&c.ev_stop));
    HIP_TRY(hipEventCreateWithFlags(&c.ev_in, hipEventDisableTiming));
    HIP_TRY(hipEventCreate(&c.ev_p0));
    HIP_TRY(hipEventCreate(&c.ev_p1));
    HIP_TRY(hipEventCreate(&c.ev_up0));
    HIP_TRY(hipEventCreate(&c.ev_up1));
    HIP_TRY(hipEventCreateWithFlags(&c.ev_sync, hipEventBlockingSync | hipEventDisableTiming));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&c.pinned), kPinnedWords * sizeof(uint32_t),
                          hipHostMallocDefault));
    dfa_tuning_default(&c.tune);
    c.inited = true;
    return DFA_OK;
}

// Waits for the context's stream: spinning (the default, lowest latency) or
// sleeping on a blocking-sync event (server lanes).
hipError_t stream_sync(Ctx &c) {
    if (!c.blocking_sync || !c.ev_sync) return hipStreamSynchronize(c.stream);
    hipError_t e = hipEventRecord(c.ev_sync, c.stream);
    if (e != hipSuccess) return e;
    return hipEventSynchronize(c.ev_sync);
}

dfa_options resolve(const dfa_options *o) {
    dfa_options r;
    dfa_options_default(&r);
    if (o) r = *o;
    return r;
}

uint32_t floor_log2(uint64_t x) {
    uint32_t l = 0;
    while (x > 1) {
        x >>= 1;
        ++l;
    }
    return l;
}

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Copy `words` uint32 from device to the pinned buffer and wait.
int read_back(Ctx &c, const void *dev, size_t bytes) {
    if (bytes > kPinnedWords * sizeof(uint32_t)) return fail(DFA_EINVAL, "readback too large");
    HIP_TRY(hipMemcpyAsync(c.pinned, dev, bytes, hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(stream_sync(c));
    return DFA_OK;
}

int upload(Ctx &c, void *dev, const void *host, size_t bytes) {
    if (bytes > kPinnedWords * sizeof(uint32_t)) return fail(DFA_EINVAL, "upload too large");
    // the pinned buffer may still be read by an earlier async copy
    HIP_TRY(stream_sync(c));
    std::memcpy(c.pinned, host, bytes);
    HIP_TRY(hipMemcpyAsync(dev, c.pinned, bytes, hipMemcpyHostToDevice, c.stream));
    HIP_TRY(stream_sync(c));
    return DFA_OK;
}

// ---- kernel timing ----

enum class Kern {
    Mark, Signature, Insert, SortGroup, RoundEnd, Pattern, Packed, LeaderElect, LeaderMove,
    LeaderEnd, PbGather, SignaturePb, SegPattern, PackedPb
};

int prof_event(Ctx &c, size_t &idx) {
    if (c.ev_used == c.evpool.size()) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        c.evpool.push_back(e);
    }
    idx = c.ev_used++;
    return DFA_OK;
}

// Algorithmic bytes per refined state of each round kernel (k = k_eff):
//   signature  4k (column entries) + 4 (own block id) + 4k (successor ids);
//              in rounds that gather through LDS slices the successor ids are
//              charged to the gather pass (4k) and the rest (4k + 4) to the
//              signature pass
//   insert     4 (the new block id)
//   pattern    4k (columns) + (k + 1) (acceptance of q and successors) + 4 (label);
//              the same for round 0 of a segmented refinement by patterns
//   packed     4k (columns) + (k + 1) (byte labels) + 4 (label)
//   elect      per compared (non-leader) state: 4k (own columns) + 4k (the
//              leader's columns) + 8k (the two successor ids per letter)
uint32_t kern_bytes(Kern kind, uint32_t k_eff) {
    switch (kind) {
        case Kern::Signature: return 8 * k_eff + 4;
        case Kern::PbGather: return 4 * k_eff;
        case Kern::SignaturePb: return 4 * k_eff + 4;
        case Kern::Insert: return 4;
        case Kern::Pattern:
        case Kern::Packed:
        case Kern::PackedPb:
        case Kern::SegPattern: return 5 * k_eff + 5;
        case Kern::LeaderElect: return 16 * k_eff;
        default: return 0;
    }
}

const char *kern_name(Kern kind) {
    switch (kind) {
        case Kern::Mark: return "k_mark";
        case Kern::Signature: return "k_signature";
        case Kern::Insert: return "k_insert";
        case Kern::SortGroup: return "sort_group";
        case Kern::RoundEnd: return "k_round_end";
        case Kern::Pattern: return "k_pattern_round";
        case Kern::Packed: return "k_packed_round";
        case Kern::LeaderElect: return "k_leader_elect";
        case Kern::LeaderMove: return "k_leader_move";
        case Kern::PbGather: return "k_pb_gather";
        case Kern::SegPattern: return "k_seg_pattern";
        case Kern::PackedPb: return "k_packed_pb";
        case Kern::SignaturePb: return "k_signature_pb";
        default: return "k_leader_end";
    }
}

// Launches one round kernel, bracketed by events when timing is on.
template <class Args>
int launch_kern(Ctx &c, Kern kind, const Args &a, uint32_t round) {
    size_t e0 = 0, e1 = 0;
    const bool timed = c.profiling && (c.prof_only.empty() || c.prof_only == kern_name(kind));
    if (timed) {
        DFA_TRY(prof_event(c, e0));
        HIP_TRY(hipEventRecord(c.evpool[e0], c.stream));
    }
    if constexpr (std::is_same_v<Args, RoundArgs>) {
        switch (kind) {
            case Kern::Mark: launch_mark(a, c.stream); break;
            case Kern::Signature: launch_signature(a, c.stream); break;
            case Kern::PbGather: launch_pb_gather(a, c.stream); break;
            case Kern::SegPattern: launch_seg_pattern(a, c.stream); break;
            case Kern::PackedPb: launch_packed_pb(a, c.stream); break;
            case Kern::SignaturePb: launch_signature_pb(a, c.stream); break;
            case Kern::Insert: launch_insert(a, c.stream); break;
            case Kern::SortGroup: launch_sort_group(a, c.stream); break;
            case Kern::RoundEnd: launch_round_end(a, c.stream); break;
            case Kern::Pattern: launch_pattern_kernel(a, c.stream); break;
            case Kern::Packed: launch_packed_kernel(a, c.stream); break;
            default: return fail(DFA_EDEVICE, "internal: leader kernel with round arguments");
        }
    } else {
        switch (kind) {
            case Kern::LeaderElect: launch_leader_elect(a, c.stream); break;
            case Kern::LeaderMove: launch_leader_move(a, c.stream); break;
            case Kern::LeaderEnd: launch_leader_end(a, c.stream); break;
            default: return fail(DFA_EDEVICE, "internal: round kernel with leader arguments");
        }
    }
    if (timed) {
        DFA_TRY(prof_event(c, e1));
        HIP_TRY(hipEventRecord(c.evpool[e1], c.stream));
        c.pending.push_back({kern_name(kind), e0, e1, round, kern_bytes(kind, a.k_eff), a.k_eff});
    }
    return DFA_OK;
}

int launch_full_round(Ctx &c, const RoundArgs &a, uint32_t round) {
    DFA_TRY(launch_kern(c, Kern::Mark, a, round));
    if (a.pb.nb) {
        DFA_TRY(launch_kern(c, Kern::PbGather, a, round));
        DFA_TRY(launch_kern(c, Kern::SignaturePb, a, round));
    }
    DFA_TRY(launch_kern(c, Kern::Signature, a, round));
    DFA_TRY(launch_kern(c, a.grouping ? Kern::SortGroup : Kern::Insert, a, round));
    if (a.seg.nseg) launch_seg_round(a, c.stream);
    return launch_kern(c, Kern::RoundEnd, a, round);
}

int launch_full_round(Ctx &c, const LeaderArgs &a, uint32_t round) {
    DFA_TRY(launch_kern(c, Kern::LeaderElect, a, round));
    DFA_TRY(launch_kern(c, Kern::LeaderMove, a, round));
    return launch_kern(c, Kern::LeaderEnd, a, round);
}

// Folds the timed launches into the totals (the stream has been synchronised).
int prof_collect(Ctx &c, const RoundCtl &ctl) {
    for (const auto &p : c.pending) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c.evpool[p.ev0], c.evpool[p.ev1]));
        auto &t = c.ktimes[p.name];
        t.launches += 1;
        t.ms += ms;
        // the signature kernel and the two slice passes stand in for each
        // other round by round: only the path the round took is charged
        const bool pb = ((ctl.pb_rounds >> (p.round % 64)) & 1ull) != 0;
        const bool sig = std::strcmp(p.name, "k_signature") == 0;
        const bool pass = std::strcmp(p.name, "k_pb_gather") == 0 ||
                          std::strcmp(p.name, "k_signature_pb") == 0;
        const bool did_work = !((sig && pb) || (pass && !pb));
        if (did_work && p.round < ctl.round && ctl.round - p.round <= kActiveHist) {
            const uint64_t refined = ctl.active_hist[p.round % kActiveHist];
            t.bytes += refined * p.bytes_per_state;
            t.states += refined;
            t.state_letters += refined * p.k_eff;
        }
    }
    c.pending.clear();
    c.ev_used = 0;
    return DFA_OK;
}

// flags layout (uint32 words): [0] target >= n, [1] some state accepts,
// [2] some state rejects, [3 .. 3+ncols) column is not the identity,
// [3+ncols .. 3+2*ncols) column differs from the previous closure level.
constexpr size_t kFlagErr = 0, kFlagClass = 1, kFlagNonid = 3;

struct RefineResult {
    RoundCtl ctl{};
    uint32_t label_rounds = 0;  // rounds 0..label_rounds-1 produced labels, not state ids
    uint32_t k_eff = 0;
    uint32_t tc_used = 0, tc_levels = 0, plain_rounds = 0;
    const uint32_t *final_block = nullptr;
    uint64_t transitions = 0, bytes = 0;
    uint32_t N = 0;  // states refined
};

// Whether plain rounds have stalled, after at least 8 rounds: over the last
// four rounds no round added more than 1/4096 of the states still to be
// separated (large inputs), or, after 16 rounds, no more than 1/64 of them
// (small ones, where the closure is cheap and the remaining rounds would
// each split a block or two).
bool splitting_stalled(const RoundCtl &ctl, size_t N) {
    if (ctl.round < 8) return false;
    const uint64_t left = N - ctl.prev_count;
    uint64_t recent_gain = 0;
    for (uint32_t i = 1; i <= 4 && i <= ctl.round; ++i)
        recent_gain = std::max<uint64_t>(recent_gain, ctl.gain_hist[(ctl.round - i) % kActiveHist]);
    return (left >= 4096 && recent_gain * 4096 < left) ||
           (ctl.round >= 16 && recent_gain * 64 < left);
}

// Rounds in the next chunk when the caller leaves the length to the library:
// the tuned start length, doubled after every chunk that did not finish, up
// to 256 rounds (8 while the closure may still be switched on, so that a
// stall is seen soon after it starts).  Short refinements keep few no-op
// rounds; long ones need few host round trips.
uint32_t grown_chunk(uint32_t chunk, bool tc_pending, bool profiling) {
    uint32_t cap = tc_pending ? 8u : 256u;
    if (profiling) cap = std::min(cap, kActiveHist);
    return std::max(chunk, std::min(chunk * 2, cap));
}

// Builds the closure columns (all levels) from level 0 in c.cols, and the
// signature column list.  Returns DFA_ENOMEM if the table does not fit.
int build_closure(Ctx &c, size_t N, uint32_t k, std::vector<uint32_t> &colmap, uint32_t &levels,
                  const unsigned long long *single = nullptr) {
    const uint32_t L = floor_log2(N);
    const size_t ncols = static_cast<size_t>(L + 1) * k;
    DFA_TRY(c.tc_cols.ensure(ncols * N * sizeof(uint32_t), "closure columns"));
    DFA_TRY(c.flags.ensure((kFlagNonid + 2 * ncols) * sizeof(uint32_t), "flags"));
    uint32_t *flags = c.flags.as<uint32_t>();
    uint32_t *nonid = flags + kFlagNonid;
    uint32_t *diff = nonid + ncols;
    HIP_TRY(hipMemcpyAsync(c.tc_cols.p, c.cols.p, static_cast<size_t>(k) * N * sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, c.stream));
    HIP_TRY(hipMemsetAsync(nonid + k, 0, (ncols - k) * sizeof(uint32_t), c.stream));
    HIP_TRY(hipMemsetAsync(diff, 0, ncols * sizeof(uint32_t), c.stream));
    for (uint32_t i = 1; i <= L; ++i)
        launch_jump(c.tc_cols.as<uint32_t>(), N, k, i, diff, nonid, c.stream);
    if (single) {
        // on demand, mid-refinement: only the states outside singleton
        // blocks are refined from here on, so the columns are judged on them
        HIP_TRY(hipMemsetAsync(nonid, 0, 2 * ncols * sizeof(uint32_t), c.stream));
        launch_column_flags(c.tc_cols.as<uint32_t>(), N, k, static_cast<uint32_t>(ncols), single,
                            diff, nonid, c.stream);
    }
    HIP_TRY(hipGetLastError());
    DFA_TRY(read_back(c, nonid, 2 * ncols * sizeof(uint32_t)));
    const uint32_t *h_nonid = c.pinned, *h_diff = c.pinned + ncols;
    colmap.clear();
    for (uint32_t i = 0; i <= L; ++i)
        for (uint32_t a = 0; a < k; ++a) {
            const size_t col = static_cast<size_t>(i) * k + a;
            // an identity letter repeats the leading block id; a level equal
            // to the previous one (and all above it) repeats that letter
            if (h_nonid[col] && (i == 0 || h_diff[col])) colmap.push_back(static_cast<uint32_t>(col));
        }
    levels = L;
    return DFA_OK;
}

// Judges the closure columns again on the states outside singleton blocks
// (only those are refined from now on) and keeps, of `colmap`, the columns
// that are not the identity there and differ from their letter's previous
// level there; a dropped column only repeats a key component on those states.
int rejudge_columns(Ctx &c, size_t N, uint32_t k, uint32_t levels,
                    const std::vector<uint32_t> &colmap, std::vector<uint32_t> &kept) {
    const size_t ncols = static_cast<size_t>(levels + 1) * k;
    uint32_t *nonid = c.flags.as<uint32_t>() + kFlagNonid;
    uint32_t *diff = nonid + ncols;
    HIP_TRY(hipMemsetAsync(nonid, 0, 2 * ncols * sizeof(uint32_t), c.stream));
    launch_column_flags(c.tc_cols.as<uint32_t>(), N, k, static_cast<uint32_t>(ncols),
                        c.single.as<unsigned long long>(), diff, nonid, c.stream);
    HIP_TRY(hipGetLastError());
    DFA_TRY(read_back(c, nonid, 2 * ncols * sizeof(uint32_t)));
    kept.clear();
    for (uint32_t col : colmap)
        if (c.pinned[col] && (col < k || c.pinned[ncols + col])) kept.push_back(col);
    return DFA_OK;
}

int set_colmap(Ctx &c, const std::vector<uint32_t> &colmap) {
    DFA_TRY(c.colmap.ensure(std::max<size_t>(colmap.size(), 1) * sizeof(uint32_t), "colmap"));
    // the list usually repeats from call to call: upload (a synchronous
    // copy) only when the device does not hold it already
    if (colmap.empty() ||
        (c.colmap.allocation == c.colmap_on_device_in && colmap == c.colmap_on_device))
        return DFA_OK;
    DFA_TRY(upload(c, c.colmap.p, colmap.data(), colmap.size() * sizeof(uint32_t)));
    c.colmap_on_device = colmap;
    c.colmap_on_device_in = c.colmap.allocation;
    return DFA_OK;
}

// Adds the first `bytes` of b (rounded up to 8) to a zeroing list.
int zero_add(ZeroList &z, Buffer &b, size_t bytes) {
    if (z.count >= kZeroRegions) return fail(DFA_EDEVICE, "internal: zeroing list is full");
    z.p[z.count] = b.as<unsigned long long>();
    z.words[z.count] = (bytes + 7) / 8;
    ++z.count;
    return DFA_OK;
}

// Builds `rounds` rounds into an executable graph, node by node (the launch
// helpers append kernel nodes while a recorder is set on this thread), so no
// stream is captured and no other thread's call can disturb the build.
int build_round_graph(const RoundArgs &ra, const LeaderArgs *la, uint32_t rounds,
                      hipGraphExec_t &out) {
    out = nullptr;
    GraphRecorder rec;
    HIP_TRY(hipGraphCreate(&rec.graph, 0));
    {
        struct Recording {
            explicit Recording(GraphRecorder *r) { graph_recorder() = r; }
            ~Recording() { graph_recorder() = nullptr; }
        } recording(&rec);
        for (uint32_t i = 0; i < rounds && rec.error == hipSuccess; ++i) {
            if (la)
                launch_leader_round(*la, nullptr);
            else
                launch_round(ra, nullptr);
        }
    }
    hipError_t e = rec.error;
    if (e == hipSuccess) e = hipGraphInstantiate(&out, rec.graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(rec.graph);
    if (e != hipSuccess) {
        out = nullptr;
        return fail(DFA_EDEVICE, "building the round graph: %s", hipGetErrorString(e));
    }
    return DFA_OK;
}

// Enqueues `rounds` rounds of signature (ra) or leader (la != nullptr)
// refinement, from a graph in GRAPH mode.
int run_chunk(Ctx &c, const RoundArgs &ra, uint32_t rounds, int mode, uint32_t first_round,
              const LeaderArgs *la = nullptr) {
    if (mode == DFA_LOOP_PERSISTENT && !c.profiling) {
        const hipError_t e = la ? launch_leader_persistent(*la, rounds, c.stream)
                                : launch_rounds_persistent(ra, rounds, c.stream);
        if (e != hipSuccess)
            return fail(DFA_EDEVICE, "persistent round loop: %s", hipGetErrorString(e));
        return DFA_OK;
    }
    if (mode == DFA_LOOP_GRAPH && !c.profiling) {
        GraphKey key;
        std::memset(&key, 0, sizeof key);
        if (la)
            std::memcpy(&key.largs, la, sizeof *la);
        else
            std::memcpy(&key.args, &ra, sizeof ra);
        key.chunk = rounds;
        key.leader = la ? 1u : 0u;
        int slot = -1;
        for (int i = 0; i < Ctx::kGraphSlots; ++i)
            if (c.graphs[i] && c.graph_keys[i] == key) slot = i;
        if (slot < 0) {
            slot = c.graph_victim;
            c.graph_victim = (c.graph_victim + 1) % Ctx::kGraphSlots;
            if (c.graphs[slot]) {
                (void)hipGraphExecDestroy(c.graphs[slot]);
                c.graphs[slot] = nullptr;
            }
            DFA_TRY(build_round_graph(ra, la, rounds, c.graphs[slot]));
            c.graph_keys[slot] = key;
        }
        HIP_TRY(hipGraphLaunch(c.graphs[slot], c.stream));
    } else {
        for (uint32_t i = 0; i < rounds; ++i) {
            if (la)
                DFA_TRY(launch_full_round(c, *la, first_round + i));
            else
                DFA_TRY(launch_full_round(c, ra, first_round + i));
        }
        HIP_TRY(hipGetLastError());
    }
    return DFA_OK;
}

// Signature rounds over N states whose level-0 columns are in c.cols and
// whose initial labels are in c.blockA (flags already written by the ingest
// and init kernels).
RoundArgs make_round_args(Ctx &c, const uint32_t *cols, size_t N, uint32_t k_eff, uint64_t cap,
                          int lds_stage, bool packed, const SegArgs *seg, uint32_t grouping) {
    RoundArgs ra;
    std::memset(&ra, 0, sizeof ra);
    if (seg) ra.seg = *seg;
    ra.cols = cols;
    ra.colmap = c.colmap.as<uint32_t>();
    ra.N = N;
    ra.k_eff = k_eff;
    ra.blockA = c.blockA.as<uint32_t>();
    ra.blockB = c.blockB.as<uint32_t>();
    ra.sig = c.sig.as<uint32_t>();
    ra.hash = c.hash.as<uint64_t>();
    ra.table = c.table.as<unsigned long long>();
    ra.table_cap = cap;
    ra.multi = c.multi.as<uint32_t>();
    ra.active = c.active.as<unsigned long long>();
    ra.accbits = c.accbits.as<unsigned long long>();
    ra.counters = c.counters.as<uint32_t>();
    ra.presence = c.presence.as<uint32_t>();
    ra.presence_packed = packed ? c.presence_packed.as<uint32_t>() : nullptr;
    ra.lab8 = packed ? c.lab8.as<uint8_t>() : nullptr;
    ra.ctl = c.ctl.as<RoundCtl>();
    ra.lds_stage = lds_stage;
    ra.round_grid_cap = c.tune.round_grid_cap;
    ra.pattern_grid_cap = c.tune.label_grid_cap;
    ra.cached_probe = c.tune.cached_probe;
    ra.insert_pair = c.tune.insert_pair;
    ra.chg = c.chg.as<unsigned long long>();
    ra.chg_sum = c.chg_sum.as<unsigned long long>();
    ra.single = c.single.as<unsigned long long>();
    ra.touched = c.touched.as<unsigned long long>();
    ra.grouping = grouping;
    ra.hash_bits = c.tune.hash_bits;
    if (grouping) {
        ra.sort.keys[0] = c.sort_keys0.as<unsigned long long>();
        ra.sort.keys[1] = c.sort_keys1.as<unsigned long long>();
        ra.sort.vals[0] = c.sort_vals0.as<uint32_t>();
        ra.sort.vals[1] = c.sort_vals1.as<uint32_t>();
        ra.sort.hist = c.sort_hist.as<uint32_t>();
        ra.sort.partials = c.sort_partials.as<uint32_t>();
        ra.sort.runhead = c.sort_runhead.as<uint32_t>();
        ra.sort.m = c.sort_m.as<uint32_t>();
    }
    return ra;
}

// Signature rounds over N states whose level-0 columns are in c.cols and
// whose initial labels are in c.blockA (flags already written by the ingest
// and init kernels).  With state_ids, a partition that ends in label ids
// (a stable partition found by a label round) gets one more table round,
// which keeps the partition and turns the labels into state ids.
// Buckets the edges by target slice when the refinement is large enough for
// dense rounds to gain from gathering through LDS (dfa_tuning.slice_min_states)
// and its signature width has a specialised kernel; pb.nb == 0 otherwise.
// Not for segmented refinements, closure columns or the persistent loop.
int build_slices(Ctx &c, const uint32_t *cols, size_t N, uint32_t k_eff, const dfa_options &o,
                 bool excluded, PbArgs &pb) {
    pb = PbArgs{};
    const bool width = k_eff >= 1 && (k_eff <= 8 || k_eff == 16);
    if (excluded || !width || o.loop_mode == DFA_LOOP_PERSISTENT || !c.tune.slice_min_states ||
        N < c.tune.slice_min_states || N > (static_cast<size_t>(kPbMaxBuckets) << kPbSliceLog))
        return DFA_OK;
    const uint32_t nb = static_cast<uint32_t>((N + (1u << kPbSliceLog) - 1) >> kPbSliceLog);
    const uint32_t ntiles = static_cast<uint32_t>((N + kPbTile - 1) / kPbTile);
    const size_t E = N * k_eff;
    const uint64_t L = static_cast<uint64_t>(nb) * ntiles;
    DFA_TRY(c.pb_tl.ensure(E * sizeof(uint16_t), "slice targets"));
    DFA_TRY(c.pb_src.ensure(E * sizeof(uint16_t), "slice sources"));
    DFA_TRY(c.pb_val.ensure(E * sizeof(uint32_t), "slice values"));
    // run lengths and starts, bucket starts; then the scan's chunk sums and
    // bucket totals
    DFA_TRY(c.pb_off.ensure((2 * L + nb + 1) * sizeof(uint32_t), "slice runs"));
    DFA_TRY(c.pb_partials.ensure((pb_chunk_words(nb, ntiles) + nb) * sizeof(uint32_t),
                                 "slice scan"));
    pb.tl = c.pb_tl.as<uint16_t>();
    pb.src = c.pb_src.as<uint16_t>();
    pb.val = c.pb_val.as<uint32_t>();
    pb.cnt = c.pb_off.as<uint32_t>();
    pb.off = pb.cnt + L;
    pb.bstart = pb.off + L;
    pb.nb = nb;
    pb.ntiles = ntiles;
    uint32_t *csum = c.pb_partials.as<uint32_t>();
    launch_pb_build(cols, c.colmap.as<uint32_t>(), N, k_eff, pb, csum,
                    csum + pb_chunk_words(nb, ntiles), c.stream);
    HIP_TRY(hipGetLastError());
    return DFA_OK;
}

int refine(Ctx &c, size_t N, uint32_t k, const dfa_options &o, uint32_t check_eq, uint32_t eq_a,
           uint32_t eq_b, bool state_ids, RefineResult &res, const SegArgs *seg = nullptr) {
    res.N = static_cast<uint32_t>(N);
    // state that starts empty, cleared in one launch queued before the
    // readback below, so that the device clears while the host waits
    const uint64_t cap = next_pow2(std::max<uint64_t>(2 * N, 1024));
    const size_t words64 = (N + 63) / 64;
    const size_t sum_words = summary_words(N);
    DFA_TRY(c.table.ensure(cap * sizeof(unsigned long long), "hash table"));
    DFA_TRY(c.chg.ensure(words64 * sizeof(unsigned long long), "changed-id bits"));
    DFA_TRY(c.single.ensure(words64 * sizeof(unsigned long long), "singleton bits"));
    DFA_TRY(c.touched.ensure(2 * words64 * sizeof(unsigned long long), "touched-block bits"));
    DFA_TRY(c.chg_sum.ensure(2 * sum_words * sizeof(unsigned long long), "changed-wave summary"));
    // label rounds: the packed-label map too when k letters could use it
    // (identity letters, known after the readback, only make k_eff smaller)
    const bool packed_possible = !seg && (k + 1) * (k + 1) <= kPackedMaxBits;
    if (packed_possible)
        DFA_TRY(c.presence_packed.ensure(kLabelMapBytes, "label map"));
    {
        ZeroList z{};
        DFA_TRY(zero_add(z, c.table, cap * sizeof(unsigned long long)));
        DFA_TRY(zero_add(z, c.single, words64 * sizeof(unsigned long long)));
        DFA_TRY(zero_add(z, c.touched, 2 * words64 * sizeof(unsigned long long)));
        DFA_TRY(zero_add(z, c.chg_sum, 2 * sum_words * sizeof(unsigned long long)));
        if (packed_possible)
            DFA_TRY(zero_add(z, c.presence_packed, kLabelMapBytes));
        launch_zero(z, c.stream);
        HIP_TRY(hipGetLastError());
    }
    // target check, classes, identity letters (one readback)
    DFA_TRY(read_back(c, c.flags.p, (kFlagNonid + k) * sizeof(uint32_t)));
    if (c.pinned[kFlagErr]) return fail(DFA_EINVAL, "a transition target is >= n");
    std::vector<uint32_t> colmap;
    for (uint32_t a = 0; a < k; ++a)
        if (c.pinned[kFlagNonid + a]) colmap.push_back(a);

    DFA_TRY(c.ctl.ensure(sizeof(RoundCtl), "round state"));
    RoundCtl *ctl = c.ctl.as<RoundCtl>();

    const uint32_t *cols = c.cols.as<uint32_t>();
    res.tc_used = 0;
    res.tc_levels = 0;
    if (o.tc_mode == DFA_TC_ON) {
        DFA_TRY(build_closure(c, N, k, colmap, res.tc_levels));
        cols = c.tc_cols.as<uint32_t>();
        res.tc_used = 1;
    }
    DFA_TRY(set_colmap(c, colmap));
    uint32_t k_eff = static_cast<uint32_t>(colmap.size());
    // closure columns are judged once more on the states outside singleton
    // blocks: built first (tc ON), once a quarter of the states are
    // singletons; built on demand, after the first chunk on the new columns
    // (singleton marks lag a round behind the splits)
    bool rejudged = false;
    uint32_t switched_at = 0;
    DFA_TRY(c.sig.ensure(N * (k_eff + 1) * sizeof(uint32_t), "signatures"));
    DFA_TRY(c.hash.ensure(N * sizeof(uint64_t), "hashes"));
    const uint32_t grouping = (o.algorithm == DFA_ALGO_SORT && !seg) ? 1u : 0u;
    // edges bucketed by target slice, for the dense rounds of the first chunk
    PbArgs pb{};
    DFA_TRY(build_slices(c, cols, N, k_eff, o, seg != nullptr || res.tc_used, pb));
    if (grouping) {
        const SortPlan pl = sort_plan(N);
        DFA_TRY(c.sort_keys0.ensure(N * sizeof(unsigned long long), "sort keys"));
        DFA_TRY(c.sort_keys1.ensure(N * sizeof(unsigned long long), "sort keys"));
        DFA_TRY(c.sort_vals0.ensure(N * sizeof(uint32_t), "sort values"));
        DFA_TRY(c.sort_vals1.ensure(N * sizeof(uint32_t), "sort values"));
        DFA_TRY(c.sort_hist.ensure(pl.hist_words * sizeof(uint32_t), "digit counts"));
        DFA_TRY(c.sort_partials.ensure(pl.partial_words * sizeof(uint32_t), "scan partials"));
        DFA_TRY(c.sort_runhead.ensure(N * sizeof(uint32_t), "run heads"));
        DFA_TRY(c.sort_m.ensure(sizeof(uint32_t), "sort count"));
    }
    // label rounds need at least three rounds of budget (ids become state
    // ids in the round after them)
    // (segmented refinements keep their segment labels: no label rounds)
    const bool budget = (o.max_rounds == 0 || o.max_rounds > 2) && !seg;
    const uint32_t pattern_first =
        (c.tune.label_rounds >= 1 && budget && k_eff + 1 <= kPatternMaxBits) ? 1u : 0u;
    const uint32_t packed_second =
        (pattern_first && c.tune.label_rounds >= 2 && (k_eff + 1) * (k_eff + 1) <= kPackedMaxBits)
            ? 1u
            : 0u;
    if (packed_second) {
        DFA_TRY(c.lab8.ensure(N, "byte labels"));
        if (!packed_possible) {  // not cleared above
            DFA_TRY(c.presence_packed.ensure(kLabelMapBytes, "label map"));
            HIP_TRY(hipMemsetAsync(c.presence_packed.p, 0, kLabelMapBytes,
                                   c.stream));
        }
    }
    res.label_rounds = pattern_first + packed_second;
    // segmented refinements: round 0 by acceptance patterns when the keys of
    // all segments fit the pattern table
    const uint32_t segpat_bits = k_eff + 1;
    const bool segpat = seg && c.tune.label_rounds >= 1 && !grouping && !res.tc_used &&
                        segpat_bits <= kSegPatMaxBits &&
                        (static_cast<uint64_t>(seg->nseg) << segpat_bits) <= kSegPatMaxWords;
    if (segpat) {
        DFA_TRY(c.segpat_table.ensure((static_cast<size_t>(seg->nseg) << segpat_bits) *
                                          sizeof(uint32_t),
                                      "pattern table"));
        DFA_TRY(c.segpat.ensure(N * sizeof(uint16_t), "patterns"));
    }
    launch_ctl_reset(ctl, c.flags.as<uint32_t>() + kFlagClass, o.max_rounds, check_eq, eq_a, eq_b,
                     pattern_first, packed_second, seg ? seg->init_count : nullptr, c.stream);

    const int mode = o.loop_mode;
    uint32_t chunk = o.chunk ? o.chunk : c.tune.chunk;
    if (c.profiling) chunk = std::min(chunk, kActiveHist);
    uint32_t last_round = 0;
    unsigned long long last_active_sum = 0;
    bool tc_failed = false;
    res.transitions = 0;
    res.bytes = 0;
    bool first = true;
    bool first_chunk = true;
    for (;;) {
        RoundArgs ra = make_round_args(c, cols, N, k_eff, cap, o.lds_stage, packed_second, seg, grouping);
        // the dense rounds come first (the first table rounds); later chunks
        // gather directly, so a long refinement pays nothing for the passes
        if (first_chunk) ra.pb = pb;
        if (segpat && first) {
            ra.segpat_table = c.segpat_table.as<uint32_t>();
            ra.segpat = c.segpat.as<uint16_t>();
            ra.segpat_bits = segpat_bits;
        }
        if (first) {
            // rounds 0 (and 1) run on their own: label rounds when the
            // signatures are short enough
            if (pattern_first) {
                DFA_TRY(launch_kern(c, Kern::Pattern, ra, 0));
                DFA_TRY(launch_kern(c, Kern::RoundEnd, ra, 0));
            } else if (ra.segpat_bits) {
                DFA_TRY(launch_kern(c, Kern::Mark, ra, 0));
                DFA_TRY(launch_kern(c, Kern::SegPattern, ra, 0));
                launch_seg_round(ra, c.stream);
                DFA_TRY(launch_kern(c, Kern::RoundEnd, ra, 0));
            } else {
                DFA_TRY(launch_full_round(c, ra, 0));
            }
            if (packed_second) {
                // through the slices when the edges are bucketed (k_eff <= 4)
                DFA_TRY(launch_kern(c, ra.pb.nb ? Kern::PackedPb : Kern::Packed, ra, 1));
                DFA_TRY(launch_kern(c, Kern::RoundEnd, ra, 1));
            }
            HIP_TRY(hipGetLastError());
            first = false;
        }
        // rounds launched so far: the label rounds, then last_round onwards
        const uint32_t next_round = std::max(last_round, res.label_rounds ? res.label_rounds : 1u);
        DFA_TRY(run_chunk(c, ra, mode == DFA_LOOP_HOST ? 1u : chunk, mode, next_round));
        first_chunk = false;
        DFA_TRY(read_back(c, ctl, sizeof(RoundCtl)));
        std::memcpy(&res.ctl, c.pinned, sizeof(RoundCtl));
        if (c.profiling) DFA_TRY(prof_collect(c, res.ctl));
        const uint32_t done_rounds = res.ctl.round - last_round;
        res.transitions += static_cast<uint64_t>(done_rounds) * N * k_eff;
        res.bytes += (res.ctl.active_sum - last_active_sum) * (8ull * k_eff + 8ull);
        last_round = res.ctl.round;
        last_active_sum = res.ctl.active_sum;
        if (res.ctl.done) break;
        // closure on demand: splitting has stalled (the chain-like regime
        // where plain rounds each split only a few blocks)
        if (o.tc_mode == DFA_TC_AUTO && !seg && !res.tc_used && !tc_failed &&
            splitting_stalled(res.ctl, N)) {
            std::vector<uint32_t> tcmap;
            uint32_t levels = 0;
            int rc = build_closure(c, N, k, tcmap, levels, c.single.as<unsigned long long>());
            if (rc == DFA_ENOMEM) {  // stay on the plain letters
                tc_failed = true;
                g_last_error.clear();
                continue;
            }
            DFA_TRY(rc);
            DFA_TRY(set_colmap(c, tcmap));
            colmap = tcmap;
            switched_at = res.ctl.round;
            k_eff = static_cast<uint32_t>(tcmap.size());
            DFA_TRY(c.sig.ensure(N * (k_eff + 1) * sizeof(uint32_t), "signatures"));
            // new letters: the next round refines every multi-state block
            launch_ctl_full(ctl, c.stream);
            cols = c.tc_cols.as<uint32_t>();
            res.tc_used = 1;
            res.tc_levels = levels;
            res.plain_rounds = res.ctl.round;
        }
        // the closure's columns judged again on the states outside singleton
        // blocks (see above)
        if (res.tc_used && !rejudged && !seg &&
            (switched_at ? res.ctl.round > switched_at : res.ctl.prev_count >= N / 4)) {
            rejudged = true;
            std::vector<uint32_t> kept;
            DFA_TRY(rejudge_columns(c, N, k, res.tc_levels, colmap, kept));
            if (!kept.empty() && kept.size() < colmap.size()) {
                colmap = kept;
                DFA_TRY(set_colmap(c, colmap));
                k_eff = static_cast<uint32_t>(colmap.size());
            }
        }
        if (!o.chunk)
            chunk = grown_chunk(chunk, o.tc_mode == DFA_TC_AUTO && !seg && !res.tc_used && !tc_failed,
                                c.profiling);
    }
    res.k_eff = k_eff;
    uint32_t rounds_run = res.ctl.round;
    if (state_ids && res.ctl.stable && res.ctl.round <= res.label_rounds) {
        launch_ctl_resume(ctl, c.stream);
        DFA_TRY(launch_full_round(c, make_round_args(c, cols, N, k_eff, cap, o.lds_stage,
                                                     packed_second, seg, grouping),
                                  res.ctl.round));
        HIP_TRY(hipGetLastError());
        DFA_TRY(read_back(c, ctl, sizeof(RoundCtl)));
        const RoundCtl *after = reinterpret_cast<const RoundCtl *>(c.pinned);
        if (c.profiling) DFA_TRY(prof_collect(c, *after));
        if (!after->stable || after->prev_count != res.ctl.prev_count)
            return fail(DFA_EDEVICE, "internal: relabelling round changed the partition");
        rounds_run = after->round;
    }
    const uint32_t r_last = rounds_run - 1;
    res.final_block = (r_last & 1u) ? c.blockA.as<uint32_t>() : c.blockB.as<uint32_t>();
    return DFA_OK;
}

// Leader rounds (naivePR) over N states whose level-0 columns are in c.cols
// and whose acceptance bits are in c.accbits (flags written by the ingest
// and init kernels).  Block ids are leaders, i.e. state ids, throughout; the
// result is in c.blockA.
int refine_leader(Ctx &c, size_t N, uint32_t k, const dfa_options &o, uint32_t check_eq,
                  uint32_t eq_a, uint32_t eq_b, RefineResult &res) {
    res.N = static_cast<uint32_t>(N);
    DFA_TRY(read_back(c, c.flags.p, (kFlagNonid + k) * sizeof(uint32_t)));
    if (c.pinned[kFlagErr]) return fail(DFA_EINVAL, "a transition target is >= n");
    std::vector<uint32_t> colmap;
    // an identity letter never separates a state from its leader
    for (uint32_t a = 0; a < k; ++a)
        if (c.pinned[kFlagNonid + a]) colmap.push_back(a);
    DFA_TRY(c.ctl.ensure(sizeof(RoundCtl), "round state"));
    RoundCtl *ctl = c.ctl.as<RoundCtl>();
    const uint32_t *cols = c.cols.as<uint32_t>();
    res.tc_used = 0;
    res.tc_levels = 0;
    res.label_rounds = 0;
    if (o.tc_mode == DFA_TC_ON) {
        DFA_TRY(build_closure(c, N, k, colmap, res.tc_levels));
        cols = c.tc_cols.as<uint32_t>();
        res.tc_used = 1;
    }
    DFA_TRY(set_colmap(c, colmap));
    uint32_t k_eff = static_cast<uint32_t>(colmap.size());
    DFA_TRY(c.new_leader.ensure(N * sizeof(unsigned long long), "leader slots"));
    DFA_TRY(c.moved.ensure((N + 63) / 64 * sizeof(unsigned long long), "separation masks"));
    DFA_TRY(c.scalars.ensure(16 * sizeof(uint32_t), "scalars"));
    HIP_TRY(hipMemsetAsync(c.new_leader.p, 0xFF, N * sizeof(unsigned long long), c.stream));
    HIP_TRY(hipMemsetD32Async(c.scalars.as<uint32_t>(), 0xFFFFFFFFu, 2, c.stream));
    launch_leader_init(c.accbits.as<unsigned long long>(), N, c.scalars.as<uint32_t>(),
                       c.blockA.as<uint32_t>(), c.stream);
    launch_ctl_reset(ctl, c.flags.as<uint32_t>() + kFlagClass, o.max_rounds, check_eq, eq_a, eq_b,
                     0, 0, nullptr, c.stream);
    HIP_TRY(hipGetLastError());

    const int mode = o.loop_mode;
    uint32_t chunk = o.chunk ? o.chunk : c.tune.chunk;
    if (c.profiling) chunk = std::min(chunk, kActiveHist);
    uint32_t last_round = 0;
    unsigned long long last_active_sum = 0;
    bool tc_failed = false;
    res.transitions = 0;
    res.bytes = 0;
    RoundArgs none;
    std::memset(&none, 0, sizeof none);
    for (;;) {
        LeaderArgs la;
        std::memset(&la, 0, sizeof la);
        la.cols = cols;
        la.colmap = c.colmap.as<uint32_t>();
        la.N = N;
        la.k_eff = k_eff;
        la.block = c.blockA.as<uint32_t>();
        la.new_leader = c.new_leader.as<unsigned long long>();
        la.moved = c.moved.as<unsigned long long>();
        la.counters = c.counters.as<uint32_t>();
        la.ctl = ctl;
        DFA_TRY(run_chunk(c, none, mode == DFA_LOOP_HOST ? 1u : chunk, mode, last_round, &la));
        DFA_TRY(read_back(c, ctl, sizeof(RoundCtl)));
        std::memcpy(&res.ctl, c.pinned, sizeof(RoundCtl));
        if (c.profiling) DFA_TRY(prof_collect(c, res.ctl));
        const uint32_t done_rounds = res.ctl.round - last_round;
        res.transitions += static_cast<uint64_t>(done_rounds) * N * k_eff;
        res.bytes += static_cast<uint64_t>(done_rounds) * N * 4 +
                     (res.ctl.active_sum - last_active_sum) * (16ull * k_eff);
        last_round = res.ctl.round;
        last_active_sum = res.ctl.active_sum;
        if (res.ctl.done) break;
        // closure on demand, by the rule of the signature rounds
        if (o.tc_mode == DFA_TC_AUTO && !res.tc_used && !tc_failed &&
            splitting_stalled(res.ctl, N)) {
            std::vector<uint32_t> tcmap;
            uint32_t levels = 0;
            int rc = build_closure(c, N, k, tcmap, levels);
            if (rc == DFA_ENOMEM) {
                tc_failed = true;
                g_last_error.clear();
                continue;
            }
            DFA_TRY(rc);
            DFA_TRY(set_colmap(c, tcmap));
            k_eff = static_cast<uint32_t>(tcmap.size());
            cols = c.tc_cols.as<uint32_t>();
            res.tc_used = 1;
            res.tc_levels = levels;
            res.plain_rounds = res.ctl.round;
        }
        if (!o.chunk)
            chunk = grown_chunk(chunk, o.tc_mode == DFA_TC_AUTO && !res.tc_used && !tc_failed,
                                c.profiling);
    }
    res.k_eff = k_eff;
    res.final_block = c.blockA.as<uint32_t>();
    return DFA_OK;
}

// Dispatch on the refinement algorithm of the options.
int refine_any(Ctx &c, size_t N, uint32_t k, const dfa_options &o, uint32_t check_eq,
               uint32_t eq_a, uint32_t eq_b, bool state_ids, RefineResult &res) {
    if (o.algorithm == DFA_ALGO_LEADER) return refine_leader(c, N, k, o, check_eq, eq_a, eq_b, res);
    return refine(c, N, k, o, check_eq, eq_a, eq_b, state_ids, res);
}

void fill_stats(dfa_stats *st, const RefineResult &r) {
    if (!st) return;
    st->rounds = r.ctl.round;
    st->changing_rounds = r.ctl.changing;
    st->num_blocks = r.ctl.prev_count;
    st->k_eff = r.k_eff;
    st->tc_used = r.tc_used;
    st->tc_levels = r.tc_levels;
    st->plain_rounds = r.tc_used ? r.plain_rounds : r.ctl.round;
    st->transitions_refined = r.transitions;
    st->algorithmic_bytes = r.bytes;
    st->reachable = r.N;
}

int check_options(const dfa_options &o) {
    if (o.tc_mode < DFA_TC_OFF || o.tc_mode > DFA_TC_AUTO) return fail(DFA_EINVAL, "bad tc_mode");
    if (o.loop_mode < DFA_LOOP_HOST || o.loop_mode > DFA_LOOP_PERSISTENT)
        return fail(DFA_EINVAL, "bad loop_mode");
    if (o.lds_stage < 0 || o.lds_stage > 2) return fail(DFA_EINVAL, "bad lds_stage");
    if (o.algorithm != DFA_ALGO_SIGNATURE && o.algorithm != DFA_ALGO_LEADER &&
        o.algorithm != DFA_ALGO_SORT)
        return fail(DFA_EINVAL, "bad algorithm");
    if (o.prune != 0 && o.prune != 1) return fail(DFA_EINVAL, "bad prune");
    if (o.equiv_method != DFA_EQ_UNION && o.equiv_method != DFA_EQ_PRODUCT)
        return fail(DFA_EINVAL, "bad equiv_method");
    if (o.loop_mode == DFA_LOOP_PERSISTENT && o.algorithm == DFA_ALGO_SORT)
        return fail(DFA_EINVAL, "the persistent loop groups with the hash table (not with sort)");
    return DFA_OK;
}

int check_batch_options(const dfa_options &o) {
    DFA_TRY(check_options(o));
    if (o.algorithm != DFA_ALGO_SIGNATURE)
        return fail(DFA_EINVAL, "batched calls run signature rounds only");
    if (o.prune) return fail(DFA_EINVAL, "batched calls partition every state (prune = 0)");
    if (o.equiv_method != DFA_EQ_UNION)
        return fail(DFA_EINVAL, "batched equivalence refines unions (equiv_method = DFA_EQ_UNION)");
    return DFA_OK;
}

int prepare_refinement(Ctx &c, size_t N, uint32_t k) {
    const uint32_t L = floor_log2(N);
    const size_t ncols = static_cast<size_t>(L + 1) * k;
    const size_t words64 = (N + 63) / 64;
    DFA_TRY(c.cols.ensure(static_cast<size_t>(k) * N * sizeof(uint32_t), "columns"));
    DFA_TRY(c.flags.ensure((kFlagNonid + 2 * ncols + 2) * sizeof(uint32_t), "flags"));
    DFA_TRY(c.blockA.ensure(N * sizeof(uint32_t), "blocks"));
    DFA_TRY(c.blockB.ensure(N * sizeof(uint32_t), "blocks"));
    DFA_TRY(c.multi.ensure((N + 1) * sizeof(uint32_t), "block marks"));
    DFA_TRY(c.active.ensure(words64 * sizeof(unsigned long long), "active masks"));
    DFA_TRY(c.accbits.ensure(words64 * sizeof(unsigned long long), "acceptance bits"));
    DFA_TRY(c.counters.ensure(kSpread * kSpreadStride * sizeof(uint32_t) + 8, "counters"));
    DFA_TRY(c.presence.ensure((1u << kPatternMaxBits) / 8, "pattern bitmap"));
    // every clear in one launch (separate memsets cost host time each)
    ZeroList z{};
    DFA_TRY(zero_add(z, c.flags, (kFlagNonid + k) * sizeof(uint32_t)));
    DFA_TRY(zero_add(z, c.multi, N * sizeof(uint32_t)));
    DFA_TRY(zero_add(z, c.accbits, words64 * sizeof(unsigned long long)));
    DFA_TRY(zero_add(z, c.counters, kSpread * kSpreadStride * sizeof(uint32_t)));
    DFA_TRY(zero_add(z, c.presence, (1u << kPatternMaxBits) / 8));
    launch_zero(z, c.stream);
    HIP_TRY(hipGetLastError());
    return DFA_OK;
}

int minimise_pruned(Ctx &c, uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *acc,
                    uint32_t *block_out, dfa_quotient *q, const dfa_options &o, dfa_stats *st);

int minimise_impl(Ctx &c, uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *acc,
                  uint32_t *block_out, dfa_quotient *q, const dfa_options &o, dfa_stats *st) {
    if (o.prune) return minimise_pruned(c, n, k, delta, acc, block_out, q, o, st);
    DFA_TRY(prepare_refinement(c, n, k));
    const size_t id_range = n;  // refine() returns state ids
    DFA_TRY(c.canon.ensure(id_range * sizeof(uint32_t), "canonical ids"));
    // (a context without events, the allocation-free one, times on the host)
    if (c.ev_start) HIP_TRY(hipEventRecord(c.ev_start, c.stream));
    uint32_t *flags = c.flags.as<uint32_t>();
    launch_ingest(delta, n, k, c.cols.as<uint32_t>(), n, 0, 0, flags + kFlagErr, flags + kFlagNonid,
                  c.stream);
    launch_init_blocks(acc, n, 0, c.blockA.as<uint32_t>(), c.accbits.as<unsigned long long>(),
                       flags + kFlagClass, c.stream);
    HIP_TRY(hipGetLastError());
    RefineResult r;
    int rc = refine_any(c, n, k, o, 0, 0, 0, true, r);
    if (rc != DFA_OK) return rc;
    launch_canonicalise(r.final_block, n, id_range, c.canon.as<uint32_t>(), block_out, c.stream);
    if (q) {
        DFA_TRY(c.scalars.ensure(16 * sizeof(uint32_t), "scalars"));
        uint32_t *sc = c.scalars.as<uint32_t>();
        if (r.ctl.prev_count == n) {
            // every block is one state: the quotient is the input itself
            HIP_TRY(hipMemsetD32Async(sc, n, 1, c.stream));
            launch_quotient_identity(delta, acc, n, k, o.start, q->delta, q->accepting, sc + 1,
                                     c.stream);
        } else {
            const size_t ntiles = (static_cast<size_t>(n) + kScanTile - 1) / kScanTile;
            DFA_TRY(c.partials.ensure((ntiles + 1) * sizeof(uint32_t), "scan partials"));
            DFA_TRY(c.dense.ensure(static_cast<size_t>(n) * sizeof(uint32_t), "dense ids"));
            DFA_TRY(c.leader_of.ensure(static_cast<size_t>(n) * sizeof(uint32_t), "leaders"));
            launch_dense_leaders(block_out, n, c.partials.as<uint32_t>(), c.dense.as<uint32_t>(),
                                 c.leader_of.as<uint32_t>(), sc, c.stream);
            // the canonicalisation scratch is free again: it holds dq
            launch_quotient(delta, acc, k, block_out, c.dense.as<uint32_t>(),
                            c.leader_of.as<uint32_t>(), sc, n, o.start, c.canon.as<uint32_t>(),
                            q->delta, q->accepting, sc + 1, c.stream);
        }
        HIP_TRY(hipGetLastError());
    }
    if (c.ev_stop) HIP_TRY(hipEventRecord(c.ev_stop, c.stream));
    if (q) {
        DFA_TRY(read_back(c, c.scalars.p, 2 * sizeof(uint32_t)));
        q->num_blocks = c.pinned[0];
        q->start = c.pinned[1];
    } else {
        HIP_TRY(stream_sync(c));
    }
    if (r.ctl.limit) {
        fill_stats(st, r);
        return fail(DFA_ELIMIT, "max_rounds (%u) reached before the partition was stable",
                    o.max_rounds);
    }
    if (st) {
        fill_stats(st, r);
        if (c.ev_start && c.ev_stop) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, c.ev_start, c.ev_stop));
            st->device_ms = ms;
        }
    }
    return DFA_OK;
}

// Minimisation of the part reachable from o.start: breadth-first search,
// dense renumbering of the reachable states (in increasing order), the
// sub-automaton, its minimisation, and the ids mapped back (smallest
// reachable member of each block; DFA_UNREACHABLE elsewhere).
int minimise_pruned(Ctx &c, uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *acc,
                    uint32_t *block_out, dfa_quotient *q, const dfa_options &o, dfa_stats *st) {
    if (o.start >= n) return fail(DFA_EINVAL, "start (%u) >= n (%u)", o.start, n);
    const size_t words64 = (static_cast<size_t>(n) + 63) / 64;
    const size_t ntiles = (static_cast<size_t>(n) + kScanTile - 1) / kScanTile;
    DFA_TRY(c.flags.ensure(4 * sizeof(uint32_t), "flags"));
    DFA_TRY(c.scalars.ensure(16 * sizeof(uint32_t), "scalars"));
    DFA_TRY(c.reach_visited.ensure(words64 * sizeof(unsigned long long), "visited bits"));
    DFA_TRY(c.reach_qa.ensure(static_cast<size_t>(n) * sizeof(uint32_t), "search queue"));
    DFA_TRY(c.reach_qb.ensure(static_cast<size_t>(n), "search marks"));
    DFA_TRY(c.reach_flags.ensure(static_cast<size_t>(n) * sizeof(uint32_t), "reachable flags"));
    DFA_TRY(c.reach_dense.ensure(static_cast<size_t>(n) * sizeof(uint32_t), "reachable numbering"));
    DFA_TRY(c.reach_orig.ensure(static_cast<size_t>(n) * sizeof(uint32_t), "reachable states"));
    DFA_TRY(c.partials.ensure((ntiles + 1) * sizeof(uint32_t), "scan partials"));
    HIP_TRY(hipEventRecord(c.ev_p0, c.stream));
    uint32_t *err = c.flags.as<uint32_t>();
    HIP_TRY(hipMemsetAsync(err, 0, sizeof(uint32_t), c.stream));
    launch_check_targets(delta, static_cast<uint64_t>(n) * k, n, err, c.stream);
    HIP_TRY(hipGetLastError());
    DFA_TRY(read_back(c, err, sizeof(uint32_t)));
    if (c.pinned[0]) return fail(DFA_EINVAL, "a transition target is >= n");

    uint32_t *sizes = c.scalars.as<uint32_t>();
    ReachArgs ra{delta, n, k, c.reach_visited.as<unsigned long long>(), c.reach_qb.as<uint8_t>(),
                 c.reach_qa.as<uint32_t>(), sizes};
    HIP_TRY(hipMemsetAsync(ra.visited, 0, words64 * sizeof(unsigned long long), c.stream));
    HIP_TRY(hipMemsetAsync(ra.mark, 0, n, c.stream));
    launch_bfs_init(ra, o.start, c.stream);
    // small frontiers: a queue expanded in one workgroup; large ones: dense
    // levels over the marks (frontier mark f, alternating 2 / 3)
    const uint64_t cap = bfs_narrow_cap();
    bool dense = false;
    uint8_t f = 2;
    for (;;) {
        HIP_TRY(hipGetLastError());
        if (!dense) {
            DFA_TRY(read_back(c, sizes, sizeof(uint32_t)));
            const uint32_t frontier = c.pinned[0];
            if (frontier == 0) break;
            if (static_cast<uint64_t>(frontier) * k <= cap) {
                launch_bfs_narrow(ra, c.stream);
                continue;
            }
            launch_bfs_list_to_marks(ra, frontier, f, c.stream);
            dense = true;
        }
        const uint8_t nf = f == 2 ? 3 : 2;
        launch_bfs_dense(ra, f, nf, c.stream);
        HIP_TRY(hipGetLastError());
        DFA_TRY(read_back(c, sizes + 1, sizeof(uint32_t)));
        const uint32_t stored = c.pinned[0];  // >= the new states; 0 iff none
        if (stored == 0) break;
        f = nf;
        if (static_cast<uint64_t>(stored) * k <= cap) {
            launch_bfs_marks_to_list(ra, f, c.stream);
            dense = false;
        }
    }
    // dense numbering of the reachable states; m = their count
    launch_reach_flags(ra.mark, n, c.reach_flags.as<uint32_t>(), c.stream);
    launch_dense_leaders(c.reach_flags.as<uint32_t>(), n, c.partials.as<uint32_t>(),
                         c.reach_dense.as<uint32_t>(), c.reach_orig.as<uint32_t>(), sizes + 2,
                         c.stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(sizes + 3, c.reach_dense.as<uint32_t>() + o.start, sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, c.stream));
    DFA_TRY(read_back(c, sizes + 2, 2 * sizeof(uint32_t)));
    const uint32_t m = c.pinned[0], sub_start = c.pinned[1];
    DFA_TRY(c.sub_delta.ensure(static_cast<size_t>(m) * k * sizeof(uint32_t), "sub-automaton"));
    DFA_TRY(c.sub_acc.ensure(m, "sub-automaton"));
    DFA_TRY(c.sub_block.ensure(static_cast<size_t>(m) * sizeof(uint32_t), "sub-automaton ids"));
    launch_sub_dfa(delta, acc, k, c.reach_orig.as<uint32_t>(), c.reach_dense.as<uint32_t>(),
                   sizes + 2, m, c.sub_delta.as<uint32_t>(), c.sub_acc.as<uint8_t>(), c.stream);
    HIP_TRY(hipGetLastError());
    dfa_options o2 = o;
    o2.prune = 0;
    o2.start = sub_start;
    int rc = minimise_impl(c, m, k, c.sub_delta.as<uint32_t>(), c.sub_acc.as<uint8_t>(),
                           c.sub_block.as<uint32_t>(), q, o2, st);
    if (rc != DFA_OK && rc != DFA_ELIMIT) return rc;
    launch_reach_expand(ra.mark, n, c.reach_dense.as<uint32_t>(), c.reach_orig.as<uint32_t>(),
                        c.sub_block.as<uint32_t>(), block_out, c.stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(c.ev_p1, c.stream));
    HIP_TRY(stream_sync(c));
    if (st) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c.ev_p0, c.ev_p1));
        st->device_ms = ms;
        st->reachable = m;
    }
    return rc;
}

int included_impl(Ctx &c, const dfa_view &a, const dfa_view &b, int *verdict, uint64_t *visited,
                  dfa_stats *st, int mode);

int equivalent_impl(Ctx &c, const dfa_view &a, const dfa_view &b, int *verdict,
                    const dfa_options &o, dfa_stats *st) {
    if (o.equiv_method == DFA_EQ_PRODUCT) return included_impl(c, a, b, verdict, nullptr, st, 1);
    const size_t N = static_cast<size_t>(a.n) + b.n;
    if (N >= 0xFFFFFFFFull) return fail(DFA_EINVAL, "nA + nB must be < 2^32 - 1");
    const uint32_t k = a.k;
    DFA_TRY(prepare_refinement(c, N, k));
    HIP_TRY(hipEventRecord(c.ev_start, c.stream));
    uint32_t *flags = c.flags.as<uint32_t>();
    uint32_t *cols = c.cols.as<uint32_t>();
    // two separate target checks: A's targets < nA, B's < nB
    launch_ingest(a.delta, a.n, k, cols, N, 0, 0, flags + kFlagErr, flags + kFlagNonid, c.stream);
    launch_ingest(b.delta, b.n, k, cols, N, a.n, a.n, flags + kFlagErr, flags + kFlagNonid,
                  c.stream);
    launch_init_blocks(a.accepting, a.n, 0, c.blockA.as<uint32_t>(),
                       c.accbits.as<unsigned long long>(), flags + kFlagClass, c.stream);
    launch_init_blocks(b.accepting, b.n, a.n, c.blockA.as<uint32_t>(),
                       c.accbits.as<unsigned long long>(), flags + kFlagClass, c.stream);
    HIP_TRY(hipGetLastError());
    RefineResult r;
    DFA_TRY(refine_any(c, N, k, o, 1, a.start, a.n + b.start, false, r));
    HIP_TRY(hipEventRecord(c.ev_stop, c.stream));
    HIP_TRY(stream_sync(c));
    fill_stats(st, r);
    if (st) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c.ev_start, c.ev_stop));
        st->device_ms = ms;
    }
    if (r.ctl.separated) {
        *verdict = 0;
        return DFA_OK;
    }
    if (r.ctl.limit)
        return fail(DFA_ELIMIT, "max_rounds (%u) reached before the verdict was known",
                    o.max_rounds);
    *verdict = 1;
    return DFA_OK;
}

// Breadth-first exploration of the synchronous product from (start_a,
// start_b), one level per launch.  mode 0: inclusion (refuted by p accepting,
// q rejecting); mode 1: equivalence (refuted by exactly one accepting side).
int included_impl(Ctx &c, const dfa_view &a, const dfa_view &b, int *verdict, uint64_t *visited,
                  dfa_stats *st, int mode = 0) {
    const uint32_t k = a.k;
    // reuse the flag buffer for the target checks (no refinement here)
    DFA_TRY(c.flags.ensure((kFlagNonid + k) * sizeof(uint32_t), "flags"));
    const size_t N = static_cast<size_t>(a.n) + b.n;
    DFA_TRY(c.cols.ensure(static_cast<size_t>(k) * N * sizeof(uint32_t), "columns"));
    HIP_TRY(hipMemsetAsync(c.flags.p, 0, (kFlagNonid + k) * sizeof(uint32_t), c.stream));
    HIP_TRY(hipEventRecord(c.ev_start, c.stream));
    uint32_t *flags = c.flags.as<uint32_t>();
    launch_ingest(a.delta, a.n, k, c.cols.as<uint32_t>(), N, 0, 0, flags + kFlagErr,
                  flags + kFlagNonid, c.stream);
    launch_ingest(b.delta, b.n, k, c.cols.as<uint32_t>(), N, a.n, a.n, flags + kFlagErr,
                  flags + kFlagNonid, c.stream);
    HIP_TRY(hipGetLastError());
    DFA_TRY(read_back(c, flags, sizeof(uint32_t)));
    if (c.pinned[0]) return fail(DFA_EINVAL, "a transition target is >= n");

    uint64_t cap = next_pow2(std::max<uint64_t>(4 * N, 4096));
    DFA_TRY(c.visited.ensure(cap * sizeof(unsigned long long), "visited set"));
    launch_visited_clear(c.visited.as<unsigned long long>(), cap, c.stream);
    const unsigned long long start = (static_cast<unsigned long long>(a.start) << 32) | b.start;
    launch_visited_insert_start(c.visited.as<unsigned long long>(), cap, start, c.stream);
    // both frontier buffers hold at least a narrow launch's frontier
    DFA_TRY(c.front0.ensure(kProductNarrowCap * sizeof(unsigned long long), "frontier"));
    DFA_TRY(c.front1.ensure(kProductNarrowCap * sizeof(unsigned long long), "frontier"));
    DFA_TRY(upload(c, c.front0.p, &start, sizeof start));
    DFA_TRY(c.scalars.ensure(16 * sizeof(uint32_t), "scalars"));
    uint32_t *sc = c.scalars.as<uint32_t>();
    Buffer *cur = &c.front0, *nxt = &c.front1;
    uint64_t count = 1, fsize = 1;
    uint32_t levels = 0;
    int v = 1;
    // levels per narrow launch: bounds the pairs one launch may add
    constexpr uint32_t kNarrowLevels = 256;
    while (fsize > 0) {
        if (fsize * k <= kProductNarrowCap) {
            // thin frontier: levels expanded inside one workgroup, the set
            // sized first for every pair the launch may add (at half load)
            const uint64_t most = count + static_cast<uint64_t>(kNarrowLevels) * kProductNarrowCap;
            if (most * 2 > cap) {
                const uint64_t ncap = next_pow2(most * 2);
                DFA_TRY(c.visited2.ensure(ncap * sizeof(unsigned long long), "visited set"));
                launch_visited_clear(c.visited2.as<unsigned long long>(), ncap, c.stream);
                launch_rehash(c.visited.as<unsigned long long>(), cap,
                              c.visited2.as<unsigned long long>(), ncap, c.stream);
                std::swap(c.visited, c.visited2);
                cap = ncap;
            }
            HIP_TRY(hipMemsetAsync(sc + 4, 0, 4 * sizeof(uint32_t), c.stream));
            ProductArgs pa{a.delta, b.delta, a.accepting, b.accepting, k, mode,
                           cur->as<unsigned long long>(), static_cast<uint32_t>(fsize), nullptr, 0,
                           nullptr, c.visited.as<unsigned long long>(), cap, nullptr, nullptr};
            launch_product_narrow(pa, kNarrowLevels, sc + 4, c.stream);
            HIP_TRY(hipGetLastError());
            DFA_TRY(read_back(c, sc + 4, 4 * sizeof(uint32_t)));
            fsize = c.pinned[0];
            count += c.pinned[1];
            levels += c.pinned[2];
            if (c.pinned[3]) {
                v = 0;
                break;
            }
            continue;
        }
        ++levels;
        const uint64_t need = fsize * k;
        if (need >= 0xFFFFFFFFull) return fail(DFA_ENOMEM, "frontier too large");
        DFA_TRY(nxt->ensure(need * sizeof(unsigned long long), "frontier"));
        if ((count + need) * 2 > cap) {
            const uint64_t ncap = next_pow2((count + need) * 2);
            DFA_TRY(c.visited2.ensure(ncap * sizeof(unsigned long long), "visited set"));
            launch_visited_clear(c.visited2.as<unsigned long long>(), ncap, c.stream);
            launch_rehash(c.visited.as<unsigned long long>(), cap,
                          c.visited2.as<unsigned long long>(), ncap, c.stream);
            std::swap(c.visited, c.visited2);
            cap = ncap;
        }
        HIP_TRY(hipMemsetAsync(sc, 0, 3 * sizeof(uint32_t), c.stream));
        ProductArgs pa{a.delta, b.delta, a.accepting, b.accepting, k, mode,
                       cur->as<unsigned long long>(), static_cast<uint32_t>(fsize),
                       nxt->as<unsigned long long>(), static_cast<uint32_t>(need), sc,
                       c.visited.as<unsigned long long>(), cap, sc + 1, sc + 2};
        launch_product_level(pa, c.stream);
        HIP_TRY(hipGetLastError());
        DFA_TRY(read_back(c, sc, 3 * sizeof(uint32_t)));
        if (c.pinned[2]) return fail(DFA_EDEVICE, "internal: frontier overflow");
        if (c.pinned[1]) {
            v = 0;
            break;
        }
        fsize = c.pinned[0];
        count += fsize;
        std::swap(cur, nxt);
    }
    HIP_TRY(hipEventRecord(c.ev_stop, c.stream));
    HIP_TRY(stream_sync(c));
    *verdict = v;
    if (visited) *visited = count;
    if (st) {
        std::memset(st, 0, sizeof *st);
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c.ev_start, c.ev_stop));
        st->device_ms = ms;
        st->rounds = levels;
        st->reachable = static_cast<uint32_t>(std::min<uint64_t>(count, 0xFFFFFFFFull));
    }
    return DFA_OK;
}

// ---- argument checks ----

int check_view(const dfa_view *v, const char *name) {
    if (!v) return fail(DFA_EINVAL, "%s is NULL", name);
    if (v->n == 0 || v->k == 0) return fail(DFA_EINVAL, "%s: n and k must be >= 1", name);
    if (v->n == 0xFFFFFFFFu) return fail(DFA_EINVAL, "%s: n must be < 2^32 - 1", name);
    if (!v->delta || !v->accepting) return fail(DFA_EINVAL, "%s: NULL delta/accepting", name);
    if (v->start >= v->n) return fail(DFA_EINVAL, "%s: start %u >= n %u", name, v->start, v->n);
    return DFA_OK;
}

int check_pair(const dfa_view *a, const dfa_view *b, const int *verdict) {
    DFA_TRY(check_view(a, "a"));
    DFA_TRY(check_view(b, "b"));
    if (a->k != b->k) return fail(DFA_EINVAL, "alphabet sizes differ (%u vs %u)", a->k, b->k);
    if (!verdict) return fail(DFA_EINVAL, "verdict is NULL");
    return DFA_OK;
}

int check_minimise(uint32_t n, uint32_t k, const void *delta, const void *acc, const void *out,
                   const dfa_quotient *q, const dfa_options &o) {
    if (n == 0 || k == 0) return fail(DFA_EINVAL, "n and k must be >= 1");
    if (n == 0xFFFFFFFFu) return fail(DFA_EINVAL, "n must be < 2^32 - 1");
    if (!delta || !acc || !out) return fail(DFA_EINVAL, "NULL delta/accepting/block_out");
    if (q && (!q->delta || !q->accepting)) return fail(DFA_EINVAL, "NULL quotient arrays");
    if (o.start >= n) return fail(DFA_EINVAL, "start %u >= n %u", o.start, n);
    return check_options(o);
}

// Orders the work already queued on the caller's stream (NULL = the legacy
// default stream) before the library's own stream.
int join_stream(Ctx &c, void *stream) {
    auto s = static_cast<hipStream_t>(stream);
    if (s == c.stream) return DFA_OK;
    HIP_TRY(hipEventRecord(c.ev_in, s));
    HIP_TRY(hipStreamWaitEvent(c.stream, c.ev_in, 0));
    return DFA_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ---- batches: many DFAs in one segmented refinement ----

// memcpy split over a few threads for large inputs (one thread reaches about
// a quarter of the host's copy bandwidth).
// Runs part(0) .. part(parts - 1): part 0 on the calling thread, the others
// on threads of their own.  If a thread cannot be started, the calling
// thread runs the parts left over, so no exception leaves with a joinable
// thread.
template <typename F>
void parallel_for(size_t parts, const F &part) {
    std::vector<std::thread> th;
    size_t next = 1;  // first part not handed to a thread
    try {
        th.reserve(parts);
        for (; next < parts; ++next) th.emplace_back(part, next);
    } catch (const std::exception &) {
    }
    if (parts) part(0);
    for (size_t i = next; i < parts; ++i) part(i);
    for (auto &t : th) t.join();
}

void parallel_copy(void *dst, const void *src, size_t bytes) {
    constexpr size_t kSplitBytes = size_t(8) << 20;
    if (bytes < kSplitBytes) {
        std::memcpy(dst, src, bytes);
        return;
    }
    const unsigned hw = std::max(2u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>({8, hw / 2, bytes / (kSplitBytes / 4)});
    const size_t chunk = ((bytes + nt - 1) / nt + 63) & ~size_t(63);
    auto part = [=](size_t i) {
        const size_t off = i * chunk;
        if (off < bytes)
            std::memcpy(static_cast<char *>(dst) + off, static_cast<const char *>(src) + off,
                        std::min(chunk, bytes - off));
    };
    parallel_for(nt, part);
}

// Many small copies (the DFAs of a batch) on up to 8 threads, each taking a
// run of consecutive copies of about equal total size.
struct CopyJob {
    void *dst;
    const void *src;
    size_t bytes;
};

void parallel_copies(const std::vector<CopyJob> &jobs) {
    size_t total = 0;
    for (const CopyJob &j : jobs) total += j.bytes;
    if (jobs.size() == 1) {
        parallel_copy(jobs[0].dst, jobs[0].src, jobs[0].bytes);
        return;
    }
    const unsigned hw = std::max(2u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>({8, hw / 2, total / (size_t(2) << 20) + 1});
    auto run = [&jobs](size_t lo, size_t hi) {
        for (size_t i = lo; i < hi; ++i) std::memcpy(jobs[i].dst, jobs[i].src, jobs[i].bytes);
    };
    if (nt <= 1) {
        run(0, jobs.size());
        return;
    }
    // cut the job list where the running total passes each 1/nt of the bytes
    std::vector<size_t> cut{0};
    size_t acc = 0;
    for (size_t i = 0; i < jobs.size() && cut.size() < nt; ++i) {
        acc += jobs[i].bytes;
        if (acc * nt >= total * cut.size()) cut.push_back(i + 1);
    }
    cut.push_back(jobs.size());
    parallel_for(cut.size() - 1, [&](size_t t) { run(cut[t], cut[t + 1]); });
}

int ensure_pinned_batch(Ctx &c, size_t bytes) {
    if (c.pinned_batch && bytes <= c.pinned_batch_cap) return DFA_OK;
    if (c.pinned_batch) {
        HIP_TRY(stream_sync(c));
        (void)hipHostFree(c.pinned_batch);
        c.pinned_batch = nullptr;
        c.pinned_batch_cap = 0;
    }
    const size_t want = std::max<size_t>(bytes, 1 << 20);
    if (hipHostMalloc(reinterpret_cast<void **>(&c.pinned_batch), want, hipHostMallocDefault) !=
        hipSuccess) {
        (void)hipGetLastError();
        c.pinned_batch = nullptr;
        return fail(DFA_ENOMEM, "pinned host allocation of %zu bytes failed", want);
    }
    c.pinned_batch_cap = want;
    return DFA_OK;
}

// parts (host vector, device pointers inside) -> device SegArgs.
int upload_plan(Ctx &c, const std::vector<Part> &parts, uint32_t nseg, bool pairs, size_t N,
                SegArgs &g) {
    const size_t tiles = (N + kBlock - 1) / kBlock;
    std::vector<uint32_t> tile_part(tiles);
    uint32_t p = 0;
    for (size_t t = 0; t < tiles; ++t) {
        const size_t first = t * kBlock;
        while (static_cast<size_t>(parts[p].off) + parts[p].n <= first) ++p;
        tile_part[t] = p;
    }
    DFA_TRY(c.parts.ensure(parts.size() * sizeof(Part), "batch parts"));
    DFA_TRY(c.tile_part.ensure(tiles * sizeof(uint32_t), "batch tiles"));
    DFA_TRY(c.seg_words.ensure((5 * static_cast<size_t>(nseg) + 1) * sizeof(uint32_t),
                               "segment counters"));
    // flags, then (2-byte aligned) the holder counts of decided tiles
    const size_t lead_at = (tiles + 1) & ~static_cast<size_t>(1);
    DFA_TRY(c.tile_dead.ensure(lead_at + 2 * tiles, "decided tiles"));
    HIP_TRY(hipMemcpy(c.parts.p, parts.data(), parts.size() * sizeof(Part),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c.tile_part.p, tile_part.data(), tiles * sizeof(uint32_t),
                      hipMemcpyHostToDevice));
    uint32_t *w = c.seg_words.as<uint32_t>();
    HIP_TRY(hipMemsetAsync(w, 0, (5 * static_cast<size_t>(nseg) + 1) * sizeof(uint32_t), c.stream));
    HIP_TRY(hipMemsetAsync(c.tile_dead.p, 0, tiles, c.stream));
    g.parts = c.parts.as<Part>();
    g.tile_part = c.tile_part.as<uint32_t>();
    g.nparts = static_cast<uint32_t>(parts.size());
    g.nseg = nseg;
    g.seg_cnt = w;
    g.seg_prev = w + nseg;
    g.seg_changing = w + 2 * static_cast<size_t>(nseg);
    g.seg_flags = w + 3 * static_cast<size_t>(nseg);
    g.seg_done = w + 4 * static_cast<size_t>(nseg);
    g.init_count = w + 5 * static_cast<size_t>(nseg);
    g.pairs = pairs ? 1u : 0u;
    g.tile_dead = c.tile_dead.as<uint8_t>();
    g.tile_lead = reinterpret_cast<uint16_t *>(c.tile_dead.as<uint8_t>() + lead_at);
    return DFA_OK;
}

// Refines the union described by parts; fills per-segment block counts and
// changing rounds (host vectors).
int refine_segments(Ctx &c, const std::vector<Part> &parts, uint32_t nseg, bool pairs,
                    uint32_t kmax, const dfa_options &o, RefineResult &r, SegArgs &g,
                    std::vector<uint32_t> &seg_blocks, std::vector<uint32_t> &seg_changing) {
    const Part &last = parts.back();
    const size_t N = static_cast<size_t>(last.off) + last.n;
    if (N >= 0xFFFFFFFFull) return fail(DFA_EINVAL, "total number of states must be < 2^32 - 1");
    DFA_TRY(upload_plan(c, parts, nseg, pairs, N, g));
    DFA_TRY(prepare_refinement(c, N, kmax));
    uint32_t *flags = c.flags.as<uint32_t>();
    launch_ingest_parts(g, N, kmax, c.cols.as<uint32_t>(), flags + kFlagErr, flags + kFlagNonid,
                        c.stream);
    launch_init_parts(g, N, c.blockA.as<uint32_t>(), c.accbits.as<unsigned long long>(), c.stream);
    HIP_TRY(hipGetLastError());
    dfa_options ob = o;
    if (ob.tc_mode == DFA_TC_AUTO) ob.tc_mode = DFA_TC_OFF;  // no closure on demand in batches
    DFA_TRY(refine(c, N, kmax, ob, 0, 0, 0, false, r, &g));
    seg_blocks.resize(nseg);
    seg_changing.resize(nseg);
    HIP_TRY(hipMemcpyAsync(seg_blocks.data(), g.seg_prev, nseg * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(hipMemcpyAsync(seg_changing.data(), g.seg_changing, nseg * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(stream_sync(c));
    return DFA_OK;
}

void fill_batch_stats(dfa_batch_stats *st, uint32_t count, const RefineResult &r, size_t N,
                      uint64_t transitions) {
    if (!st) return;
    st->count = count;
    st->rounds = r.ctl.round;
    st->k_eff = r.k_eff;
    st->states = N;
    st->transitions_refined = transitions;
    st->algorithmic_bytes = r.bytes;
}

// Places the views' arrays (host memory) into one pinned buffer and copies
// it to the device; returns device views.
int stage_views(Ctx &c, uint32_t count, const dfa_view *const *lists, int nlists,
                std::vector<dfa_view> &dev_views, double &h2d_ms) {
    size_t bytes = 0;
    for (int l = 0; l < nlists; ++l)
        for (uint32_t i = 0; i < count; ++i) {
            const dfa_view &v = lists[l][i];
            bytes += ((static_cast<size_t>(v.n) * v.k * 4 + 255) & ~size_t(255)) +
                     ((static_cast<size_t>(v.n) + 255) & ~size_t(255));
        }
    DFA_TRY(ensure_pinned_batch(c, bytes));
    DFA_TRY(c.batch_in.ensure(bytes, "batched inputs"));
    auto t0 = std::chrono::steady_clock::now();
    size_t off = 0;
    dev_views.clear();
    uint8_t *dev = c.batch_in.as<uint8_t>();
    std::vector<CopyJob> jobs;
    jobs.reserve(2 * static_cast<size_t>(count) * nlists);
    for (int l = 0; l < nlists; ++l)
        for (uint32_t i = 0; i < count; ++i) {
            const dfa_view &v = lists[l][i];
            dfa_view d = v;
            const size_t db = static_cast<size_t>(v.n) * v.k * 4;
            jobs.push_back({c.pinned_batch + off, v.delta, db});
            d.delta = reinterpret_cast<const uint32_t *>(dev + off);
            off += (db + 255) & ~size_t(255);
            jobs.push_back({c.pinned_batch + off, v.accepting, v.n});
            d.accepting = dev + off;
            off += (static_cast<size_t>(v.n) + 255) & ~size_t(255);
            dev_views.push_back(d);
        }
    parallel_copies(jobs);
    HIP_TRY(hipMemcpyAsync(dev, c.pinned_batch, off, hipMemcpyHostToDevice, c.stream));
    HIP_TRY(stream_sync(c));
    h2d_ms = ms_since(t0);
    return DFA_OK;
}

int check_views(uint32_t count, const dfa_view *v, const char *name) {
    if (count == 0) return fail(DFA_EINVAL, "count must be >= 1");
    if (!v) return fail(DFA_EINVAL, "%s is NULL", name);
    for (uint32_t i = 0; i < count; ++i) {
        int rc = check_view(v + i, name);
        if (rc != DFA_OK) return fail(rc, "%s[%u]: %s", name, i, g_last_error.c_str());
    }
    return DFA_OK;
}

// Batched minimisation on device views; out_dev receives the block ids,
// part i at out_off[i].
// Largest job (states) that goes to the one-workgroup path: the tuning's
// limit, lowered to what one workgroup's LDS holds on this device.
uint32_t small_cutoff(Ctx &c) {
    uint32_t cut = std::min(c.tune.batch_lds_states, kSmallMaxStates);
    if (!cut) return 0;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device) !=
        hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    // (plus the kernel's own few static words)
    while (cut && static_cast<int>(small_refine_lds_bytes(cut)) + 256 > lds) cut >>= 1;
    return cut;
}

// Queues the small jobs (one workgroup each, largest first); their results
// are read back by finish_small_jobs after the stream is synchronised.
int launch_small_jobs(Ctx &c, std::vector<SmallJob> &jobs, uint32_t slots, uint32_t *out_dev,
                      uint32_t max_rounds) {
    std::sort(jobs.begin(), jobs.end(), [](const SmallJob &x, const SmallJob &y) {
        return x.na + x.nb > y.na + y.nb;
    });
    const uint32_t nmax = jobs.front().na + jobs.front().nb;
    const uint32_t lds = small_refine_lds_bytes(nmax);
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device));
    const int fit = small_refine_max_groups(lds, cus);
    if (fit <= 0) return fail(DFA_EDEVICE, "no workgroup of %u LDS bytes fits the device", lds);
    const uint32_t groups = std::min<uint32_t>(static_cast<uint32_t>(jobs.size()),
                                               static_cast<uint32_t>(fit));
    DFA_TRY(c.small_jobs.ensure(jobs.size() * sizeof(SmallJob), "small jobs"));
    DFA_TRY(c.small_results.ensure(static_cast<size_t>(slots) * sizeof(SmallResult),
                                   "small results"));
    DFA_TRY(c.small_ctl.ensure(2 * sizeof(uint32_t), "small job counter"));
    HIP_TRY(hipMemcpyAsync(c.small_jobs.p, jobs.data(), jobs.size() * sizeof(SmallJob),
                           hipMemcpyHostToDevice, c.stream));
    uint32_t *ctl = c.small_ctl.as<uint32_t>();
    launch_small_refine(c.small_jobs.as<SmallJob>(), static_cast<uint32_t>(jobs.size()), groups,
                        lds, ctl, out_dev, c.small_results.as<SmallResult>(), max_rounds, ctl + 1,
                        c.stream);
    HIP_TRY(hipGetLastError());
    return DFA_OK;
}

// After the stream has been synchronised: the small jobs' results (indexed
// by DFA / pair) and their target check.
int finish_small_jobs(Ctx &c, uint32_t slots, std::vector<SmallResult> &res) {
    res.resize(slots);
    HIP_TRY(hipMemcpy(res.data(), c.small_results.p, slots * sizeof(SmallResult),
                      hipMemcpyDeviceToHost));
    uint32_t err = 0;
    HIP_TRY(hipMemcpy(&err, c.small_ctl.as<uint32_t>() + 1, sizeof err, hipMemcpyDeviceToHost));
    if (err) return fail(DFA_EINVAL, "a transition target is >= n");
    return DFA_OK;
}

int minimise_batch_impl(Ctx &c, uint32_t count, const dfa_view *views, uint32_t *out_dev,
                        const uint64_t *out_off, uint32_t *num_blocks, uint32_t *rounds,
                        const dfa_options &o, dfa_batch_stats *st) {
    // small DFAs: one workgroup each; the others: one segmented refinement
    const uint32_t cutoff = small_cutoff(c);
    std::vector<Part> parts;
    std::vector<uint32_t> large_of;  // DFA index of each segment
    std::vector<SmallJob> small;
    uint64_t off = 0, out = 0, total = 0;
    uint32_t kmax = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const dfa_view &v = views[i];
        const uint64_t out_i = out_off ? out_off[i] : out;
        out += v.n;
        total += v.n;
        if (v.n <= cutoff && v.k <= kSmallMaxK) {
            SmallJob j;
            std::memset(&j, 0, sizeof j);
            j.delta_a = v.delta;
            j.acc_a = v.accepting;
            j.na = v.n;
            j.k = v.k;
            j.index = i;
            j.out = out_i;
            small.push_back(j);
            continue;
        }
        Part p;
        std::memset(&p, 0, sizeof p);
        p.delta = v.delta;
        p.accepting = v.accepting;
        p.n = v.n;
        p.k = v.k;
        p.off = static_cast<uint32_t>(off);
        p.seg = static_cast<uint32_t>(parts.size());
        p.start = v.start;
        p.out = out_i;
        off += v.n;
        kmax = std::max(kmax, v.k);
        if (off >= 0xFFFFFFFFull) return fail(DFA_EINVAL, "total number of states must be < 2^32 - 1");
        parts.push_back(p);
        large_of.push_back(i);
    }
    HIP_TRY(hipEventRecord(c.ev_start, c.stream));
    if (!small.empty()) DFA_TRY(launch_small_jobs(c, small, count, out_dev, o.max_rounds));
    RefineResult r;
    SegArgs g{};
    std::vector<uint32_t> blocks, changing;
    const size_t N = off;
    if (!parts.empty()) {
        DFA_TRY(refine_segments(c, parts, static_cast<uint32_t>(parts.size()), false, kmax, o,
                                r, g, blocks, changing));
        DFA_TRY(c.canon.ensure(N * sizeof(uint32_t), "canonical ids"));
        // canonical ids go to the block buffer that does not hold the result
        uint32_t *canon_ids = c.blockA.as<uint32_t>() == r.final_block ? c.blockB.as<uint32_t>()
                                                                       : c.blockA.as<uint32_t>();
        launch_canonicalise(r.final_block, N, N, c.canon.as<uint32_t>(), canon_ids, c.stream);
        launch_part_output(g, N, canon_ids, out_dev, c.stream);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipEventRecord(c.ev_stop, c.stream));
    HIP_TRY(stream_sync(c));
    std::vector<SmallResult> sres;
    if (!small.empty()) DFA_TRY(finish_small_jobs(c, count, sres));
    uint64_t transitions = 0, small_bytes = 0;
    uint32_t joint_rounds = parts.empty() ? 0 : r.ctl.round;
    bool limit = !parts.empty() && r.ctl.limit;
    auto record = [&](uint32_t i, uint32_t nb, uint32_t ch) {
        if (num_blocks) num_blocks[i] = nb;
        if (rounds) rounds[i] = ch + 1;
        transitions += static_cast<uint64_t>(views[i].n) * views[i].k * (ch + 1);
    };
    for (size_t j = 0; j < parts.size(); ++j) record(large_of[j], blocks[j], changing[j]);
    for (const SmallJob &j : small) {
        const SmallResult &sr = sres[j.index];
        record(j.index, sr.num_blocks, sr.changing);
        joint_rounds = std::max(joint_rounds, sr.rounds);
        limit |= sr.limit != 0;
        small_bytes += static_cast<uint64_t>(j.na) * sr.rounds * (8ull * j.k + 8ull);
    }
    if (st) {
        fill_batch_stats(st, count, r, total, transitions);
        st->rounds = joint_rounds;
        if (parts.empty()) st->k_eff = 0;
        st->algorithmic_bytes = (parts.empty() ? 0 : r.bytes) + small_bytes;
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c.ev_start, c.ev_stop));
        st->device_ms = ms;
    }
    if (limit)
        return fail(DFA_ELIMIT, "max_rounds (%u) reached before every partition was stable",
                    o.max_rounds);
    return DFA_OK;
}

int equivalent_batch_impl(Ctx &c, uint32_t count, const dfa_view *a, const dfa_view *b,
                          int32_t *verdicts, const dfa_options &o, dfa_batch_stats *st,
                          uint32_t *rounds_out = nullptr) {
    // small pairs: one workgroup each; the others: one segmented refinement
    const uint32_t cutoff = small_cutoff(c);
    std::vector<Part> parts;
    std::vector<uint32_t> large_of;  // pair index of each segment
    std::vector<SmallJob> small;
    uint64_t off = 0, total = 0;
    uint32_t kmax = 0;
    for (uint32_t i = 0; i < count; ++i) {
        total += static_cast<uint64_t>(a[i].n) + b[i].n;
        if (static_cast<uint64_t>(a[i].n) + b[i].n <= cutoff && a[i].k <= kSmallMaxK) {
            SmallJob j;
            std::memset(&j, 0, sizeof j);
            j.delta_a = a[i].delta;
            j.acc_a = a[i].accepting;
            j.delta_b = b[i].delta;
            j.acc_b = b[i].accepting;
            j.na = a[i].n;
            j.nb = b[i].n;
            j.k = a[i].k;
            j.start_a = a[i].start;
            j.start_b = b[i].start;
            j.index = i;
            small.push_back(j);
            continue;
        }
        const uint32_t seg = static_cast<uint32_t>(large_of.size());
        for (int side = 0; side < 2; ++side) {
            const dfa_view &v = side ? b[i] : a[i];
            Part p;
            std::memset(&p, 0, sizeof p);
            p.delta = v.delta;
            p.accepting = v.accepting;
            p.n = v.n;
            p.k = v.k;
            p.off = static_cast<uint32_t>(off);
            p.seg = seg;
            p.start = v.start;
            off += v.n;
            kmax = std::max(kmax, v.k);
            if (off >= 0xFFFFFFFFull)
                return fail(DFA_EINVAL, "total number of states must be < 2^32 - 1");
            parts.push_back(p);
        }
        large_of.push_back(i);
    }
    HIP_TRY(hipEventRecord(c.ev_start, c.stream));
    if (!small.empty()) DFA_TRY(launch_small_jobs(c, small, count, nullptr, o.max_rounds));
    RefineResult r;
    SegArgs g{};
    std::vector<uint32_t> blocks, changing;
    const uint32_t nseg = static_cast<uint32_t>(large_of.size());
    std::vector<int32_t> seg_verdicts(nseg);
    if (nseg) {
        DFA_TRY(refine_segments(c, parts, nseg, true, kmax, o, r, g, blocks, changing));
        DFA_TRY(c.batch_out.ensure(nseg * sizeof(int32_t), "verdicts"));
        launch_pair_verdicts(g, r.final_block, c.batch_out.as<int32_t>(), c.stream);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(seg_verdicts.data(), c.batch_out.p, nseg * sizeof(int32_t),
                               hipMemcpyDeviceToHost, c.stream));
    }
    HIP_TRY(hipEventRecord(c.ev_stop, c.stream));
    HIP_TRY(stream_sync(c));
    std::vector<SmallResult> sres;
    if (!small.empty()) DFA_TRY(finish_small_jobs(c, count, sres));
    uint64_t transitions = 0, small_bytes = 0;
    uint32_t joint_rounds = nseg ? r.ctl.round : 0;
    bool limit = nseg && r.ctl.limit;
    auto record = [&](uint32_t i, int32_t verdict, uint32_t ch) {
        verdicts[i] = verdict;
        if (rounds_out) rounds_out[i] = ch + 1;
        transitions += (static_cast<uint64_t>(a[i].n) + b[i].n) * a[i].k * (ch + 1);
    };
    for (uint32_t j = 0; j < nseg; ++j) record(large_of[j], seg_verdicts[j], changing[j]);
    for (const SmallJob &j : small) {
        const SmallResult &sr = sres[j.index];
        record(j.index, static_cast<int32_t>(sr.verdict), sr.changing);
        joint_rounds = std::max(joint_rounds, sr.rounds);
        limit |= sr.limit != 0;
        small_bytes += (static_cast<uint64_t>(j.na) + j.nb) * sr.rounds * (8ull * j.k + 8ull);
    }
    if (st) {
        fill_batch_stats(st, count, r, total, transitions);
        st->rounds = joint_rounds;
        if (!nseg) st->k_eff = 0;
        st->algorithmic_bytes = (nseg ? r.bytes : 0) + small_bytes;
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c.ev_start, c.ev_stop));
        st->device_ms = ms;
    }
    if (limit)
        return fail(DFA_ELIMIT, "max_rounds (%u) reached before every verdict was known",
                    o.max_rounds);
    return DFA_OK;
}

// dfa_minimise on an initialised context (host pointers in and out).

// Copies of large pageable host arrays go through two page-locked chunks:
// host threads fill (or drain) one chunk while the DMA engine moves the
// other, instead of the runtime's own single-threaded staging of pageable
// memory.  Small arrays are copied directly.
constexpr size_t kRingChunk = size_t(16) << 20;
constexpr size_t kRingMinBytes = size_t(8) << 20;

int ensure_ring(Ctx &c) {
    for (int i = 0; i < 2; ++i) {
        if (!c.ring[i] &&
            hipHostMalloc(reinterpret_cast<void **>(&c.ring[i]), kRingChunk, hipHostMallocDefault) !=
                hipSuccess) {
            c.ring[i] = nullptr;
            (void)hipGetLastError();
            return fail(DFA_ENOMEM, "page-locked staging of %zu bytes failed", kRingChunk);
        }
        if (!c.ring_ev[i]) HIP_TRY(hipEventCreateWithFlags(&c.ring_ev[i], hipEventDisableTiming));
    }
    return DFA_OK;
}

// Host -> device on the context's stream; returns once the last chunk is
// queued (the caller synchronises the stream).
int copy_to_device(Ctx &c, void *dst, const void *src, size_t bytes) {
    if (bytes < kRingMinBytes) {
        HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c.stream));
        return DFA_OK;
    }
    DFA_TRY(ensure_ring(c));
    size_t i = 0;
    for (size_t off = 0; off < bytes; off += kRingChunk, ++i) {
        const size_t len = std::min(kRingChunk, bytes - off);
        const int slot = static_cast<int>(i & 1);
        // the chunk's previous DMA (of this call or an earlier one) must be
        // done before it is refilled
        if (c.ring_recorded[slot]) HIP_TRY(hipEventSynchronize(c.ring_ev[slot]));
        parallel_copy(c.ring[slot], static_cast<const char *>(src) + off, len);
        HIP_TRY(hipMemcpyAsync(static_cast<char *>(dst) + off, c.ring[slot], len,
                               hipMemcpyHostToDevice, c.stream));
        HIP_TRY(hipEventRecord(c.ring_ev[slot], c.stream));
        c.ring_recorded[slot] = true;
    }
    return DFA_OK;
}

// Device -> host, after the work queued on the context's stream.  A large
// array is in `dst` on return; a small one once the caller has synchronised
// the stream.
int copy_to_host(Ctx &c, void *dst, const void *src, size_t bytes) {
    if (bytes < kRingMinBytes) {
        HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c.stream));
        return DFA_OK;
    }
    DFA_TRY(ensure_ring(c));
    const size_t chunks = (bytes + kRingChunk - 1) / kRingChunk;
    auto queue = [&](size_t i) -> int {
        const size_t off = i * kRingChunk;
        const int slot = static_cast<int>(i & 1);
        HIP_TRY(hipMemcpyAsync(c.ring[slot], static_cast<const char *>(src) + off,
                               std::min(kRingChunk, bytes - off), hipMemcpyDeviceToHost,
                               c.stream));
        HIP_TRY(hipEventRecord(c.ring_ev[slot], c.stream));
        c.ring_recorded[slot] = true;
        return DFA_OK;
    };
    DFA_TRY(queue(0));
    if (chunks > 1) DFA_TRY(queue(1));
    for (size_t i = 0; i < chunks; ++i) {
        const int slot = static_cast<int>(i & 1);
        const size_t off = i * kRingChunk;
        HIP_TRY(hipEventSynchronize(c.ring_ev[slot]));
        parallel_copy(static_cast<char *>(dst) + off, c.ring[slot],
                      std::min(kRingChunk, bytes - off));
        if (i + 2 < chunks) DFA_TRY(queue(i + 2));
    }
    return DFA_OK;
}

int minimise_host(Ctx &c_, uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *accepting,
                  uint32_t *block_out, dfa_quotient *q_out, const dfa_options &o,
                  dfa_stats *stats) {
    Ctx *c = &c_;
    if (stats) std::memset(stats, 0, sizeof *stats);
    const size_t nk = static_cast<size_t>(n) * k;
    DFA_TRY(c->stage_delta.ensure(nk * sizeof(uint32_t), "input copy"));
    DFA_TRY(c->stage_acc.ensure(n, "input copy"));
    DFA_TRY(c->stage_block.ensure(static_cast<size_t>(n) * sizeof(uint32_t), "output copy"));
    if (q_out) {
        DFA_TRY(c->stage_qdelta.ensure(nk * sizeof(uint32_t), "quotient copy"));
        DFA_TRY(c->stage_qacc.ensure(n, "quotient copy"));
    }
    auto t0 = std::chrono::steady_clock::now();
    DFA_TRY(copy_to_device(*c, c->stage_delta.p, delta, nk * sizeof(uint32_t)));
    DFA_TRY(copy_to_device(*c, c->stage_acc.p, accepting, n));
    HIP_TRY(stream_sync(*c));
    const double h2d = ms_since(t0);
    dfa_quotient dq{};
    if (q_out) {
        dq.delta = c->stage_qdelta.as<uint32_t>();
        dq.accepting = c->stage_qacc.as<uint8_t>();
    }
    int rc = minimise_impl(*c, n, k, c->stage_delta.as<uint32_t>(), c->stage_acc.as<uint8_t>(),
                           c->stage_block.as<uint32_t>(), q_out ? &dq : nullptr, o, stats);
    if (rc != DFA_OK && rc != DFA_ELIMIT) return rc;
    t0 = std::chrono::steady_clock::now();
    DFA_TRY(copy_to_host(*c, block_out, c->stage_block.p, static_cast<size_t>(n) * sizeof(uint32_t)));
    if (q_out) {
        DFA_TRY(copy_to_host(*c, q_out->delta, dq.delta,
                             static_cast<size_t>(dq.num_blocks) * k * sizeof(uint32_t)));
        DFA_TRY(copy_to_host(*c, q_out->accepting, dq.accepting, dq.num_blocks));
        q_out->num_blocks = dq.num_blocks;
        q_out->start = dq.start;
    }
    HIP_TRY(stream_sync(*c));
    if (stats) {
        stats->h2d_ms = h2d;
        stats->d2h_ms = ms_since(t0);
    }
    return rc;
}


int stage_view(Ctx &c, Buffer &bd, Buffer &ba, const dfa_view *v, dfa_view &out) {
    const size_t nk = static_cast<size_t>(v->n) * v->k;
    DFA_TRY(bd.ensure(nk * sizeof(uint32_t), "input copy"));
    DFA_TRY(ba.ensure(v->n, "input copy"));
    DFA_TRY(copy_to_device(c, bd.p, v->delta, nk * sizeof(uint32_t)));
    DFA_TRY(copy_to_device(c, ba.p, v->accepting, v->n));
    out = *v;
    out.delta = bd.as<uint32_t>();
    out.accepting = ba.as<uint8_t>();
    return DFA_OK;
}


// dfa_equivalent on an initialised context (host views).
int equivalent_host(Ctx &c, const dfa_view *a, const dfa_view *b, int *verdict,
                    const dfa_options &o, dfa_stats *stats) {
    if (stats) std::memset(stats, 0, sizeof *stats);
    auto t0 = std::chrono::steady_clock::now();
    dfa_view da, db;
    DFA_TRY(stage_view(c, c.stage_delta, c.stage_acc, a, da));
    DFA_TRY(stage_view(c, c.stage_delta_b, c.stage_acc_b, b, db));
    HIP_TRY(stream_sync(c));
    const double h2d = ms_since(t0);
    int rc = equivalent_impl(c, da, db, verdict, o, stats);
    if (stats) stats->h2d_ms = h2d;
    return rc;
}


// ---- served requests ----
//
// A server owns `lanes` workers; each has its own stream and workspace (a
// private Ctx).  Requests wait in a FIFO and are admitted while their HBM
// footprint fits the budget.  A free lane takes the head request: a large
// one runs alone (closure on demand); small ones of the same kind are taken
// together, up to max_group, and refined as one segmented union with a
// round budget; any that are not stable within it (chain-like DFAs) are run
// again alone with the closure.  Lanes run concurrently, so requests that
// arrive while others are on the GPU start as soon as a lane and memory are
// free, and their kernels overlap on the device.  Results are canonical, so
// a request's result does not depend on the requests it ran with.

// Calls f on every device buffer of a context.
template <class F>
void for_each_buffer(Ctx &c, F &&f) {
    Buffer *bufs[] = {&c.cols, &c.tc_cols, &c.colmap, &c.blockA, &c.blockB, &c.sig, &c.hash,
                      &c.table, &c.ctl, &c.flags, &c.canon, &c.dense, &c.leader_of, &c.partials,
                      &c.scalars, &c.multi, &c.active, &c.accbits, &c.counters, &c.presence,
                      &c.presence_packed, &c.lab8, &c.stage_delta, &c.stage_acc, &c.stage_block,
                      &c.stage_qdelta, &c.stage_qacc, &c.stage_delta_b, &c.stage_acc_b,
                      &c.visited, &c.visited2, &c.front0, &c.front1, &c.parts, &c.tile_part,
                      &c.seg_words, &c.batch_in, &c.batch_out, &c.new_leader, &c.moved,
                      &c.chg, &c.single, &c.touched, &c.chg_sum, &c.reach_visited, &c.reach_qa,
                      &c.reach_qb, &c.reach_flags, &c.reach_dense, &c.reach_orig, &c.sub_delta,
                      &c.sub_acc, &c.sub_block, &c.sort_keys0, &c.sort_keys1, &c.sort_vals0,
                      &c.sort_vals1, &c.sort_hist, &c.sort_partials, &c.sort_runhead,
                      &c.sort_m, &c.serve_in, &c.small_jobs, &c.small_results,
                      &c.small_ctl, &c.pb_tl, &c.pb_src, &c.pb_val, &c.pb_off,
                      &c.pb_partials, &c.segpat_table, &c.segpat, &c.tile_dead};
    for (Buffer *b : bufs) f(*b);
}

void release_ctx(Ctx &c) {
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    for_each_buffer(c, [](Buffer &b) {
        if (b.p && !b.arena) (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        b.allocation = 0;
    });
    for (hipGraphExec_t &g : c.graphs) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    for (hipEvent_t e : c.evpool) (void)hipEventDestroy(e);
    c.evpool.clear();
    if (c.ev_start) (void)hipEventDestroy(c.ev_start);
    if (c.ev_stop) (void)hipEventDestroy(c.ev_stop);
    if (c.ev_in) (void)hipEventDestroy(c.ev_in);
    if (c.ev_sync) (void)hipEventDestroy(c.ev_sync);
    c.ev_sync = nullptr;
    if (c.ev_p0) (void)hipEventDestroy(c.ev_p0);
    if (c.ev_p1) (void)hipEventDestroy(c.ev_p1);
    c.ev_p0 = c.ev_p1 = nullptr;
    if (c.ev_up0) (void)hipEventDestroy(c.ev_up0);
    if (c.ev_up1) (void)hipEventDestroy(c.ev_up1);
    c.ev_up0 = c.ev_up1 = nullptr;
    if (c.pinned) (void)hipHostFree(c.pinned);
    if (c.pinned_batch) (void)hipHostFree(c.pinned_batch);
    for (int i = 0; i < 2; ++i) {
        if (c.ring[i]) (void)hipHostFree(c.ring[i]);
        if (c.ring_ev[i]) (void)hipEventDestroy(c.ring_ev[i]);
        c.ring[i] = nullptr;
        c.ring_ev[i] = nullptr;
        c.ring_recorded[i] = false;
    }
    // the stream goes back to the pool (it was synchronised above)
    give_stream(c.device, c.stream);
    c.ev_start = c.ev_stop = c.ev_in = nullptr;
    c.pinned = nullptr;
    c.pinned_batch = nullptr;
    c.pinned_batch_cap = 0;
    c.stream = nullptr;
    c.inited = false;
}

// ---- the allocation-free entry point's context ----

// One per device: its own stream, lock and events (made at its first call,
// the set-up), and buffers carved from the device's copy of `scratch`.
Ctx g_fixed[kMaxDevices];

// The tuning set for each device (dfa_set_tuning), which every call on the
// device reads, whichever context runs it; the defaults until one is set.
std::mutex g_tuning_mu;
dfa_tuning g_tuning[kMaxDevices];
bool g_tuning_set[kMaxDevices];

// Set-up on the current device (once): the device address of `scratch`, and
// every buffer of the context bound to it.
int init_fixed(Ctx &c) {
    if (!c.arena.base) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(DFA_EDEVICE, "device address of the fixed workspace: %s",
                        hipGetErrorString(e));
        c.arena.base = static_cast<uint8_t *>(ptr);
        c.arena.size = kFixedScratchBytes;
        c.arena.used = 0;
        for_each_buffer(c, [&c](Buffer &b) {
            b.arena = &c.arena;
            b.p = nullptr;
            b.cap = 0;
        });
    }
    return init_ctx(c);
}

// Workspace of a plain refinement (no closure, no pruning) of n states and k
// letters in the fixed context, each buffer rounded up to 256 bytes as the
// arena carves it: columns 4k, block ids 8, marks 4, signatures 4(k + 1),
// hashes 8, table <= 32, canonical ids, dense ids, leaders 12, byte labels 1,
// bit masks < 1 per state; plus the label maps and small control words;
// with `slices`, the edges bucketed by target slice (8 bytes per edge, run
// counts and starts).
size_t fixed_plain_bytes(uint64_t n, uint64_t k, bool slices) {
    const uint64_t table = 8 * next_pow2(std::max<uint64_t>(2 * n, 1024));
    uint64_t bytes = n * (8 * k + 41) + table + kLabelMapBytes +
                     (1u << kPatternMaxBits) / 8 + (size_t(64) << 10);
    if (slices) {
        const uint64_t nb = (n >> kPbSliceLog) + 1, tiles = n / kPbTile + 1;
        bytes += n * 8 * k + nb * tiles * 12 + 6 * 256;
    }
    return bytes;
}

using Clock = std::chrono::steady_clock;

// Page-locked host buffers for submitted inputs, reused across requests (one
// free list per power-of-two size class); freed with the server.
struct PinnedPool {
    std::mutex mu;
    std::map<size_t, std::vector<void *>> free_lists;
    static size_t size_class(size_t bytes) {
        size_t c = size_t(1) << 16;
        while (c < bytes) c <<= 1;
        return c;
    }
    void *get(size_t bytes, size_t &cls) {
        cls = size_class(bytes);
        {
            std::lock_guard<std::mutex> g(mu);
            auto it = free_lists.find(cls);
            if (it != free_lists.end() && !it->second.empty()) {
                void *p = it->second.back();
                it->second.pop_back();
                return p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) return nullptr;
        return p;
    }
    void put(void *p, size_t cls) {
        std::lock_guard<std::mutex> g(mu);
        free_lists[cls].push_back(p);
    }
    ~PinnedPool() {
        for (auto &kv : free_lists)
            for (void *p : kv.second) (void)hipHostFree(p);
    }
};


struct ServedRequest {
    uint64_t ticket = 0;
    int kind = DFA_REQ_MINIMISE;
    dfa_view a{}, b{};        // the inputs: host copies, then device copies while running
    void *host_in = nullptr;  // page-locked copy made at submission
    size_t host_cls = 0;
    size_t in_bytes = 0;
    size_t off_acc_a = 0, off_delta_b = 0, off_acc_b = 0;
    size_t footprint = 0;     // device bytes while it runs, inputs included
    size_t states = 0;
    Clock::time_point t_submit, t_start, t_done;
    bool done = false;
    int status = DFA_OK;
    int verdict = 0;
    uint32_t num_blocks = 0, rounds = 0;
    bool batched = false;
    uint32_t *blocks = nullptr;  // minimisation result, page-locked (server pool)
    size_t blocks_cls = 0;
    // time of the work it ran in (its group's, when batched): input copies,
    // device work (refinements, a re-run alone included), result copy
    double h2d_ms = 0, device_ms = 0, d2h_ms = 0;
};

struct Server {
    int device = 0;
    dfa_server_config cfg{};
    dfa_tuning tune{};
    PinnedPool pinned;             // host copies of submitted inputs
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ServedRequest *> pending;
    std::unordered_map<uint64_t, std::unique_ptr<ServedRequest>> requests;
    // device memory of the lanes: held[i] = bytes of lane i's workspace
    // (grow-only buffers kept between requests); while lane i runs a group,
    // reserved[i] bounds its workspace for that run
    std::vector<size_t> held, reserved;
    std::vector<char> busy;
    bool stopping = false;
    bool paused = false;   // lanes take no request until dfa_server_resume
    uint32_t waiters = 0;  // threads inside dfa_server_wait (destroy waits for them)
    std::condition_variable cv_left;  // a waiter left dfa_server_wait
    uint64_t next_ticket = 1;
    uint64_t submitted = 0, completed = 0, rejected = 0, groups = 0, solo = 0;
    std::vector<double> latencies;
    Clock::time_point t_created;
    std::vector<std::thread> workers;
    std::vector<std::unique_ptr<Ctx>> lanes;
};

// Device bytes of a lane's workspace that do not scale with the requests:
// every buffer is rounded up to 2 MiB (about 40 of them), plus the pattern
// bitmap; charged once per admitted group (each request's footprint also
// counts the packed round's label map).
constexpr size_t kGroupFixedBytes = size_t(96) << 20;

// Sum of a lane's buffer capacities.
size_t workspace_bytes(Ctx &c) {
    size_t total = 0;
    for_each_buffer(c, [&](Buffer &b) { total += b.p ? b.cap : 0; });
    return total;
}

// Device bytes a request may add to a lane's workspace while it runs
// (inputs, columns, signatures, hashes, table, block buffers and marks,
// outputs, the edges bucketed by target slice, a batch's round-0 patterns),
// apart from the fixed part.
size_t request_footprint(uint64_t n, uint32_t k, bool closure) {
    const uint64_t slices = (n >> kPbSliceLog) + 1, tiles = n / kPbTile + 1;
    uint64_t bytes = n * (4ull * k + 1)        // input copy
                     + n * 4ull * k            // columns
                     + n * 4ull * (k + 1)      // signature rows
                     + n * 8ull                // hashes
                     + n * 32ull               // table (2n slots of 8 bytes, rounded up)
                     + n * 4ull * 6            // blocks A/B, marks, canonical ids, output, scratch
                     + n * 8ull * k            // bucketed edges: target, source slot, gathered id
                     + slices * tiles * 12ull  // run lengths and starts, scan sums
                     + n * 2ull                // round-0 patterns (batches)
                     + kLabelMapBytes          // the packed round's label map
                     + (1u << 22);             // fixed buffers
    if (k + 1 <= kSegPatMaxBits) bytes += 4ull << (k + 1);  // the request's pattern-table rows
    if (closure) {
        uint32_t L = floor_log2(std::max<uint64_t>(n, 1));
        bytes += n * 4ull * k * (L + 1);
    }
    return bytes;
}

void finish(Server &s, ServedRequest *r, const std::lock_guard<std::mutex> &) {
    r->t_done = Clock::now();
    r->done = true;
    s.completed++;
    s.latencies.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
}

// Runs one request alone on a lane (closure on demand); its inputs are
// already on the device.
void run_solo(Server &s, Ctx &c, ServedRequest *r) {
    dfa_options o;
    dfa_options_default(&o);
    o.tc_mode = s.cfg.tc_mode;
    o.loop_mode = DFA_LOOP_CHUNK;
    dfa_stats st{};
    if (r->kind == DFA_REQ_MINIMISE) {
        const size_t n = r->a.n;
        r->status = c.stage_block.ensure(n * sizeof(uint32_t), "output copy");
        if (r->status == DFA_OK)
            r->status = minimise_impl(c, r->a.n, r->a.k, r->a.delta, r->a.accepting,
                                      c.stage_block.as<uint32_t>(), nullptr, o, &st);
        if (r->status == DFA_OK) {
            r->blocks = static_cast<uint32_t *>(s.pinned.get(n * sizeof(uint32_t), r->blocks_cls));
            if (!r->blocks)
                r->status = fail(DFA_ENOMEM, "page-locked result buffer of %zu bytes", n * 4);
        }
        const auto t0 = Clock::now();
        if (r->status == DFA_OK &&
            (hipMemcpyAsync(r->blocks, c.stage_block.p, n * sizeof(uint32_t),
                            hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
             stream_sync(c) != hipSuccess))
            r->status = fail(DFA_EDEVICE, "copy of the result failed");
        r->d2h_ms += std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
        r->num_blocks = st.num_blocks;
        r->rounds = st.rounds;
    } else {
        int v = 0;
        r->status = equivalent_impl(c, r->a, r->b, &v, o, &st);
        r->verdict = v;
        r->rounds = st.rounds;
    }
    r->device_ms += st.device_ms;
    r->batched = false;
}

// Runs a group of small requests of one kind as one segmented refinement;
// the ones that are not stable within the round budget run again alone.
void run_group(Server &s, Ctx &c, std::vector<ServedRequest *> &grp) {
    dfa_options o;
    dfa_options_default(&o);
    o.tc_mode = DFA_TC_OFF;
    o.loop_mode = DFA_LOOP_CHUNK;
    o.max_rounds = s.cfg.batch_round_budget;
    const uint32_t count = static_cast<uint32_t>(grp.size());
    std::vector<uint32_t> rounds(count), nb(count);
    dfa_batch_stats bs{};
    std::vector<bool> redo(count, false);
    int rc;
    if (grp[0]->kind == DFA_REQ_MINIMISE) {
        std::vector<dfa_view> dev(count);
        for (uint32_t i = 0; i < count; ++i) dev[i] = grp[i]->a;
        uint64_t total = 0;
        for (auto *r : grp) total += r->a.n;
        rc = c.batch_out.ensure(total * sizeof(uint32_t), "batched outputs");
        if (rc == DFA_OK)
            rc = minimise_batch_impl(c, count, dev.data(), c.batch_out.as<uint32_t>(), nullptr,
                                     nb.data(), rounds.data(), o, &bs);
        if (rc == DFA_OK || rc == DFA_ELIMIT) {
            const auto t0 = Clock::now();
            int rc2 = ensure_pinned_batch(c, total * sizeof(uint32_t));
            const bool copied = rc2 == DFA_OK &&
                                hipMemcpyAsync(c.pinned_batch, c.batch_out.p,
                                               total * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                               c.stream) == hipSuccess &&
                                stream_sync(c) == hipSuccess;
            const double d2h = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
            for (auto *r : grp) r->d2h_ms += d2h;
            if (copied) {
                const uint32_t *src = reinterpret_cast<const uint32_t *>(c.pinned_batch);
                uint64_t pos = 0;
                for (uint32_t i = 0; i < count; ++i) {
                    ServedRequest *r = grp[i];
                    // a DFA that changed in every round may not be stable yet
                    redo[i] = rc == DFA_ELIMIT && rounds[i] > bs.rounds;
                    if (!redo[i]) {
                        r->blocks = static_cast<uint32_t *>(
                            s.pinned.get(static_cast<size_t>(r->a.n) * sizeof(uint32_t),
                                         r->blocks_cls));
                        if (!r->blocks) {
                            r->status = fail(DFA_ENOMEM, "page-locked result buffer");
                            pos += r->a.n;
                            continue;
                        }
                        std::memcpy(r->blocks, src + pos, r->a.n * sizeof(uint32_t));
                        r->num_blocks = nb[i];
                        r->rounds = rounds[i];
                        r->status = DFA_OK;
                        r->batched = true;
                    }
                    pos += r->a.n;
                }
                rc = DFA_OK;
            } else {
                rc = rc2 != DFA_OK ? rc2 : fail(DFA_EDEVICE, "copy of batched results failed");
            }
        }
    } else {
        std::vector<dfa_view> va(count), vb(count);
        for (uint32_t i = 0; i < count; ++i) {
            va[i] = grp[i]->a;
            vb[i] = grp[i]->b;
        }
        std::vector<int32_t> verdicts(count);
        rc = equivalent_batch_impl(c, count, va.data(), vb.data(), verdicts.data(), o, &bs,
                                   rounds.data());
        if (rc == DFA_OK || rc == DFA_ELIMIT) {
            for (uint32_t i = 0; i < count; ++i) {
                redo[i] = rc == DFA_ELIMIT && rounds[i] > bs.rounds;
                if (!redo[i]) {
                    grp[i]->verdict = verdicts[i];
                    grp[i]->rounds = rounds[i];
                    grp[i]->status = DFA_OK;
                    grp[i]->batched = true;
                }
            }
            rc = DFA_OK;
        }
    }
    for (auto *r : grp) r->device_ms += bs.device_ms;
    for (uint32_t i = 0; i < count; ++i) {
        if (rc != DFA_OK) {
            grp[i]->status = rc;
        } else if (redo[i]) {
            run_solo(s, c, grp[i]);
        }
    }
}

void lane_main(Server *sp, size_t lane) {
    // the lane allocates and synchronises while other threads may capture
    RelaxedCapture relaxed;
    Server &s = *sp;
    (void)hipSetDevice(s.device);
    Ctx &c = *s.lanes[lane];
    {
        std::lock_guard<std::mutex> g(c.mu);
        if (init_ctx(c) == DFA_OK) c.tune = s.tune;
        c.blocking_sync = true;
    }
    for (;;) {
        std::vector<ServedRequest *> grp, all;
        {
            std::unique_lock<std::mutex> lk(s.mu);
            // device memory of the running lanes (their reservations)
            auto busy_bytes = [&] {
                size_t t = 0;
                for (size_t i = 0; i < s.busy.size(); ++i)
                    if (s.busy[i]) t += s.reserved[i];
                return t;
            };
            // the head fits once idle lanes give their workspaces back
            s.cv_work.wait(lk, [&] {
                return s.stopping ||
                       (!s.paused && !s.pending.empty() && busy_bytes() + kGroupFixedBytes +
                                                      s.pending.front()->footprint <=
                                                  s.cfg.hbm_budget);
            });
            if (s.stopping) return;
            ServedRequest *head = s.pending.front();
            s.pending.pop_front();
            grp.push_back(head);
            size_t idle_held = 0;
            for (size_t i = 0; i < s.busy.size(); ++i)
                if (!s.busy[i] && i != lane) idle_held += s.held[i];
            // this lane's workspace may grow by the group's footprint; when
            // that does not fit beside what the lanes hold, the idle lanes
            // (this one included) free their workspaces first
            size_t base = busy_bytes() + idle_held + s.held[lane] + kGroupFixedBytes;
            if (base + head->footprint > s.cfg.hbm_budget) {
                for (size_t i = 0; i < s.busy.size(); ++i) {
                    if (s.busy[i] || s.held[i] == 0) continue;
                    Ctx &li = *s.lanes[i];
                    std::lock_guard<std::mutex> g(li.mu);
                    if (li.stream) (void)hipStreamSynchronize(li.stream);
                    for_each_buffer(li, [](Buffer &b) {
                        if (b.p) (void)hipFree(b.p);
                        b.p = nullptr;
                        b.cap = 0;
                        b.allocation = 0;
                    });
                    s.held[i] = 0;
                }
                base = busy_bytes() + kGroupFixedBytes;
            }
            size_t fp = head->footprint;
            const bool small = head->states <= s.cfg.batch_max_states;
            if (small) {
                for (auto it = s.pending.begin();
                     it != s.pending.end() && grp.size() < s.cfg.max_group;) {
                    ServedRequest *r = *it;
                    const size_t extra = r->footprint;
                    if (r->kind == head->kind && r->states <= s.cfg.batch_max_states &&
                        base + fp + extra <= s.cfg.hbm_budget) {
                        grp.push_back(r);
                        fp += extra;
                        it = s.pending.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            s.busy[lane] = 1;
            s.reserved[lane] = s.held[lane] + kGroupFixedBytes + fp;
            const auto now = Clock::now();
            for (auto *r : grp) r->t_start = now;
            if (grp.size() > 1 || small) s.groups++;
        }
        all = grp;
        bool uploaded = false;
        try {
            std::lock_guard<std::mutex> g(c.mu);
            g_last_error.clear();
            // inputs to the device on the lane's stream (asynchronous copies
            // from page-locked memory into the lane's own grow-only buffer)
            std::vector<ServedRequest *> ready;
            size_t in_total = 0;
            for (auto *r : grp) in_total += r->in_bytes;
            if (c.serve_in.ensure(in_total, "request inputs") != DFA_OK) {
                for (auto *r : grp) r->status = DFA_ENOMEM;
            } else {
                uint8_t *dev = c.serve_in.as<uint8_t>();
                (void)hipEventRecord(c.ev_up0, c.stream);
                for (auto *r : grp) {
                    if (hipMemcpyAsync(dev, r->host_in, r->in_bytes, hipMemcpyHostToDevice,
                                       c.stream) != hipSuccess) {
                        r->status = fail(DFA_EDEVICE, "copy of the request's inputs failed");
                        dev += r->in_bytes;
                        continue;
                    }
                    r->a.delta = reinterpret_cast<const uint32_t *>(dev);
                    r->a.accepting = dev + r->off_acc_a;
                    if (r->kind == DFA_REQ_EQUIVALENT) {
                        r->b.delta = reinterpret_cast<const uint32_t *>(dev + r->off_delta_b);
                        r->b.accepting = dev + r->off_acc_b;
                    }
                    dev += r->in_bytes;
                    ready.push_back(r);
                }
                (void)hipEventRecord(c.ev_up1, c.stream);
                uploaded = true;
            }
            grp.swap(ready);
            if (grp.size() == 1 && grp[0]->states > s.cfg.batch_max_states)
                run_solo(s, c, grp[0]);
            else if (!grp.empty())
                run_group(s, c, grp);
        } catch (const std::exception &e) {
            // a host allocation failed: the group's requests fail, the lane
            // goes on with the next ones
            const int code = dynamic_cast<const std::bad_alloc *>(&e) ? DFA_ENOMEM : DFA_EDEVICE;
            for (auto *r : all) {
                r->status = code;
                r->batched = false;
            }
        }
        (void)stream_sync(c);  // the input copies have completed
        if (uploaded) {
            float up_ms = 0.f;
            if (hipEventElapsedTime(&up_ms, c.ev_up0, c.ev_up1) == hipSuccess)
                for (auto *r : all) r->h2d_ms = up_ms;
        }
        for (auto *r : all) {
            if (r->host_in) s.pinned.put(r->host_in, r->host_cls);
            r->host_in = nullptr;
        }
        size_t now_held = 0;
        {
            std::lock_guard<std::mutex> g(c.mu);
            now_held = workspace_bytes(c);
        }
        {
            std::lock_guard<std::mutex> lk(s.mu);
            s.busy[lane] = 0;
            s.reserved[lane] = 0;
            s.held[lane] = now_held;
            for (auto *r : all) {
                if (!r->batched) s.solo++;
                finish(s, r, lk);
            }
        }
        s.cv_done.notify_all();
        s.cv_work.notify_all();
    }
}

void fill_result(const ServedRequest &r, dfa_result *out) {
    std::memset(out, 0, sizeof *out);
    out->status = r.status;
    out->verdict = r.verdict;
    out->num_blocks = r.num_blocks;
    out->rounds = r.rounds;
    out->blocks = r.kind == DFA_REQ_MINIMISE && r.status == DFA_OK ? r.blocks : nullptr;
    out->n = r.a.n;
    out->batched = r.batched ? 1 : 0;
    out->queue_ms = std::chrono::duration<double, std::milli>(r.t_start - r.t_submit).count();
    out->service_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_start).count();
    out->latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
    out->h2d_ms = r.h2d_ms;
    out->device_ms = r.device_ms;
    out->d2h_ms = r.d2h_ms;
}

// Runs an entry point's body so that no C++ exception crosses the C ABI: a
// failed host allocation becomes DFA_ENOMEM, anything else DFA_EDEVICE.
template <typename F>
int guarded(F &&body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(DFA_ENOMEM, "host memory allocation failed");
    } catch (const std::exception &e) {
        return fail(DFA_EDEVICE, "host error: %s", e.what());
    } catch (...) {
        return fail(DFA_EDEVICE, "host error");
    }
}

}  // namespace
}  // namespace dfamin

using namespace dfamin;

extern "C" {

int dfa_profile_enable(int on) {
    return guarded([&]() -> int {
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        c->profiling = on != 0;
        c->ktimes.clear();
        c->pending.clear();
        c->ev_used = 0;
        return DFA_OK;
    });
}

int dfa_profile_only(const char *name) {
    return guarded([&]() -> int {
        if (name && std::strlen(name) >= sizeof(dfa_kernel_time{}.name))
            return fail(DFA_EINVAL, "kernel name too long");
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        c->prof_only = name ? name : "";
        return DFA_OK;
    });
}

int dfa_profile_read(dfa_kernel_time *out, int cap, int *count) {
    return guarded([&]() -> int {
        if (!count || (cap > 0 && !out)) return fail(DFA_EINVAL, "NULL profile buffer");
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        int i = 0;
        for (const auto &kv : c->ktimes) {
            if (i < cap) {
                std::memset(&out[i], 0, sizeof out[i]);
                std::snprintf(out[i].name, sizeof out[i].name, "%s", kv.first.c_str());
                out[i].launches = kv.second.launches;
                out[i].total_ms = kv.second.ms;
                out[i].algorithmic_bytes = kv.second.bytes;
                out[i].states = kv.second.states;
                out[i].state_letters = kv.second.state_letters;
            }
            ++i;
        }
        *count = i;
        return DFA_OK;
    });
}

void dfa_tuning_default(dfa_tuning *t) {
    if (!t) return;
    std::memset(t, 0, sizeof *t);
    t->round_grid_cap = 8192;
    t->label_grid_cap = 2048;
    t->label_rounds = 2;
    t->cached_probe = 1;
    t->chunk = 4;
    t->batch_lds_states = 4096;
    t->insert_pair = 1;
    t->slice_min_states = 1u << 20;
}

int dfa_get_tuning(dfa_tuning *t) {
    return guarded([&]() -> int {
        if (!t) return fail(DFA_EINVAL, "tuning is NULL");
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        *t = c->tune;
        return DFA_OK;
    });
}

int dfa_set_tuning(const dfa_tuning *t) {
    return guarded([&]() -> int {
        if (!t) return fail(DFA_EINVAL, "tuning is NULL");
        if (t->label_rounds > 2 || t->cached_probe > 1 || t->chunk == 0 || t->chunk > 4096 ||
            t->round_grid_cap > (1u << 24) || t->label_grid_cap > (1u << 24) || t->hash_bits > 63 ||
            t->batch_lds_states > kSmallMaxStates || t->insert_pair > 1)
            return fail(DFA_EINVAL, "tuning value out of range");
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        c->tune = *t;
        const int dev = static_cast<int>(c - g_ctx);
        std::lock_guard<std::mutex> g(g_tuning_mu);
        g_tuning[dev] = *t;
        g_tuning_set[dev] = true;
        return DFA_OK;
    });
}

void dfa_options_default(dfa_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->tc_mode = DFA_TC_AUTO;
    opt->loop_mode = DFA_LOOP_GRAPH;
    opt->start = 0;
    opt->max_rounds = 0;
    opt->chunk = 0;
    opt->lds_stage = 2;
}

const char *dfa_last_error(void) { return g_last_error.c_str(); }

int dfa_device_info(char *name, size_t name_cap, int *compute_units, size_t *hbm_bytes) {
    return guarded([&]() -> int {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        hipDeviceProp_t p;
        HIP_TRY(hipGetDeviceProperties(&p, dev));
        if (name && name_cap) {
            std::snprintf(name, name_cap, "%s (%s)", p.name, p.gcnArchName);
        }
        if (compute_units) *compute_units = p.multiProcessorCount;
        if (hbm_bytes) *hbm_bytes = p.totalGlobalMem;
        return DFA_OK;
    });
}

int dfa_minimise_device(uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *accepting,
                        uint32_t *block_out, dfa_quotient *q_out, const dfa_options *opt,
                        dfa_stats *stats, void *stream) {
    return guarded([&]() -> int {
        g_last_error.clear();
        dfa_options o = resolve(opt);
        DFA_TRY(check_minimise(n, k, delta, accepting, block_out, q_out, o));
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        DFA_TRY(join_stream(*c, stream));
        if (stats) std::memset(stats, 0, sizeof *stats);
        return minimise_impl(*c, n, k, delta, accepting, block_out, q_out, o, stats);
    });
}

int dfa_minimise_device_fixed(uint32_t n, uint32_t k, const uint32_t *delta,
                              const uint8_t *accepting, uint32_t *block_out, dfa_quotient *q_out,
                              const dfa_options *opt, dfa_stats *stats, void *stream) {
    return guarded([&]() -> int {
        g_last_error.clear();
        dfa_options o = resolve(opt);
        DFA_TRY(check_minimise(n, k, delta, accepting, block_out, q_out, o));
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        if (dev < 0 || dev >= kMaxDevices)
            return fail(DFA_EDEVICE, "device index %d out of range", dev);
        Ctx &c = g_fixed[dev];
        CallScope lock(c.mu);
        DFA_TRY(init_fixed(c));
        {  // the device's tuning, as for every other call on it
            std::lock_guard<std::mutex> g(g_tuning_mu);
            if (g_tuning_set[dev]) c.tune = g_tuning[dev];
        }
        // (the same rule as build_slices, with every letter counted)
        const bool slices = c.tune.slice_min_states && n >= c.tune.slice_min_states &&
                            n <= (static_cast<uint64_t>(kPbMaxBuckets) << kPbSliceLog) &&
                            o.loop_mode != DFA_LOOP_PERSISTENT && o.tc_mode != DFA_TC_ON;
        const size_t need = fixed_plain_bytes(n, k, slices);
        if (need > kFixedScratchBytes)
            return fail(DFA_ENOMEM,
                        "n = %u, k = %u needs about %zu bytes of workspace; the fixed workspace "
                        "holds %zu",
                        n, k, need, kFixedScratchBytes);
        // a graph's instantiation allocates: chunks are launched one by one
        if (o.loop_mode == DFA_LOOP_GRAPH) o.loop_mode = DFA_LOOP_CHUNK;
        // every call carves its buffers afresh from the start of the array
        c.arena.used = 0;
        ++c.arena.generation;
        DFA_TRY(join_stream(c, stream));
        if (stats) std::memset(stats, 0, sizeof *stats);
        return minimise_impl(c, n, k, delta, accepting, block_out, q_out, o, stats);
    });
}

int dfa_minimise(uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *accepting,
                 uint32_t *block_out, dfa_quotient *q_out, const dfa_options *opt,
                 dfa_stats *stats) {
    return guarded([&]() -> int {
        g_last_error.clear();
        dfa_options o = resolve(opt);
        DFA_TRY(check_minimise(n, k, delta, accepting, block_out, q_out, o));
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        return minimise_host(*c, n, k, delta, accepting, block_out, q_out, o, stats);
    });
}

int dfa_equivalent_device(const dfa_view *a, const dfa_view *b, int *verdict,
                          const dfa_options *opt, dfa_stats *stats, void *stream) {
    return guarded([&]() -> int {
        g_last_error.clear();
        dfa_options o = resolve(opt);
        DFA_TRY(check_pair(a, b, verdict));
        DFA_TRY(check_options(o));
        if (o.prune) return fail(DFA_EINVAL, "prune applies to dfa_minimise only");
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        DFA_TRY(join_stream(*c, stream));
        if (stats) std::memset(stats, 0, sizeof *stats);
        return equivalent_impl(*c, *a, *b, verdict, o, stats);
    });
}

int dfa_equivalent(const dfa_view *a, const dfa_view *b, int *verdict, const dfa_options *opt,
                   dfa_stats *stats) {
    return guarded([&]() -> int {
        g_last_error.clear();
        dfa_options o = resolve(opt);
        DFA_TRY(check_pair(a, b, verdict));
        DFA_TRY(check_options(o));
        if (o.prune) return fail(DFA_EINVAL, "prune applies to dfa_minimise only");
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        return equivalent_host(*c, a, b, verdict, o, stats);
    });
}

int dfa_included_device(const dfa_view *a, const dfa_view *b, int *verdict,
                        uint64_t *pairs_visited, const dfa_options *opt, dfa_stats *stats,
                        void *stream) {
    return guarded([&]() -> int {
        g_last_error.clear();
        dfa_options o = resolve(opt);
        DFA_TRY(check_pair(a, b, verdict));
        DFA_TRY(check_options(o));
        if (o.prune) return fail(DFA_EINVAL, "prune applies to dfa_minimise only");
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        DFA_TRY(join_stream(*c, stream));
        return included_impl(*c, *a, *b, verdict, pairs_visited, stats);
    });
}

int dfa_included(const dfa_view *a, const dfa_view *b, int *verdict, uint64_t *pairs_visited,
                 const dfa_options *opt, dfa_stats *stats) {
    return guarded([&]() -> int {
        g_last_error.clear();
        dfa_options o = resolve(opt);
        DFA_TRY(check_pair(a, b, verdict));
        DFA_TRY(check_options(o));
        if (o.prune) return fail(DFA_EINVAL, "prune applies to dfa_minimise only");
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        auto t0 = std::chrono::steady_clock::now();
        dfa_view da, db;
        DFA_TRY(stage_view(*c, c->stage_delta, c->stage_acc, a, da));
        DFA_TRY(stage_view(*c, c->stage_delta_b, c->stage_acc_b, b, db));
        HIP_TRY(stream_sync(*c));
        const double h2d = ms_since(t0);
        int rc = included_impl(*c, da, db, verdict, pairs_visited, stats);
        if (stats) stats->h2d_ms = h2d;
        return rc;
    });
}


int dfa_minimise_batch_device(uint32_t count, const dfa_view *dfas, uint32_t *blocks_concat,
                              const uint64_t *block_offsets, uint32_t *num_blocks,
                              uint32_t *rounds, const dfa_options *opt, dfa_batch_stats *stats,
                              void *stream) {
    return guarded([&]() -> int {
        g_last_error.clear();
        dfa_options o = resolve(opt);
        DFA_TRY(check_views(count, dfas, "dfas"));
        DFA_TRY(check_batch_options(o));
        if (!blocks_concat) return fail(DFA_EINVAL, "blocks_concat is NULL");
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        DFA_TRY(join_stream(*c, stream));
        if (stats) std::memset(stats, 0, sizeof *stats);
        return minimise_batch_impl(*c, count, dfas, blocks_concat, block_offsets, num_blocks, rounds,
                                   o, stats);
    });
}

int dfa_minimise_batch(uint32_t count, const dfa_view *dfas, uint32_t *blocks_concat,
                       const uint64_t *block_offsets, uint32_t *num_blocks, uint32_t *rounds,
                       const dfa_options *opt, dfa_batch_stats *stats) {
    return guarded([&]() -> int {
        g_last_error.clear();
        dfa_options o = resolve(opt);
        DFA_TRY(check_views(count, dfas, "dfas"));
        DFA_TRY(check_batch_options(o));
        if (!blocks_concat) return fail(DFA_EINVAL, "blocks_concat is NULL");
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        if (stats) std::memset(stats, 0, sizeof *stats);
        std::vector<dfa_view> dev;
        double h2d = 0;
        const dfa_view *lists[1] = {dfas};
        DFA_TRY(stage_views(*c, count, lists, 1, dev, h2d));
        uint64_t total = 0;
        for (uint32_t i = 0; i < count; ++i) total += dfas[i].n;
        DFA_TRY(c->batch_out.ensure(total * sizeof(uint32_t), "batched outputs"));
        int rc = minimise_batch_impl(*c, count, dev.data(), c->batch_out.as<uint32_t>(), nullptr,
                                     num_blocks, rounds, o, stats);
        if (rc != DFA_OK && rc != DFA_ELIMIT) return rc;
        auto t0 = std::chrono::steady_clock::now();
        DFA_TRY(ensure_pinned_batch(*c, total * sizeof(uint32_t)));
        HIP_TRY(hipMemcpyAsync(c->pinned_batch, c->batch_out.p, total * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(stream_sync(*c));
        uint64_t pos = 0;
        const uint32_t *src = reinterpret_cast<const uint32_t *>(c->pinned_batch);
        std::vector<CopyJob> jobs(count);
        for (uint32_t i = 0; i < count; ++i) {
            const uint64_t dst = block_offsets ? block_offsets[i] : pos;
            jobs[i] = {blocks_concat + dst, src + pos, dfas[i].n * sizeof(uint32_t)};
            pos += dfas[i].n;
        }
        parallel_copies(jobs);
        if (stats) {
            stats->h2d_ms = h2d;
            stats->d2h_ms = ms_since(t0);
        }
        return rc;
    });
}

int dfa_equivalent_batch_device(uint32_t count, const dfa_view *a, const dfa_view *b,
                                int32_t *verdicts, const dfa_options *opt,
                                dfa_batch_stats *stats, void *stream) {
    return guarded([&]() -> int {
        g_last_error.clear();
        dfa_options o = resolve(opt);
        DFA_TRY(check_views(count, a, "a"));
        DFA_TRY(check_views(count, b, "b"));
        DFA_TRY(check_batch_options(o));
        if (!verdicts) return fail(DFA_EINVAL, "verdicts is NULL");
        for (uint32_t i = 0; i < count; ++i)
            if (a[i].k != b[i].k) return fail(DFA_EINVAL, "pair %u: alphabet sizes differ", i);
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        DFA_TRY(join_stream(*c, stream));
        if (stats) std::memset(stats, 0, sizeof *stats);
        return equivalent_batch_impl(*c, count, a, b, verdicts, o, stats);
    });
}

int dfa_equivalent_batch(uint32_t count, const dfa_view *a, const dfa_view *b, int32_t *verdicts,
                         const dfa_options *opt, dfa_batch_stats *stats) {
    return guarded([&]() -> int {
        g_last_error.clear();
        dfa_options o = resolve(opt);
        DFA_TRY(check_views(count, a, "a"));
        DFA_TRY(check_views(count, b, "b"));
        DFA_TRY(check_batch_options(o));
        if (!verdicts) return fail(DFA_EINVAL, "verdicts is NULL");
        for (uint32_t i = 0; i < count; ++i)
            if (a[i].k != b[i].k) return fail(DFA_EINVAL, "pair %u: alphabet sizes differ", i);
        Ctx *c = nullptr;
        DFA_TRY(get_ctx(c));
        CallScope lock(c->mu);
        DFA_TRY(init_ctx(*c));
        if (stats) std::memset(stats, 0, sizeof *stats);
        std::vector<dfa_view> dev;
        double h2d = 0;
        const dfa_view *lists[2] = {a, b};
        DFA_TRY(stage_views(*c, count, lists, 2, dev, h2d));
        int rc = equivalent_batch_impl(*c, count, dev.data(), dev.data() + count, verdicts, o, stats);
        if (stats) stats->h2d_ms = h2d;
        return rc;
    });
}


void dfa_server_config_default(dfa_server_config *cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->hbm_budget = 0;
    cfg->lanes = 4;
    cfg->max_group = 512;
    cfg->batch_max_states = 1u << 18;
    cfg->batch_round_budget = 12;
    cfg->tc_mode = DFA_TC_AUTO;
}

dfa_server *dfa_server_create(const dfa_server_config *cfg_in) {
    try {
        RelaxedCapture relaxed;
        g_last_error.clear();
        dfa_server_config cfg;
        dfa_server_config_default(&cfg);
        if (cfg_in) cfg = *cfg_in;
        if (cfg.lanes == 0 || cfg.lanes > 16 || cfg.max_group == 0 || cfg.batch_round_budget < 3 ||
            cfg.tc_mode < DFA_TC_OFF || cfg.tc_mode > DFA_TC_AUTO) {
            fail(DFA_EINVAL, "bad server configuration");
            return nullptr;
        }
        auto s = std::make_unique<Server>();
        if (hipGetDevice(&s->device) != hipSuccess) {
            fail(DFA_EDEVICE, "no HIP device");
            return nullptr;
        }
        if (cfg.hbm_budget == 0) {
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
                fail(DFA_EDEVICE, "hipMemGetInfo failed");
                return nullptr;
            }
            cfg.hbm_budget = free_b / 2;
        }
        s->cfg = cfg;
        s->paused = cfg.paused != 0;
        {
            Ctx *dc = nullptr;
            if (get_ctx(dc) != DFA_OK) return nullptr;
            CallScope lock(dc->mu);
            if (init_ctx(*dc) != DFA_OK) return nullptr;
            s->tune = dc->tune;
        }
        s->t_created = Clock::now();
        try {
            for (uint32_t i = 0; i < cfg.lanes; ++i) s->lanes.push_back(std::make_unique<Ctx>());
            s->held.assign(cfg.lanes, 0);
            s->reserved.assign(cfg.lanes, 0);
            s->busy.assign(cfg.lanes, 0);
            Server *raw = s.get();
            for (uint32_t i = 0; i < cfg.lanes; ++i) s->workers.emplace_back(lane_main, raw, i);
        } catch (const std::exception &e) {
            // stop the lanes that did start before the server goes away
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->stopping = true;
            }
            s->cv_work.notify_all();
            for (auto &t : s->workers) t.join();
            for (auto &l : s->lanes) release_ctx(*l);
            fail(DFA_ENOMEM, "starting the server lanes failed: %s", e.what());
            return nullptr;
        }
        return reinterpret_cast<dfa_server *>(s.release());
    } catch (const std::exception &e) {
        fail(DFA_ENOMEM, "creating the server failed: %s", e.what());
        return nullptr;
    }
}

int dfa_server_footprint(const dfa_server *handle, const dfa_request *req, size_t *bytes) {
    return guarded([&]() -> int {
        g_last_error.clear();
        const Server *s = reinterpret_cast<const Server *>(handle);
        if (!s || !req || !bytes) return fail(DFA_EINVAL, "NULL server, request or bytes");
        if (req->kind != DFA_REQ_MINIMISE && req->kind != DFA_REQ_EQUIVALENT)
            return fail(DFA_EINVAL, "unknown request kind %d", req->kind);
        const uint64_t states =
            static_cast<uint64_t>(req->a.n) + (req->kind == DFA_REQ_EQUIVALENT ? req->b.n : 0u);
        *bytes = request_footprint(states, req->a.k, s->cfg.tc_mode != DFA_TC_OFF) +
                 kGroupFixedBytes;
        return DFA_OK;
    });
}

int dfa_server_submit(dfa_server *handle, const dfa_request *req, uint64_t *ticket) {
    return guarded([&]() -> int {
        RelaxedCapture relaxed;  // page-locked staging may be allocated here
        g_last_error.clear();
        Server *s = reinterpret_cast<Server *>(handle);
        if (!s || !req || !ticket) return fail(DFA_EINVAL, "NULL server, request or ticket");
        if (req->kind != DFA_REQ_MINIMISE && req->kind != DFA_REQ_EQUIVALENT)
            return fail(DFA_EINVAL, "unknown request kind %d", req->kind);
        DFA_TRY(check_view(&req->a, "a"));
        if (req->kind == DFA_REQ_EQUIVALENT) {
            DFA_TRY(check_view(&req->b, "b"));
            if (req->a.k != req->b.k) return fail(DFA_EINVAL, "alphabet sizes differ");
        }
        auto r = std::make_unique<ServedRequest>();
        r->kind = req->kind;
        const bool two = req->kind == DFA_REQ_EQUIVALENT;
        auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
        const size_t da = static_cast<size_t>(req->a.n) * req->a.k * sizeof(uint32_t);
        const size_t db = two ? static_cast<size_t>(req->b.n) * req->b.k * sizeof(uint32_t) : 0;
        r->in_bytes = al(da) + al(req->a.n) + (two ? al(db) + al(req->b.n) : 0);
        r->states = req->a.n + (two ? req->b.n : 0);
        r->footprint = request_footprint(r->states, req->a.k, s->cfg.tc_mode != DFA_TC_OFF);
        if (r->footprint + kGroupFixedBytes > s->cfg.hbm_budget) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->rejected++;
            return fail(DFA_ENOMEM, "request needs ~%zu bytes of device memory, budget is %zu",
                        r->footprint + kGroupFixedBytes, s->cfg.hbm_budget);
        }
        // the inputs are copied now (page-locked, so the lane's upload is an
        // asynchronous DMA), so the caller may free them on return
        r->off_acc_a = al(da);
        r->off_delta_b = r->off_acc_a + al(req->a.n);
        r->off_acc_b = r->off_delta_b + al(db);
        uint8_t *host = static_cast<uint8_t *>(s->pinned.get(r->in_bytes, r->host_cls));
        if (!host) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->rejected++;
            return fail(DFA_ENOMEM, "page-locked host allocation of %zu bytes failed", r->in_bytes);
        }
        r->host_in = host;
        parallel_copy(host, req->a.delta, da);
        std::memcpy(host + r->off_acc_a, req->a.accepting, req->a.n);
        r->a = req->a;
        if (two) {
            parallel_copy(host + r->off_delta_b, req->b.delta, db);
            std::memcpy(host + r->off_acc_b, req->b.accepting, req->b.n);
            r->b = req->b;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next_ticket++;
        r->t_submit = Clock::now();
        *ticket = r->ticket;
        s->pending.push_back(r.get());
        s->requests.emplace(r->ticket, std::move(r));
        s->submitted++;
        s->cv_work.notify_one();
        return DFA_OK;
    });
}

int dfa_server_poll(dfa_server *handle, uint64_t ticket, dfa_result *out) {
    return guarded([&]() -> int {
        Server *s = reinterpret_cast<Server *>(handle);
        if (!s || !out) return fail(DFA_EINVAL, "NULL server or result");
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->requests.find(ticket);
        if (it == s->requests.end()) return fail(DFA_EINVAL, "unknown ticket %llu",
                                                 static_cast<unsigned long long>(ticket));
        if (!it->second->done) return DFA_EAGAIN;
        fill_result(*it->second, out);
        return DFA_OK;
    });
}

int dfa_server_wait(dfa_server *handle, uint64_t ticket, dfa_result *out) {
    return guarded([&]() -> int {
        Server *s = reinterpret_cast<Server *>(handle);
        if (!s || !out) return fail(DFA_EINVAL, "NULL server or result");
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->requests.find(ticket);
        if (it == s->requests.end()) return fail(DFA_EINVAL, "unknown ticket %llu",
                                                 static_cast<unsigned long long>(ticket));
        ServedRequest *r = it->second.get();
        // dfa_server_destroy cancels waiting requests and then waits for
        // every waiter to leave before it frees the server
        ++s->waiters;
        s->cv_done.wait(lk, [&] { return r->done; });
        fill_result(*r, out);
        // a cancelled request's result goes away with the server
        if (r->status == DFA_ECANCELED) out->blocks = nullptr;
        if (--s->waiters == 0) s->cv_left.notify_all();
        return DFA_OK;
    });
}

int dfa_server_resume(dfa_server *handle) {
    return guarded([&]() -> int {
        Server *s = reinterpret_cast<Server *>(handle);
        if (!s) return fail(DFA_EINVAL, "NULL server");
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->paused = false;
        }
        s->cv_work.notify_all();
        return DFA_OK;
    });
}

int dfa_result_release(dfa_server *handle, uint64_t ticket) {
    return guarded([&]() -> int {
        RelaxedCapture relaxed;
        Server *s = reinterpret_cast<Server *>(handle);
        if (!s) return fail(DFA_EINVAL, "NULL server");
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->requests.find(ticket);
        if (it == s->requests.end() || !it->second->done)
            return fail(DFA_EINVAL, "ticket %llu is unknown or not finished",
                        static_cast<unsigned long long>(ticket));
        if (it->second->blocks) s->pinned.put(it->second->blocks, it->second->blocks_cls);
        s->requests.erase(it);
        return DFA_OK;
    });
}

int dfa_server_get_stats(dfa_server *handle, dfa_server_stats *out) {
    return guarded([&]() -> int {
        Server *s = reinterpret_cast<Server *>(handle);
        if (!s || !out) return fail(DFA_EINVAL, "NULL server or stats");
        std::lock_guard<std::mutex> lk(s->mu);
        std::memset(out, 0, sizeof *out);
        out->submitted = s->submitted;
        out->completed = s->completed;
        out->rejected = s->rejected;
        out->batched_groups = s->groups;
        out->solo_runs = s->solo;
        out->pending = s->pending.size();
        size_t in_use = 0;
        for (size_t i = 0; i < s->busy.size(); ++i) in_use += s->busy[i] ? s->reserved[i] : s->held[i];
        out->hbm_in_use = in_use;
        out->hbm_budget = s->cfg.hbm_budget;
        out->waiting_threads = s->waiters;
        std::vector<double> lat = s->latencies;
        if (!lat.empty()) {
            std::sort(lat.begin(), lat.end());
            auto pct = [&](double p) {
                size_t i = static_cast<size_t>(p * (lat.size() - 1) + 0.5);
                return lat[std::min(i, lat.size() - 1)];
            };
            out->p50_ms = pct(0.50);
            out->p99_ms = pct(0.99);
            double sum = 0;
            for (double v : lat) sum += v;
            out->mean_ms = sum / lat.size();
        }
        out->uptime_s = std::chrono::duration<double>(Clock::now() - s->t_created).count();
        out->requests_per_s = out->uptime_s > 0 ? s->completed / out->uptime_s : 0.0;
        return DFA_OK;
    });
}

void dfa_server_destroy(dfa_server *handle) {
    try {
        RelaxedCapture relaxed;
        Server *s = reinterpret_cast<Server *>(handle);
        if (!s) return;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stopping = true;
            for (ServedRequest *r : s->pending) {
                r->status = DFA_ECANCELED;
                r->t_start = Clock::now();
                r->done = true;
                r->t_done = r->t_start;
            }
            s->pending.clear();
        }
        s->cv_work.notify_all();
        s->cv_done.notify_all();
        for (auto &t : s->workers) t.join();
        {
            // threads blocked in dfa_server_wait have seen their request
            // finish or be cancelled; the server is freed once they left
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_done.notify_all();
            s->cv_left.wait(lk, [&] { return s->waiters == 0; });
        }
        (void)hipSetDevice(s->device);
        for (auto &c : s->lanes) release_ctx(*c);
        // host copies of cancelled requests and unreleased results go back to
        // the pool, which the server frees
        for (auto &kv : s->requests) {
            if (kv.second->host_in) s->pinned.put(kv.second->host_in, kv.second->host_cls);
            if (kv.second->blocks) s->pinned.put(kv.second->blocks, kv.second->blocks_cls);
            kv.second->host_in = nullptr;
            kv.second->blocks = nullptr;
        }
        delete s;
    } catch (...) {
        // nothing may cross the C ABI; what was not freed stays allocated
    }
}

}  // extern "C"
