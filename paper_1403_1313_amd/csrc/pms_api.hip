// pms_api.hip -- host side of the C ABI declared in include/pms.h.
//
// One context per device holds the stream, the workspace (device buffers and
// pinned host mirrors that only grow), the current launch configuration, the
// captured graph of the last batched layout, and the counters of the last
// solve.  Host-level calls take the context lock; nothing is retained from
// the caller's buffers after a call returns.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <fstream>
#include <mutex>
#include <numeric>
#include <chrono>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "pms.h"
#include "pms_internal.h"

namespace {
// A roctx range around every entry point that does device work, named after
// it: a profiler's marker trace (`rocprofv3 --marker-trace`) then shows each
// call, and each serving step (one pms_step_launch), beside its kernels.
// Without a profiler attached a range costs a call into the roctx library.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

#define PMS_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? PMS_ERR_NOMEM : PMS_ERR_DEVICE,       \
                        std::string(#call) + ": " + hipGetErrorString(e_));               \
    } while (0)

#define PMS_TRY(expr)                 \
    do {                              \
        int s_ = (expr);              \
        if (s_ != PMS_OK) return s_;  \
    } while (0)

// Forced failure for tests of error propagation: PMS_TEST_FAIL_NEXT=<status>
// makes the next call of an entry point that does device work return that
// status (the variable is then cleared); <status>:<entry point name> aims it
// at the next call of that entry point only (others leave it set).  Checked
// after argument validation, before any device work.
int test_hook(const char* entry) {
    const char* v = getenv("PMS_TEST_FAIL_NEXT");
    if (!v || !*v) return PMS_OK;
    const char* colon = strchr(v, ':');
    if (colon && strcmp(colon + 1, entry) != 0) return PMS_OK;
    const int s = atoi(v);
    unsetenv("PMS_TEST_FAIL_NEXT");
    if (s <= PMS_OK || s > PMS_ERR_DEVICE) return PMS_OK;
    return fail(s, "failure injected by PMS_TEST_FAIL_NEXT");
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Buffers that only grow.
// ---------------------------------------------------------------------------
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    int ensure(size_t bytes) {
        if (bytes <= cap) return PMS_OK;
        size_t want = std::max(bytes, cap + cap / 2);
        want = align_up(want, 1 << 16);
        if (p) {
            (void)hipFree(p);
            p = nullptr;
            cap = 0;
        }
        PMS_HIP(hipMalloc(&p, want));
        cap = want;
        return PMS_OK;
    }
    hipError_t release() {
        const hipError_t e = p ? hipFree(p) : hipSuccess;
        p = nullptr;
        cap = 0;
        return e;
    }
    template <typename T>
    T* as(size_t byte_off = 0) const { return reinterpret_cast<T*>(static_cast<char*>(p) + byte_off); }
};

struct HostBuf {
    void* p = nullptr;
    size_t cap = 0;
    int ensure(size_t bytes) {
        if (bytes <= cap) return PMS_OK;
        size_t want = align_up(std::max(bytes, cap + cap / 2), 1 << 16);
        if (p) {
            (void)hipHostFree(p);
            p = nullptr;
            cap = 0;
        }
        PMS_HIP(hipHostMalloc(&p, want, hipHostMallocDefault));
        cap = want;
        return PMS_OK;
    }
    hipError_t release() {
        const hipError_t e = p ? hipHostFree(p) : hipSuccess;
        p = nullptr;
        cap = 0;
        return e;
    }
    template <typename T>
    T* as(size_t byte_off = 0) const { return reinterpret_cast<T*>(static_cast<char*>(p) + byte_off); }
};

// ---------------------------------------------------------------------------
// Configuration.
// ---------------------------------------------------------------------------
pms_config default_config() {
    pms_config c;
    c.chunk = 1u << 12;   // one block of 4096 candidates at least; target_items sets the rest
    c.wg_waves = 4;
    c.wgs_per_cu = 0;
    c.tail_split = 0;
    c.variant = PMS_VARIANT_AUTO;
    c.filter = PMS_FILTER_DEFAULT;
    return c;
}

bool config_ok(const pms_config& c) {
    return c.chunk >= 64 && c.chunk % 64 == 0 && c.chunk <= (1u << 24) && c.wg_waves >= 1 &&
           c.wg_waves <= 16 && c.wgs_per_cu <= 64 && c.tail_split <= 64 &&
           c.variant <= PMS_VARIANT_GROUP64 && c.filter <= PMS_FILTER_OFF;
}

pms_config resolve(const pms_config* c, const pms_config& cur) {
    if (!c) return cur;
    pms_config r = *c;
    const pms_config dflt = default_config();
    if (r.chunk == 0) r.chunk = dflt.chunk;
    if (r.wg_waves == 0) r.wg_waves = dflt.wg_waves;
    return r;
}

// ---------------------------------------------------------------------------
// Per-instance planning.
// ---------------------------------------------------------------------------
struct Shape {
    int32_t n, t, l, d;              // t: the longest row
    const int32_t* lens = nullptr;   // per-row lengths (pms_solve_ex); null: every row has t
    uint32_t flags = 0;              // pms_input_flag bits
    int32_t row_len(int32_t r) const { return lens ? lens[r] : t; }
    // Window slots of a row in the table: the longest row's windows, twice
    // with both strands.
    int32_t slots() const { return (t - l + 1) * ((flags & PMS_INPUT_BOTH_STRANDS) ? 2 : 1); }
    // The row length whose t-l+1 windows fill those slots (for window_stride).
    int32_t table_t() const { return slots() + l - 1; }
};

int validate_shape(int32_t n, int32_t t, int32_t l, int32_t d) {
    if (n < 1 || n > PMS_MAX_N) return fail(PMS_ERR_INVALID, "n out of range [1, 64]");
    if (l < 1 || l > PMS_MAX_L) return fail(PMS_ERR_INVALID, "l out of range [1, 16]");
    if (t < l || t > PMS_MAX_T) return fail(PMS_ERR_INVALID, "t out of range [l, 2^17]");
    if (d < 0 || d > l) return fail(PMS_ERR_INVALID, "d out of range [0, l]");
    return PMS_OK;
}

int validate_rows(const char* const* seqs, int32_t n, int32_t t) {
    if (!seqs) return fail(PMS_ERR_INVALID, "seqs is NULL");
    for (int32_t i = 0; i < n; ++i) {
        const char* r = seqs[i];
        if (!r) return fail(PMS_ERR_INVALID, "seqs[" + std::to_string(i) + "] is NULL");
        // Branch-free pass over the row (the compiler vectorises it); the
        // position is looked up only for the error message.
        const unsigned char* u = reinterpret_cast<const unsigned char*>(r);
        unsigned bad = 0;
        for (int32_t j = 0; j < t; ++j) {
            const unsigned c = u[j] | 0x20u;
            bad |= static_cast<unsigned>(c != 'a') & static_cast<unsigned>(c != 'c') &
                   static_cast<unsigned>(c != 'g') & static_cast<unsigned>(c != 't');
        }
        if (bad) {
            for (int32_t j = 0; j < t; ++j) {
                const unsigned c = u[j] | 0x20u;
                if (c != 'a' && c != 'c' && c != 'g' && c != 't')
                    return fail(PMS_ERR_INVALID, "byte " + std::to_string(j) + " of sequence " +
                                                     std::to_string(i) + " is not A/C/G/T");
            }
        }
    }
    return PMS_OK;
}

// Rows of their own lengths under pms_input_flag options.  N/n is a valid
// byte only with PMS_INPUT_MASK_N.  *empty is set when some row has no window
// free of N (its instance then has no motifs).
int validate_rows_ex(const char* const* seqs, int32_t n, const int32_t* lens, int32_t l,
                     uint32_t flags, bool* empty) {
    if (!seqs) return fail(PMS_ERR_INVALID, "seqs is NULL");
    const bool mask_n = (flags & PMS_INPUT_MASK_N) != 0;
    *empty = false;
    for (int32_t i = 0; i < n; ++i) {
        const unsigned char* u = reinterpret_cast<const unsigned char*>(seqs[i]);
        if (!u) return fail(PMS_ERR_INVALID, "seqs[" + std::to_string(i) + "] is NULL");
        int32_t run = 0, best = 0;  // longest stretch without N
        for (int32_t j = 0; j < lens[i]; ++j) {
            const unsigned c = u[j] | 0x20u;
            const bool base = c == 'a' || c == 'c' || c == 'g' || c == 't';
            if (!base && !(mask_n && c == 'n'))
                return fail(PMS_ERR_INVALID, "byte " + std::to_string(j) + " of sequence " +
                                                 std::to_string(i) + " is not A/C/G/T" +
                                                 (mask_n ? "/N" : ""));
            run = base ? run + 1 : 0;
            best = std::max(best, run);
        }
        if (best < l) *empty = true;
    }
    return PMS_OK;
}

int32_t window_stride(int32_t t, int32_t l, int32_t layout) {
    if (l < 1 || t < l) return 0;
    const size_t nw = static_cast<size_t>(t - l + 1);
    if (layout == PMS_LAYOUT_PLANES) return static_cast<int32_t>(align_up(nw, 16));
    if (l < 2) return 0;
    return static_cast<int32_t>((nw + 31) / 32 * 2 * l);
}

// Probability that a uniform random window lies within d of a fixed l-mer,
// and the expected survivors / sequence scans under independent uniform
// background.  Used only to size buffers and order work.
struct Estimate {
    double motifs;      // expected |M|
    double visits;      // expected sequence scans per candidate
};

Estimate estimate(const Shape& s) {
    double ball = 0, binom = 1;
    for (int k = 0; k <= s.d; ++k) {
        if (k > 0) binom = binom * (s.l - k + 1) / k;
        ball += binom * std::pow(3.0, k);
    }
    const double cands = std::ldexp(1.0, 2 * s.l);
    const double p = ball / cands;
    const double nw = s.slots();
    const double ps = 1.0 - std::pow(1.0 - p, nw);
    double ev = 0, pk = 1;
    for (int k = 0; k < s.n; ++k) {
        ev += pk;
        pk *= ps;
    }
    return {cands * pk + 1.0, ev};
}

// Batch::out_cap value asking for no device output at all (a size query:
// the kernel's count is exact without it).
constexpr uint64_t kCountOnly = ~0ull;
// Batches of more instances than this bring their codes back through one
// device-side gather and one copy instead of a copy per instance.
constexpr size_t kGatherMin = 4;

// Device output slots reserved for one instance before its count is known.
// PMS_TEST_DEVICE_CAP=<k> caps the reservation (tests of the rerun path).
uint64_t output_capacity(const Shape& s) {
    const double cands = std::ldexp(1.0, 2 * s.l);
    const double e = estimate(s).motifs;
    uint64_t want = static_cast<uint64_t>(std::min(cands, 8.0 * e + 4096.0));
    if (const char* v = getenv("PMS_TEST_DEVICE_CAP")) {
        const long long k = atoll(v);
        if (k > 0 && static_cast<uint64_t>(k) < want) want = static_cast<uint64_t>(k);
    }
    return want;
}

// ---------------------------------------------------------------------------
// Device context.
// ---------------------------------------------------------------------------
struct Batch {
    // host-side description of one launch
    std::vector<Shape> shape;
    std::vector<const char* const*> rows;
    std::vector<size_t> raw_off, win_off, out_off;
    std::vector<uint64_t> out_cap;
    std::vector<pms_win_job> jobs;
    std::vector<pms_work_item> work;
    std::vector<uint32_t> items_per_inst;
    size_t raw_bytes = 0, win_words = 0, out_words = 0;
    int32_t max_n = 1, max_t = 1;
    uint32_t variant = PMS_VARIANT_LANE;  // kernel variant chosen for this launch
    uint32_t flags = 0;                   // PMS_LAUNCH_* flags of the search launch
    // meta layout (bytes) inside d_meta / h_meta
    size_t off_insts = 0, off_jobs = 0, off_work = 0, off_state = 0, off_ctr = 0, off_bad = 0,
           meta_bytes = 0;
};

// Shape of one search launch.
struct Shape2 {
    uint32_t grid = 0, waves = 0;
    uint32_t q_words = 0;          // per-lane kernel: LDS queue words per wavefront
    pms::GroupQueues gq{0, nullptr, 0};
};

struct Ctx {
    std::mutex mu;
    bool ready = false;            // stream and events created (init_ctx)
    bool dev_ready = false;        // device properties and scratch address (init_device)
    void* scratch = nullptr;       // this device's fixed scratch (device address)
    size_t scratch_bytes = 0;
    int device = 0;
    int cus = 0;
    size_t lds_per_block = 65536;
    size_t lds_per_cu = 65536;
    std::string arch;
    hipStream_t stream = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    DevBuf d_raw, d_win, d_out, d_meta, d_gq;
    HostBuf h_raw, h_meta, h_back, h_out;
    DevBuf d_gtab, d_gather;   // batch copy-back: gather table and compacted codes
    HostBuf h_gtab;
    pms_config cfg = default_config();
    pms_stats last{};
    bool last_pending = false;     // last stats still need the event times
    hipStream_t last_stream = nullptr;
    // graph cache
    hipGraphExec_t gexec = nullptr;
    std::string gsig;
    // device-level workspace for pms_solve_dev
    DevBuf dv_win, dv_meta, dv_gq;
    HostBuf hv_meta, hv_back;      // hv_back: state and counters copied after the launch
    hipEvent_t dv_copied = nullptr, dv_back = nullptr;
    bool dv_copy_live = false;
    // where the last pms_solve_dev left its state and counters (0 = none)
    size_t dv_state_off = 0, dv_ctr_off = 0;
    int32_t dv_nw = 0;
    bool dv_counters = false;
    uint32_t dv_variant = PMS_VARIANT_LANE;
    // pms_solve_dev plan of the last call: reused, and its window jobs and
    // work table left on the device, while calls repeat the same shape and
    // configuration and nothing else has written dv_meta.
    Batch dv_plan;
    std::string dv_key;
    bool dv_plan_valid = false;
    const void* dv_uploaded = nullptr;
    // entry time of the current host-level call (host_prep_ms)
    std::chrono::steady_clock::time_point t_call;
    // launch shapes by (variant, max_n, wg_waves, wgs_per_cu)
    std::map<uint64_t, Shape2> shapes;
    // pms_build_windows job tables: a ring of pinned and device slots, each
    // reused only once its copy (from kJobRing calls before) has run, so a
    // call never waits for work queued ahead of it on the stream.
    static constexpr int kJobRing = 8;
    static constexpr size_t kJobSlot = 4096;  // >= PMS_MAX_N jobs
    HostBuf bw_host;
    DevBuf bw_dev;
    hipEvent_t bw_ev[kJobRing] = {};
    bool bw_live[kJobRing] = {};
    int bw_next = 0;
    // neighbourhood-intersection method: bitmaps, window codes, ball masks
    DevBuf nb_m, nb_b, nb_codes, nb_deltas, nb_groups, nb_ne, nb_cand, nb_out, nb_count;
    DevBuf nb_tcount, nb_toff, nb_tcur, nb_rec, nb_part;
    int32_t nb_ball_l = -1, nb_ball_d = -1, nb_ball_size = 0, nb_nne = 0;
};

Ctx g_ctx;

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Work items a launch of `instances` instances is cut into, per wavefront
// the device can hold resident: about 8 for one instance and 32 for a
// batch.  Every claim is a device-scope atomic on one counter, and claims
// of one instance's small items serialize there ((15,4): 131072 items of
// 8192 candidates 1.63 ms, 65536 of 16384 0.98 ms, 32768 of 32768 0.93 ms);
// a batch keeps finer items so that its short instances finish early.
uint64_t target_items(const Ctx& c, size_t instances) {
    return static_cast<uint64_t>(std::max(c.cus, 1)) * 16u * (instances > 1 ? 32u : 8u);
}

// Device properties and the address of this device's copy of the fixed
// scratch (pms_solve_dev_noalloc): no stream, event or memory is created.
int init_device(Ctx& c) {
    if (c.dev_ready) return PMS_OK;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0)
        return fail(PMS_ERR_DEVICE, "no HIP device available");
    int dev = 0;
    if (const char* v = getenv("PMS_DEVICE")) dev = atoi(v);
    else (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= count) return fail(PMS_ERR_DEVICE, "PMS_DEVICE out of range");
    PMS_HIP(hipSetDevice(dev));
    hipDeviceProp_t prop;
    PMS_HIP(hipGetDeviceProperties(&prop, dev));
    c.device = dev;
    c.cus = prop.multiProcessorCount;
    c.lds_per_block = prop.sharedMemPerBlock;
    c.lds_per_cu = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor
                                                         : prop.sharedMemPerBlock;
    c.arch = prop.gcnArchName;
    PMS_HIP(pms::noalloc_scratch(&c.scratch, &c.scratch_bytes));
    c.dev_ready = true;
    return PMS_OK;
}

int init_ctx(Ctx& c) {
    if (c.ready) return PMS_OK;
    PMS_TRY(init_device(c));
    PMS_HIP(hipSetDevice(c.device));
    PMS_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
    for (auto& e2 : c.ev) PMS_HIP(hipEventCreate(&e2));
    PMS_HIP(hipEventCreateWithFlags(&c.dv_copied, hipEventDisableTiming));
    PMS_HIP(hipEventCreateWithFlags(&c.dv_back, hipEventDisableTiming));
    c.ready = true;
    return PMS_OK;
}

int query_shape(Ctx& c, const pms_config& cfg, int32_t max_n, uint32_t variant, Shape2* out);

// Workgroup shape, grid and queue placement for a search launch (no
// workspace attached).  The kernel attribute and occupancy queries depend
// only on (variant, max_n, wg_waves, wgs_per_cu); their answers are kept.
int cached_shape(Ctx& c, const pms_config& cfg, int32_t max_n, uint32_t variant, Shape2* out) {
    const uint64_t key = (static_cast<uint64_t>(variant) << 48) |
                         (static_cast<uint64_t>(max_n) << 32) |
                         (static_cast<uint64_t>(cfg.wg_waves) << 16) | cfg.wgs_per_cu;
    auto hit = c.shapes.find(key);
    if (hit == c.shapes.end()) {
        Shape2 sh;
        PMS_TRY(query_shape(c, cfg, max_n, variant, &sh));
        hit = c.shapes.emplace(key, sh).first;
    }
    *out = hit->second;
    return PMS_OK;
}

// As cached_shape, with the stage queues that do not fit in LDS placed in
// `ws` (grown as needed).
int launch_shape(Ctx& c, const pms_config& cfg, int32_t max_n, uint32_t variant, DevBuf& ws,
                 Shape2* out) {
    PMS_TRY(cached_shape(c, cfg, max_n, variant, out));
    if (out->gq.gq_words) {
        PMS_TRY(ws.ensure(static_cast<size_t>(out->grid) * out->waves * out->gq.gq_words * 4));
        out->gq.gq = ws.as<uint32_t>();
    }
    return PMS_OK;
}

int query_shape(Ctx& c, const pms_config& cfg, int32_t max_n, uint32_t variant, Shape2* out) {
    const uint32_t stages = static_cast<uint32_t>(max_n > 1 ? max_n - 1 : 0);
    const void* fn = variant == PMS_VARIANT_LANE
                         ? pms::search_kernel_symbol()
                         : pms::search_group_kernel_symbol(variant == PMS_VARIANT_GROUP64 ? 3 : 2);
    uint32_t lds_stages = stages, gq_words = 0;
    size_t per_wave;
    if (variant == PMS_VARIANT_LANE) {
        per_wave = static_cast<size_t>(pms::queue_words(max_n, variant) + PMS_OUTBUF) * 4;
    } else {
        const int suffix = variant == PMS_VARIANT_GROUP64 ? 3 : 2;
        const uint32_t entry = pms::stage_queue_words(suffix);
        const uint32_t fixed = pms::wave_fixed_words(suffix);
        hipFuncAttributes attr;
        PMS_HIP(hipFuncGetAttributes(&attr, fn));
        const int vgprs = std::max(attr.numRegs, 8);
        const int per_simd = std::max(1, std::min(8, 512 / ((vgprs + 7) / 8 * 8)));
        const size_t budget = c.lds_per_cu / (4 * static_cast<size_t>(per_simd));
        const size_t fit = budget / 4 > fixed ? (budget / 4 - fixed) / entry : 0;
        lds_stages = std::min<uint32_t>(stages, static_cast<uint32_t>(fit));
        gq_words = (stages - lds_stages) * entry;
        per_wave = static_cast<size_t>(lds_stages * entry + fixed) * 4;
    }
    uint32_t w = cfg.wg_waves;
    if (variant == PMS_VARIANT_GROUP64) w = std::min<uint32_t>(w, PMS_GROUP64_MAX_THREADS / 64);
    while (w > 1 && per_wave * w > c.lds_per_block) --w;
    if (per_wave * w > c.lds_per_block)
        return fail(PMS_ERR_INVALID, "stage queues exceed the LDS of one workgroup");
    int per_cu = 0;
    PMS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * w, per_wave * w));
    if (per_cu < 1) per_cu = 1;
    if (cfg.wgs_per_cu > 0 && static_cast<int>(cfg.wgs_per_cu) < per_cu) per_cu = cfg.wgs_per_cu;
    out->grid = static_cast<uint32_t>(per_cu * c.cus);
    out->waves = w;
    out->q_words = variant == PMS_VARIANT_LANE ? pms::queue_words(max_n, variant) : 0;
    out->gq = {lds_stages, nullptr, gq_words};
    return PMS_OK;
}

// Item sizes of one instance that gets `share` of a launch's work items.
// Items start on multiples of 4096 candidates where the space allows (64
// groups of 64: the grouped kernel's stage-0 batches then share all but three
// prefix bases).  Items before head_end hold `size` candidates, the rest
// `small`.
struct ItemPlan {
    uint64_t total, size, small, head_end;
};

ItemPlan item_plan(const Shape& s, double share, const pms_config& cfg, uint64_t target_items) {
    ItemPlan p;
    p.total = 1ull << (2 * s.l);
    const uint64_t want_items = std::max<uint64_t>(1, static_cast<uint64_t>(share * target_items));
    const uint64_t unit = p.total >= 4096 ? 4096 : 64;
    uint64_t size = std::max<uint64_t>(cfg.chunk, (p.total + want_items - 1) / want_items);
    p.size = std::min<uint64_t>(align_up(size, unit), 1ull << 30);
    const uint64_t tail = align_up(p.total * cfg.tail_split / 64, unit);
    p.head_end = p.total - std::min(tail, p.total);
    p.small = std::max<uint64_t>(unit, align_up(p.size / 4, unit));
    return p;
}

// Cuts each instance's candidate range into work items.  Instances go in
// ascending order of estimated work (shortest first: the wavefronts take
// items in table order, so short instances complete early instead of
// behind the long ones; the launch still ends on items of one long
// instance, which all wavefronts share).  An instance receives a
// number of items in proportion to its share of the launch's estimated work,
// about `target_items` in all, and never items smaller than `chunk`
// candidates; inside an instance the last tail_split/64 of the range uses
// items a quarter of that size, so the launch ends with small items.
void build_work(Batch& b, const std::vector<int>& order, const std::vector<double>& cost,
                const pms_config& cfg, uint64_t target_items) {
    b.work.clear();
    b.items_per_inst.assign(b.shape.size(), 0);
    double total_cost = 0;
    for (int i : order) total_cost += cost[i];
    for (int i : order) {
        const double share = total_cost > 0 ? cost[i] / total_cost : 1.0;
        const ItemPlan p = item_plan(b.shape[i], share, cfg, target_items);
        uint64_t k = 0;
        while (k < p.total) {
            const uint64_t step = k < p.head_end ? p.size : p.small;
            const uint64_t len = std::min<uint64_t>(step, p.total - k);
            b.work.push_back({k, static_cast<uint32_t>(len), static_cast<uint32_t>(i)});
            b.items_per_inst[i]++;
            k += len;
        }
    }
}

// The kernel a launch uses: the requested variant when every instance allows
// it (GROUP needs l >= 2, GROUP64 l >= 3), otherwise the next smaller one.
uint32_t choose_variant(const std::vector<Shape>& shapes, uint32_t requested) {
    int32_t min_l = PMS_MAX_L;
    for (const Shape& s : shapes) min_l = std::min(min_l, s.l);
    uint32_t v = requested == PMS_VARIANT_AUTO ? PMS_VARIANT_GROUP64 : requested;
    if (v == PMS_VARIANT_GROUP64 && min_l < 3) v = PMS_VARIANT_GROUP;
    if (v == PMS_VARIANT_GROUP && min_l < 2) v = PMS_VARIANT_LANE;
    return v;
}

// Search-launch flags of a configuration.
uint32_t launch_flags(const pms_config& cfg) {
    return cfg.filter == PMS_FILTER_OFF ? PMS_LAUNCH_NO_FILTER : 0u;
}

// Lays out raw bytes, windows, outputs and the meta block for the instances.
// target_items: about how many work items the launch should have in all.
void plan_batch(Batch& b, const pms_config& cfg, uint64_t target_items) {
    const size_t m = b.shape.size();
    b.raw_off.resize(m);
    b.win_off.resize(m);
    b.out_off.resize(m);
    b.out_cap.resize(m);
    b.jobs.clear();
    b.raw_bytes = b.win_words = b.out_words = 0;
    b.max_n = 1;
    b.max_t = 1;
    b.variant = choose_variant(b.shape, cfg.variant);
    b.flags = launch_flags(cfg);
    const int32_t layout = b.variant == PMS_VARIANT_LANE ? PMS_LAYOUT_PLANES : PMS_LAYOUT_BITSLICED;
    std::vector<double> cost(m);
    for (size_t i = 0; i < m; ++i) {
        const Shape& s = b.shape[i];
        const int32_t stride = window_stride(s.table_t(), s.l, layout);
        b.raw_off[i] = b.raw_bytes;
        b.win_off[i] = b.win_words;
        b.out_off[i] = b.out_words;
        if (b.out_cap[i] == kCountOnly) b.out_cap[i] = 0;  // size query: no device codes
        else if (b.out_cap[i] == 0) b.out_cap[i] = output_capacity(s);
        size_t row_off = 0;  // rows are packed back to back
        for (int32_t r = 0; r < s.n; ++r) {
            b.jobs.push_back({b.raw_off[i] + row_off, b.win_off[i] + static_cast<size_t>(r) * stride,
                              s.row_len(r), s.l, stride, static_cast<int32_t>(i), layout,
                              static_cast<int32_t>(s.flags)});
            row_off += static_cast<size_t>(s.row_len(r));
        }
        b.raw_bytes += align_up(row_off, 256);
        b.win_words += static_cast<size_t>(s.n) * stride;
        b.out_words += align_up(b.out_cap[i], 64);
        b.max_n = std::max(b.max_n, s.n);
        b.max_t = std::max(b.max_t, s.t);
        cost[i] = std::ldexp(1.0, 2 * s.l) * s.slots() * estimate(s).visits;
    }
    std::vector<int> order(m);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] < cost[c]; });
    build_work(b, order, cost, cfg, target_items);
    // Per-call records first (instances, then state, counters and bad-byte
    // flags, which come back after the launch), then the plan's tables
    // (window jobs, work items): a call that reuses a plan uploads
    // [0, off_jobs) in one copy, and the results are [off_state, off_jobs).
    size_t off = 0;
    b.off_insts = off;
    off = align_up(off + m * sizeof(pms_dev_instance), 256);
    b.off_state = off;
    off = align_up(off + m * sizeof(pms_dev_state), 256);
    b.off_ctr = off;
    off = align_up(off + sizeof(pms_dev_counters), 256);
    b.off_bad = off;
    off = align_up(off + m * sizeof(uint32_t), 256);
    b.off_jobs = off;
    off = align_up(off + b.jobs.size() * sizeof(pms_win_job), 256);
    b.off_work = off;
    off = align_up(off + b.work.size() * sizeof(pms_work_item), 256);
    b.meta_bytes = off;
}

// Fills the pinned staging buffers for a planned batch.
int stage_batch(Ctx& c, Batch& b) {
    PMS_TRY(c.d_raw.ensure(std::max<size_t>(b.raw_bytes, 256)));
    PMS_TRY(c.d_win.ensure(std::max<size_t>(b.win_words * 4, 256)));
    PMS_TRY(c.d_out.ensure(std::max<size_t>(b.out_words * 4, 256)));
    PMS_TRY(c.d_meta.ensure(b.meta_bytes));
    PMS_TRY(c.h_raw.ensure(std::max<size_t>(b.raw_bytes, 256)));
    PMS_TRY(c.h_meta.ensure(b.meta_bytes));
    PMS_TRY(c.h_back.ensure(b.meta_bytes));
    const size_t m = b.shape.size();
    for (size_t i = 0; i < m; ++i) {
        const Shape& s = b.shape[i];
        char* dst = c.h_raw.as<char>(b.raw_off[i]);
        for (int32_t r = 0; r < s.n; ++r) {
            memcpy(dst, b.rows[i][r], static_cast<size_t>(s.row_len(r)));
            dst += s.row_len(r);
        }
    }
    memset(c.h_meta.p, 0, b.meta_bytes);
    pms_dev_instance* insts = c.h_meta.as<pms_dev_instance>(b.off_insts);
    pms_dev_state* state = c.h_meta.as<pms_dev_state>(b.off_state);
    for (size_t i = 0; i < m; ++i) {
        const Shape& s = b.shape[i];
        insts[i].windows = c.d_win.as<uint32_t>() + b.win_off[i];
        insts[i].out = c.d_out.as<uint32_t>() + b.out_off[i];
        insts[i].out_cap = b.out_cap[i];
        insts[i].n = s.n;
        insts[i].nw_stride = window_stride(
            s.table_t(), s.l, b.variant == PMS_VARIANT_LANE ? PMS_LAYOUT_PLANES : PMS_LAYOUT_BITSLICED);
        insts[i].l = s.l;
        insts[i].d = s.d;
        state[i].items_left = b.items_per_inst[i];
    }
    memcpy(c.h_meta.as<char>(b.off_jobs), b.jobs.data(), b.jobs.size() * sizeof(pms_win_job));
    memcpy(c.h_meta.as<char>(b.off_work), b.work.data(), b.work.size() * sizeof(pms_work_item));
    return PMS_OK;
}

hipError_t launch_variant(uint32_t variant, uint32_t flags, const pms_dev_instance* insts,
                          const pms_work_item* work, uint32_t n_work, pms_dev_state* state,
                          pms_dev_counters* ctr, const Shape2& sh, hipStream_t s) {
    if (variant == PMS_VARIANT_LANE)
        return pms::launch_search(insts, work, n_work, state, ctr, sh.q_words, sh.grid, sh.waves, s);
    return pms::launch_search_group(insts, work, n_work, state, ctr, sh.gq, sh.grid, sh.waves, s,
                                    variant == PMS_VARIANT_GROUP64 ? 3 : 2, flags);
}

// Enqueues copy-in, both kernels and copy-back of the state block on c.stream.
int enqueue_batch(Ctx& c, const Batch& b, bool timed, const Shape2& sh) {
    char* dm = c.d_meta.as<char>();
    PMS_HIP(hipMemcpyAsync(c.d_raw.p, c.h_raw.p, b.raw_bytes, hipMemcpyHostToDevice, c.stream));
    PMS_HIP(hipMemcpyAsync(dm, c.h_meta.p, b.meta_bytes, hipMemcpyHostToDevice, c.stream));
    if (timed) PMS_HIP(hipEventRecord(c.ev[0], c.stream));
    PMS_HIP(pms::launch_windows(reinterpret_cast<const pms_win_job*>(dm + b.off_jobs),
                                static_cast<int32_t>(b.jobs.size()), b.max_t,
                                c.d_raw.as<uint8_t>(), c.d_win.as<uint32_t>(),
                                reinterpret_cast<uint32_t*>(dm + b.off_bad), c.stream));
    if (timed) PMS_HIP(hipEventRecord(c.ev[1], c.stream));
    PMS_HIP(launch_variant(b.variant, b.flags, reinterpret_cast<const pms_dev_instance*>(dm + b.off_insts),
                           reinterpret_cast<const pms_work_item*>(dm + b.off_work),
                           static_cast<uint32_t>(b.work.size()),
                           reinterpret_cast<pms_dev_state*>(dm + b.off_state),
                           reinterpret_cast<pms_dev_counters*>(dm + b.off_ctr), sh, c.stream));
    if (timed) PMS_HIP(hipEventRecord(c.ev[2], c.stream));
    PMS_HIP(hipMemcpyAsync(c.h_back.as<char>(b.off_state), dm + b.off_state,
                           b.off_jobs - b.off_state, hipMemcpyDeviceToHost, c.stream));
    return PMS_OK;
}

std::string graph_signature(const Ctx& c, const Batch& b, const pms_config& cfg) {
    std::ostringstream o;
    o << c.d_raw.p << ':' << c.d_win.p << ':' << c.d_out.p << ':' << c.d_meta.p << ':'
      << c.h_raw.p << ':' << c.h_meta.p << ':' << c.h_back.p << ':' << b.raw_bytes << ':'
      << b.meta_bytes << ':' << b.off_state << ':' << b.jobs.size() << ':' << b.work.size()
      << ':' << b.max_n << ':' << b.max_t << ':' << cfg.chunk << ':' << cfg.wg_waves << ':'
      << cfg.wgs_per_cu << ':' << b.shape.size() << ':' << b.off_insts << ':' << b.off_jobs << ':'
      << b.off_work << ':' << b.off_ctr << ':' << b.off_bad << ':' << b.variant << ':' << b.flags;
    return o.str();
}

// Runs a staged batch: eagerly (timed with events) or through the graph.
int run_batch(Ctx& c, Batch& b, const pms_config& cfg, bool use_graph) {
    Shape2 sh;
    PMS_TRY(launch_shape(c, cfg, b.max_n, b.variant, c.d_gq, &sh));
    const uint32_t grid = sh.grid, waves = sh.waves;
    if (use_graph) {
        const std::string sig = graph_signature(c, b, cfg) + ":" +
                                std::to_string(reinterpret_cast<uintptr_t>(sh.gq.gq)) + ":" +
                                std::to_string(sh.gq.lds_stages) + ":" + std::to_string(grid);
        if (!c.gexec || sig != c.gsig) {
            if (c.gexec) {
                (void)hipGraphExecDestroy(c.gexec);
                c.gexec = nullptr;
            }
            PMS_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
            const int s = enqueue_batch(c, b, false, sh);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(c.stream, &graph);
            if (s != PMS_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return s;
            }
            PMS_HIP(e);
            const hipError_t ei = hipGraphInstantiate(&c.gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            PMS_HIP(ei);
            c.gsig = sig;
        }
        PMS_HIP(hipEventRecord(c.ev[0], c.stream));
        PMS_HIP(hipGraphLaunch(c.gexec, c.stream));
        PMS_HIP(hipEventRecord(c.ev[2], c.stream));
        PMS_HIP(hipStreamSynchronize(c.stream));
        float ms = 0;
        PMS_HIP(hipEventElapsedTime(&ms, c.ev[0], c.ev[2]));
        c.last.kernel_ms = ms;  // whole graph: copies + both kernels
        c.last.windows_ms = 0;
    } else {
        PMS_TRY(enqueue_batch(c, b, true, sh));
        PMS_HIP(hipStreamSynchronize(c.stream));
        float w_ms = 0, k_ms = 0;
        PMS_HIP(hipEventElapsedTime(&w_ms, c.ev[0], c.ev[1]));
        PMS_HIP(hipEventElapsedTime(&k_ms, c.ev[1], c.ev[2]));
        c.last.windows_ms = w_ms;
        c.last.kernel_ms = k_ms;
    }
    c.last.grid = grid;
    c.last.wg_waves = waves;
    c.last.chunk = cfg.chunk;
    c.last.variant = b.variant;
    c.last.work_items = static_cast<uint32_t>(b.work.size());
    c.last_pending = false;
    return PMS_OK;
}

// Ascending order of k motif codes of `bits` significant bits (2l).  Small
// sets go to std::sort; larger ones to a least-significant-digit radix sort
// with at most 11-bit digits (two passes up to l = 11, three up to l = 16),
// which is several times faster than a comparison sort at 10^5 codes.
void sort_codes(uint32_t* v, size_t k, int bits, std::vector<uint32_t>& tmp) {
    if (k < 4096 || bits <= 0) {
        std::sort(v, v + k);
        return;
    }
    const int passes = (bits + 10) / 11;
    const int w = (bits + passes - 1) / passes;
    const uint32_t buckets = 1u << w, digit = buckets - 1;
    tmp.resize(k);
    std::vector<size_t> hist(buckets);
    uint32_t* src = v;
    uint32_t* dst = tmp.data();
    for (int pass = 0; pass < passes; ++pass) {
        const int sh = pass * w;
        std::fill(hist.begin(), hist.end(), 0);
        for (size_t i = 0; i < k; ++i) ++hist[(src[i] >> sh) & digit];
        size_t sum = 0;
        for (uint32_t b = 0; b < buckets; ++b) {
            const size_t h = hist[b];
            hist[b] = sum;
            sum += h;
        }
        for (size_t i = 0; i < k; ++i) dst[hist[(src[i] >> sh) & digit]++] = src[i];
        std::swap(src, dst);
    }
    if (src != v) memcpy(v, src, k * 4);
}

// Candidate scan slots of a launch: 64 lanes x candidates per lane per
// batch; GROUP64's single-candidate batches hold one candidate per lane.
uint64_t candidate_slots(const pms_dev_counters& ctr, uint32_t variant) {
    const uint64_t singles = ctr.single_batches;
    return (ctr.batches - singles) * 64u * pms::candidates_per_lane(variant) + singles * 64u;
}

bool use_graph_default() {
    const char* v = getenv("PMS_NO_GRAPH");
    return !(v && *v && *v != '0');
}

// Host-level solve of a set of already validated instances.  caps[i] is the
// caller's capacity; outs[i] its buffer.  Fills counts and per-instance status.
int solve_instances(Ctx& c, const std::vector<Shape>& shapes,
                    const std::vector<const char* const*>& rows,
                    const std::vector<uint32_t*>& outs, const std::vector<uint64_t>& caps,
                    std::vector<int>& status, std::vector<uint64_t>& counts,
                    std::vector<double>& latency, bool use_graph) {
    const size_t m = shapes.size();
    const pms_config cfg = c.cfg;
    Batch b;
    b.shape = shapes;
    b.rows = rows;
    b.out_cap.resize(m);
    for (size_t i = 0; i < m; ++i) b.out_cap[i] = caps[i] == 0 ? kCountOnly : 0;
    plan_batch(b, cfg, target_items(c, m));
    PMS_TRY(stage_batch(c, b));
    const double prep_ms = ms_since(c.t_call);
    PMS_TRY(run_batch(c, b, cfg, use_graph));
    const auto t_back = std::chrono::steady_clock::now();
    counts.assign(m, 0);
    latency.assign(m, 0.0);
    status.assign(m, PMS_OK);
    const pms_dev_state* st = c.h_back.as<pms_dev_state>(b.off_state);
    const pms_dev_counters* ctr = c.h_back.as<pms_dev_counters>(b.off_ctr);
    const uint32_t* bad = c.h_back.as<uint32_t>(b.off_bad);
    uint64_t visits = 0, wcmp = 0;
    std::vector<size_t> rerun;
    for (size_t i = 0; i < m; ++i) {
        counts[i] = st[i].count;
        visits += st[i].visits;
        wcmp += st[i].visits * static_cast<uint64_t>(shapes[i].slots());
        latency[i] = st[i].t_done > ctr->t_start ? (st[i].t_done - ctr->t_start) * 1e-5 : 0.0;
        if (bad[i]) status[i] = fail(PMS_ERR_INVALID, "a byte is not A/C/G/T");
        if (st[i].items_left != 0 || ctr->error)
            return fail(PMS_ERR_DEVICE, "search ended with unfinished work items");
        if (caps[i] > 0 && counts[i] > b.out_cap[i]) rerun.push_back(i);
    }
    c.last.seq_visits = visits;
    c.last.window_compares = wcmp;
    c.last.batches = ctr->batches;
    c.last.single_batches = ctr->single_batches;
    c.last.filtered_batches = ctr->filtered_batches;
    c.last.filtered_groups = ctr->filtered_groups;
    c.last.candidate_slots = candidate_slots(*ctr, b.variant);
    c.last.reruns = 0;
    // Step a7.  Every instance's codes go to its segment of one pinned
    // buffer: asynchronous copies, one synchronisation.  Outputs larger than
    // the device estimate are solved again with the exact capacity (the count
    // is exact, so one rerun suffices) once those copies have landed.
    std::vector<size_t> seg(m + 1, 0);
    // (A size query, capacity 0, needs the count only: no codes come back.)
    for (size_t i = 0; i < m; ++i)
        seg[i + 1] = seg[i] + (status[i] == PMS_OK && caps[i] > 0 ? counts[i] : 0);
    PMS_TRY(c.h_out.ensure(std::max<size_t>(seg[m] * 4, 256)));
    uint32_t* const h_codes = c.h_out.as<uint32_t>();
    auto takes = [&](size_t i) {
        return status[i] == PMS_OK && caps[i] > 0 && counts[i] && counts[i] <= b.out_cap[i];
    };
    if (m > kGatherMin) {
        // Many instances: the device packs their codes into one array
        // (pms_gather_kernel) and one copy brings it back.
        PMS_TRY(c.h_gtab.ensure(m * 3 * sizeof(uint64_t)));
        PMS_TRY(c.d_gtab.ensure(m * 3 * sizeof(uint64_t)));
        PMS_TRY(c.d_gather.ensure(std::max<size_t>(seg[m] * 4, 256)));
        uint64_t* const tab = c.h_gtab.as<uint64_t>();
        for (size_t i = 0; i < m; ++i) {
            tab[3 * i] = b.out_off[i];
            tab[3 * i + 1] = seg[i];
            tab[3 * i + 2] = takes(i) ? counts[i] : 0;
        }
        PMS_HIP(hipMemcpyAsync(c.d_gtab.p, tab, m * 3 * sizeof(uint64_t), hipMemcpyHostToDevice,
                               c.stream));
        PMS_HIP(pms::launch_gather(c.d_out.as<uint32_t>(), c.d_gtab.as<uint64_t>(),
                                   static_cast<uint32_t>(m), c.d_gather.as<uint32_t>(), c.stream));
        if (seg[m])
            PMS_HIP(hipMemcpyAsync(h_codes, c.d_gather.p, seg[m] * 4, hipMemcpyDeviceToHost,
                                   c.stream));
    } else {
        for (size_t i = 0; i < m; ++i)
            if (takes(i))
                PMS_HIP(hipMemcpyAsync(h_codes + seg[i], c.d_out.as<uint32_t>() + b.out_off[i],
                                       counts[i] * 4, hipMemcpyDeviceToHost, c.stream));
    }
    PMS_HIP(hipStreamSynchronize(c.stream));
    for (size_t i : rerun) {
        if (status[i] != PMS_OK) continue;
        Batch r;
        r.shape = {shapes[i]};
        r.rows = {rows[i]};
        r.out_cap = {counts[i]};
        plan_batch(r, cfg, target_items(c, 1));
        PMS_TRY(stage_batch(c, r));
        PMS_TRY(run_batch(c, r, cfg, false));
        const pms_dev_state* rs = c.h_back.as<pms_dev_state>(r.off_state);
        if (rs[0].count != counts[i]) return fail(PMS_ERR_DEVICE, "rerun changed the motif count");
        PMS_HIP(hipMemcpy(h_codes + seg[i], c.d_out.as<uint32_t>(), counts[i] * 4,
                          hipMemcpyDeviceToHost));
        c.last.reruns++;
    }
    // Ascending order, then the caller's capacity; instances are
    // independent, so host threads take them in turn.
    std::atomic<size_t> next{0};
    std::atomic<bool> dup{false};
    auto worker = [&]() {
        std::vector<uint32_t> tmp;
        for (size_t i = next++; i < m; i = next++) {
            if (status[i] != PMS_OK) continue;
            uint32_t* const v = h_codes + seg[i];
            const size_t k_all = seg[i + 1] - seg[i];
            sort_codes(v, k_all, 2 * shapes[i].l, tmp);
            if (std::adjacent_find(v, v + k_all) != v + k_all) {
                dup = true;
                continue;
            }
            const uint64_t k = std::min<uint64_t>(caps[i], k_all);
            if (k) memcpy(outs[i], v, k * 4);
        }
    };
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned nthreads =
        seg[m] < (1u << 16) ? 1u : std::min<unsigned>(std::min(hw, 16u), static_cast<unsigned>(m));
    std::vector<std::thread> pool;
    for (unsigned w = 1; w < nthreads; ++w) pool.emplace_back(worker);
    worker();
    for (auto& th : pool) th.join();
    if (dup) return fail(PMS_ERR_DEVICE, "duplicate motif in device output");
    for (size_t i = 0; i < m; ++i)
        if (status[i] == PMS_OK && counts[i] > caps[i])
            status[i] = fail(PMS_ERR_OVERFLOW, "more motifs than capacity");
    c.last.host_prep_ms = prep_ms;
    c.last.host_finish_ms = ms_since(t_back);
    return PMS_OK;
}

// ---------------------------------------------------------------------------
// Autotune helpers: a small FM-shaped instance from a fixed seed.
// ---------------------------------------------------------------------------
uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

std::vector<std::string> synthetic_rows(int32_t n, int32_t t, int32_t l, int32_t d, uint64_t seed) {
    const char* acgt = "ACGT";
    std::vector<std::string> rows(n, std::string(t, 'A'));
    std::string cons(l, 'A');
    for (auto& ch : cons) ch = acgt[splitmix(seed) & 3];
    for (auto& r : rows)
        for (auto& ch : r) ch = acgt[splitmix(seed) & 3];
    for (auto& r : rows) {
        std::string inst = cons;
        std::vector<int> pos(l);
        std::iota(pos.begin(), pos.end(), 0);
        for (int k = 0; k < d; ++k) {
            const int j = k + static_cast<int>(splitmix(seed) % (l - k));
            std::swap(pos[k], pos[j]);
            const int b = static_cast<int>(strchr(acgt, inst[pos[k]]) - acgt);
            inst[pos[k]] = acgt[(b + 1 + splitmix(seed) % 3) & 3];
        }
        const int off = static_cast<int>(splitmix(seed) % (t - l + 1));
        r.replace(off, l, inst);
    }
    return rows;
}

// Cache key of a tuned configuration: the build (a hash of the library's
// sources, so that a setting tuned on other kernels is never reused), the
// device, the requested variant and filter, and the shape bucket.
#ifndef PMS_BUILD_ID
#define PMS_BUILD_ID "unversioned"
#endif
std::string tune_key(const Ctx& c, int32_t n, int32_t t, int32_t l, int32_t d) {
    std::ostringstream o;
    o << PMS_BUILD_ID << "/" << c.arch << "/cu" << c.cus << "/v" << c.cfg.variant << "/f"
      << c.cfg.filter << "/l" << l << "/d" << d << "/n" << n << "/nw"
      << align_up(static_cast<size_t>(t - l + 1), 128);
    return o.str();
}

// The cache file is one flat JSON object:
// {"key": [chunk, wg_waves, wgs_per_cu, tail_split, variant, filter], ...}
bool cache_lookup(const std::string& path, const std::string& key, pms_config* out) {
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    const std::string pat = "\"" + key + "\": [";
    const size_t p = s.find(pat);
    if (p == std::string::npos) return false;
    unsigned a = 0, b = 0, cc = 0, dd = 0, ee = 0, ff = 0;
    if (sscanf(s.c_str() + p + pat.size(), "%u, %u, %u, %u, %u, %u", &a, &b, &cc, &dd, &ee, &ff) != 6)
        return false;
    pms_config r{a, b, cc, dd, ee, ff};
    if (!config_ok(r)) return false;
    *out = r;
    return true;
}

void cache_store(const std::string& path, const std::string& key, const pms_config& cfg) {
    std::vector<std::pair<std::string, std::string>> entries;
    {
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line)) {
            const size_t a = line.find('"');
            const size_t b = line.find("\": [");
            if (a == std::string::npos || b == std::string::npos || b <= a) continue;
            const std::string k = line.substr(a + 1, b - a - 1);
            const size_t e = line.find(']', b);
            if (e == std::string::npos) continue;
            if (k != key) entries.emplace_back(k, line.substr(b + 4, e - b - 4));
        }
    }
    std::ostringstream v;
    v << cfg.chunk << ", " << cfg.wg_waves << ", " << cfg.wgs_per_cu << ", " << cfg.tail_split << ", "
      << cfg.variant << ", " << cfg.filter;
    entries.emplace_back(key, v.str());
    std::ofstream f(path + ".tmp");
    f << "{\n";
    for (size_t i = 0; i < entries.size(); ++i)
        f << "  \"" << entries[i].first << "\": [" << entries[i].second << "]"
          << (i + 1 < entries.size() ? ",\n" : "\n");
    f << "}\n";
    f.close();
    rename((path + ".tmp").c_str(), path.c_str());
}

// Times the candidate-chunk x workgroup-shape x tail-split grid (and the
// given variants) on these instances with eager launches, `reps` times each,
// and returns the configuration with the shortest search-kernel time.
int tune_grid(Ctx& c, const std::vector<Shape>& shapes,
              const std::vector<const char* const*>& rows, const std::vector<uint32_t>& variants,
              int reps, pms_config* best) {
    uint64_t total = 0;
    for (const Shape& s : shapes) total = std::max<uint64_t>(total, 1ull << (2 * s.l));
    *best = c.cfg;
    double best_ms = 1e300;
    const uint32_t chunks[] = {1u << 11, 1u << 12, 1u << 13, 1u << 14, 1u << 15, 1u << 16};
    const uint32_t waves[] = {1, 2, 4, 8};
    const uint32_t tails[] = {0, 8};
    for (uint32_t v : variants)
        for (uint32_t ch : chunks) {
            if (ch > total && ch != chunks[0]) continue;
            // From l = 6 on items are whole multiples of 4096 candidates, so a
            // smaller chunk gives the same plan as 4096.
            if (ch < 4096 && total >= 4096) continue;
            for (uint32_t w : waves)
                for (uint32_t tail : tails) {
                    pms_config cfg{ch, w, 0, tail, v, c.cfg.filter};
                    Batch b;
                    b.shape = shapes;
                    b.rows = rows;
                    b.out_cap.assign(shapes.size(), 0);
                    plan_batch(b, cfg, target_items(c, shapes.size()));
                    PMS_TRY(stage_batch(c, b));
                    double ms = 1e300;
                    for (int rep = 0; rep < reps; ++rep) {
                        PMS_TRY(run_batch(c, b, cfg, false));
                        ms = std::min(ms, c.last.kernel_ms);
                    }
                    if (ms < best_ms) {
                        best_ms = ms;
                        *best = cfg;
                    }
                }
        }
    return PMS_OK;
}

// Cache key of a batch: the build, the device, the requested variant and
// filter, and a hash of the instances' shapes in order.
std::string tune_key_many(const Ctx& c, const std::vector<Shape>& shapes) {
    uint64_t h = 0xcbf29ce484222325ull;   // FNV-1a over the shapes
    for (const Shape& s : shapes)
        for (int32_t v : {s.n, s.t, s.l, s.d})
            for (int k = 0; k < 4; ++k) {
                h ^= static_cast<uint64_t>((static_cast<uint32_t>(v) >> (8 * k)) & 0xffu);
                h *= 0x100000001b3ull;
            }
    std::ostringstream o;
    o << PMS_BUILD_ID << "/" << c.arch << "/cu" << c.cus << "/v" << c.cfg.variant << "/f"
      << c.cfg.filter << "/batch" << shapes.size() << "/" << std::hex << h;
    return o.str();
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* pms_status_string(int status) {
    switch (status) {
        case PMS_OK: return "ok";
        case PMS_ERR_INVALID: return "invalid argument";
        case PMS_ERR_OVERFLOW: return "output capacity exceeded";
        case PMS_ERR_NOMEM: return "out of memory";
        case PMS_ERR_DEVICE: return "device error";
        default: return "unknown status";
    }
}

const char* pms_last_error(void) { return g_last_error.c_str(); }

int pms_sort_codes(uint32_t* codes, uint64_t count, int32_t l) {
    g_last_error.clear();
    if (l < 1 || l > PMS_MAX_L) return fail(PMS_ERR_INVALID, "l out of range [1, 16]");
    if (count > 0 && !codes) return fail(PMS_ERR_INVALID, "codes is NULL");
    const uint32_t mask = l == 16 ? ~0u : ((1u << (2 * l)) - 1u);
    for (uint64_t i = 0; i < count; ++i)
        if (codes[i] & ~mask) return fail(PMS_ERR_INVALID, "a code has bits above 2l");
    std::vector<uint32_t> tmp;
    sort_codes(codes, static_cast<size_t>(count), 2 * l, tmp);
    for (uint64_t i = 1; i < count; ++i)
        if (codes[i] == codes[i - 1]) return fail(PMS_ERR_DEVICE, "duplicate motif code");
    return PMS_OK;
}

int32_t pms_fill_work_items(uint64_t begin, uint64_t count, uint32_t item_len, uint32_t inst,
                            pms_work_item* out, int32_t max_items) {
    if (item_len == 0 || (max_items > 0 && !out)) return -1;
    if (begin > (1ull << 32) || count > (1ull << 32) - begin) return -1;
    int32_t k = 0;
    for (uint64_t at = begin, end = begin + count; at < end && k < max_items; at += item_len, ++k) {
        const uint64_t len = std::min<uint64_t>(item_len, end - at);
        out[k] = pms_work_item{at, static_cast<uint32_t>(len), inst};
    }
    return k;
}

void pms_decode(uint32_t code, int32_t l, char* out) {
    if (!out || l < 1 || l > PMS_MAX_L) return;
    for (int32_t p = 0; p < l; ++p) out[p] = "ACGT"[(code >> (2 * (l - 1 - p))) & 3u];
}

int32_t pms_window_stride(int32_t t, int32_t l, int32_t layout) {
    if (l < 1 || l > PMS_MAX_L || t < l || t > PMS_MAX_T) return 0;
    if (layout != PMS_LAYOUT_PLANES && layout != PMS_LAYOUT_BITSLICED) return 0;
    return window_stride(t, l, layout);
}

int pms_set_config(const pms_config* cfg) {
    g_last_error.clear();
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    if (!cfg) {
        g_ctx.cfg = default_config();
        return PMS_OK;
    }
    const pms_config r = resolve(cfg, g_ctx.cfg);
    if (!config_ok(r)) return fail(PMS_ERR_INVALID, "configuration field out of range");
    g_ctx.cfg = r;
    return PMS_OK;
}

int pms_get_config(pms_config* cfg) {
    if (!cfg) return fail(PMS_ERR_INVALID, "cfg is NULL");
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    *cfg = g_ctx.cfg;
    return PMS_OK;
}

int pms_solve(const char* const* seqs, int32_t n, int32_t t, int32_t l, int32_t d,
              uint32_t* out_motifs, uint64_t* out_count) {
    const TraceRange trace_range("pms_solve");
    const auto t_call = std::chrono::steady_clock::now();
    g_last_error.clear();
    if (!out_count) return fail(PMS_ERR_INVALID, "out_count is NULL");
    const uint64_t cap = *out_count;
    *out_count = 0;
    PMS_TRY(validate_shape(n, t, l, d));
    if (cap > 0 && !out_motifs) return fail(PMS_ERR_INVALID, "out_motifs is NULL with capacity > 0");
    PMS_TRY(validate_rows(seqs, n, t));
    PMS_TRY(test_hook("pms_solve"));
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    PMS_TRY(init_ctx(g_ctx));
    g_ctx.t_call = t_call;
    std::vector<int> status;
    std::vector<uint64_t> counts;
    std::vector<double> lat;
    PMS_TRY(solve_instances(g_ctx, {Shape{n, t, l, d}}, {seqs}, {out_motifs}, {cap}, status,
                            counts, lat, false));
    *out_count = counts[0];
    return status[0];
}

int pms_solve_ex(const char* const* seqs, int32_t n, const int32_t* lengths, int32_t l,
                 int32_t d, uint32_t flags, uint32_t* out_motifs, uint64_t* out_count) {
    const TraceRange trace_range("pms_solve_ex");
    const auto t_call = std::chrono::steady_clock::now();
    g_last_error.clear();
    if (!out_count) return fail(PMS_ERR_INVALID, "out_count is NULL");
    const uint64_t cap = *out_count;
    *out_count = 0;
    if (!lengths) return fail(PMS_ERR_INVALID, "lengths is NULL");
    if (flags & ~static_cast<uint32_t>(PMS_INPUT_MASK_N | PMS_INPUT_BOTH_STRANDS))
        return fail(PMS_ERR_INVALID, "unknown input flag");
    if (n < 1 || n > PMS_MAX_N) return fail(PMS_ERR_INVALID, "n out of range [1, 64]");
    int32_t t_max = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (lengths[i] < l || lengths[i] > PMS_MAX_T)
            return fail(PMS_ERR_INVALID, "length of sequence " + std::to_string(i) +
                                             " out of range [l, 2^17]");
        t_max = std::max(t_max, lengths[i]);
    }
    PMS_TRY(validate_shape(n, t_max, l, d));
    if (cap > 0 && !out_motifs) return fail(PMS_ERR_INVALID, "out_motifs is NULL with capacity > 0");
    bool empty = false;
    PMS_TRY(validate_rows_ex(seqs, n, lengths, l, flags, &empty));
    PMS_TRY(test_hook("pms_solve_ex"));
    if (empty) return PMS_OK;  // a sequence without windows: no l-mer matches all
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    PMS_TRY(init_ctx(g_ctx));
    g_ctx.t_call = t_call;
    std::vector<int> status;
    std::vector<uint64_t> counts;
    std::vector<double> lat;
    Shape shape{n, t_max, l, d};
    shape.lens = lengths;
    shape.flags = flags;
    PMS_TRY(solve_instances(g_ctx, {shape}, {seqs}, {out_motifs}, {cap}, status, counts, lat,
                            false));
    *out_count = counts[0];
    return status[0];
}

// XOR masks of the distance-d ball around an l-mer code: every choice of at
// most d of the l 2-bit digits, each changed to one of the other three bases
// (digit XOR 1, 2 or 3).  |Ball| = sum_{k<=d} C(l,k) 3^k.
void ball_masks(int32_t l, int32_t d, std::vector<uint32_t>& out) {
    out.clear();
    std::vector<int32_t> pos;
    std::function<void(int32_t, uint32_t)> rec = [&](int32_t start, uint32_t mask) {
        out.push_back(mask);
        if (static_cast<int32_t>(pos.size()) == d) return;
        for (int32_t p = start; p < l; ++p) {
            pos.push_back(p);
            for (uint32_t g = 1; g <= 3; ++g) rec(p + 1, mask | (g << (2 * (l - 1 - p))));
            pos.pop_back();
        }
    };
    rec(0, 0u);
}

uint64_t ball_size(int32_t l, int32_t d) {
    uint64_t total = 0, binom = 1, pow3 = 1;
    for (int32_t k = 0; k <= d; ++k) {
        if (k > 0) {
            binom = binom * static_cast<uint64_t>(l - k + 1) / static_cast<uint64_t>(k);
            pow3 *= 3;
        }
        total += binom * pow3;
    }
    return total;
}

int pms_solve_intersect(const char* const* seqs, int32_t n, int32_t t, int32_t l, int32_t d,
                        uint32_t* out_motifs, uint64_t* out_count) {
    const TraceRange trace_range("pms_solve_intersect");
    const auto t_call = std::chrono::steady_clock::now();
    g_last_error.clear();
    if (!out_count) return fail(PMS_ERR_INVALID, "out_count is NULL");
    const uint64_t cap = *out_count;
    *out_count = 0;
    PMS_TRY(validate_shape(n, t, l, d));
    if (cap > 0 && !out_motifs) return fail(PMS_ERR_INVALID, "out_motifs is NULL with capacity > 0");
    if (ball_size(l, d) > PMS_NBHD_MAX_BALL)
        return fail(PMS_ERR_INVALID, "distance-d ball larger than PMS_NBHD_MAX_BALL masks");
    PMS_TRY(validate_rows(seqs, n, t));
    PMS_TRY(test_hook("pms_solve_intersect"));
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    Ctx& c = g_ctx;
    PMS_TRY(init_ctx(c));
    hipStream_t s = c.stream;
    const int32_t nw = t - l + 1;
    // Tiles of 2^T candidate bits (at most 32 KiB of LDS), small enough that
    // there are about 1024 of them from l = 9 on, the whole map below l = 4;
    // the map is whole 16-byte vectors.
    const int32_t T = 2 * l < 7 ? 2 * l : std::min(18, std::max(7, 2 * l - 10));
    const uint32_t tiles = 1u << (2 * l - T);
    const uint32_t tile_words = std::max<uint32_t>(4u, (1u << T) / 32u);
    const uint64_t words = static_cast<uint64_t>(tiles) * tile_words;
    if (c.nb_ball_l != l || c.nb_ball_d != d) {
        // The ball's masks grouped by their bits above T (group h: the masks
        // that move a window's high bits by h), with the groups' offsets.
        std::vector<uint32_t> masks;
        ball_masks(l, d, masks);
        std::stable_sort(masks.begin(), masks.end(),
                         [T](uint32_t a, uint32_t b) { return (a >> T) < (b >> T); });
        std::vector<uint32_t> off(tiles + 1, 0);
        for (uint32_t x : masks) ++off[(x >> T) + 1];
        for (uint32_t h = 0; h < tiles; ++h) off[h + 1] += off[h];
        std::vector<uint32_t> ne;   // the non-empty groups
        for (uint32_t h = 0; h < tiles; ++h)
            if (off[h + 1] > off[h]) ne.push_back(h);
        PMS_TRY(c.nb_deltas.ensure(masks.size() * 4));
        PMS_TRY(c.nb_groups.ensure(off.size() * 4));
        PMS_TRY(c.nb_ne.ensure(ne.size() * 4));
        PMS_HIP(hipMemcpy(c.nb_deltas.p, masks.data(), masks.size() * 4, hipMemcpyHostToDevice));
        PMS_HIP(hipMemcpy(c.nb_groups.p, off.data(), off.size() * 4, hipMemcpyHostToDevice));
        PMS_HIP(hipMemcpy(c.nb_ne.p, ne.data(), ne.size() * 4, hipMemcpyHostToDevice));
        c.nb_ball_l = l;
        c.nb_ball_d = d;
        c.nb_ball_size = static_cast<int32_t>(masks.size());
        c.nb_nne = static_cast<int32_t>(ne.size());
    }
    const int32_t nd = c.nb_ball_size;
    PMS_TRY(c.d_raw.ensure(std::max<size_t>(static_cast<size_t>(n) * t, 256)));
    PMS_TRY(c.h_raw.ensure(std::max<size_t>(static_cast<size_t>(n) * t, 256)));
    PMS_TRY(c.nb_codes.ensure(static_cast<size_t>(n) * nw * 4));
    PMS_TRY(c.nb_m.ensure(words * 4));
    PMS_TRY(c.nb_count.ensure(256));
    PMS_TRY(c.h_back.ensure(256));
    for (int32_t r = 0; r < n; ++r) memcpy(c.h_raw.as<char>(static_cast<size_t>(r) * t), seqs[r], t);
    const double prep_ms = ms_since(t_call);
    uint32_t* m = c.nb_m.as<uint32_t>();
    auto* cnt = c.nb_count.as<unsigned long long>();
    auto* h_cnt = c.h_back.as<unsigned long long>();
    const uint32_t grid = static_cast<uint32_t>(c.cus) * 16u;
    PMS_HIP(hipEventRecord(c.ev[0], s));
    PMS_HIP(hipMemcpyAsync(c.d_raw.p, c.h_raw.p, static_cast<size_t>(n) * t, hipMemcpyHostToDevice, s));
    PMS_HIP(pms::launch_nbhd_codes(c.d_raw.as<uint8_t>(), t, l, n, c.nb_codes.as<uint32_t>(), s));
    // Each pass is tiled or scattered, whichever costs less: a tiled pass
    // pays for every tile's look-up of every window's mask group, the bits
    // set in LDS and one or two streams of the map; a scatter pass pays for
    // its global atomics, zeroing B and the AND (three streams after the
    // first sequence).  Bitmap passes go on while they are the cheaper way:
    // once the candidates left are few, checking them against the remaining
    // sequences directly costs less than another pass.  Rates are round
    // figures measured on one MI355X.
    // A tiled pass finds each tile's (window, group) pairs either by looking
    // up every window's group in every tile or, when that is dearer, from
    // records sorted by tile (count, scan, fill: nw x non-empty groups).
    constexpr double kLdsBitsPerS = 3e11, kAtomicBitsPerS = 1e10, kStreamBytesPerS = 4e12,
                     kLookupS = 7.6e-12, kRecordS = 4e-11, kRecordFixedS = 2e-5,
                     kComparesPerS = 5e12;
    constexpr uint64_t kMaxRecords = 1u << 24;
    const double bits_set = static_cast<double>(nw) * nd;
    const double map_bytes = static_cast<double>(words) * 4.0;
    const uint64_t records = static_cast<uint64_t>(nw) * static_cast<uint64_t>(c.nb_nne);
    const double lookup_s = static_cast<double>(tiles) * nw * kLookupS;
    const double record_s = static_cast<double>(records) * kRecordS + kRecordFixedS;
    bool use_records = records <= kMaxRecords && record_s < lookup_s;
    auto tiled_s = [&](bool first) {
        return (use_records ? record_s : lookup_s) + bits_set / kLdsBitsPerS +
               (first ? 1.0 : 2.0) * map_bytes / kStreamBytesPerS;
    };
    auto scatter_s = [&](bool first) {
        return bits_set / kAtomicBitsPerS + (first ? 1.0 : 4.0) * map_bytes / kStreamBytesPerS;
    };
    bool tiled_first = tiled_s(true) <= scatter_s(true);
    bool tiled_next = tiled_s(false) <= scatter_s(false);
    // PMS_TEST_NBHD_PASS=tiled|records|scatter forces one form (tests of
    // every form): tiled with look-ups, tiled with records, or scattered.
    if (const char* v = getenv("PMS_TEST_NBHD_PASS")) {
        if (!strcmp(v, "tiled")) tiled_first = tiled_next = true, use_records = false;
        if (!strcmp(v, "records") && records <= kMaxRecords)
            tiled_first = tiled_next = true, use_records = true;
        if (!strcmp(v, "scatter")) tiled_first = tiled_next = false;
    }
    PMS_TRY(c.nb_part.ensure(static_cast<size_t>(std::max<uint32_t>(tiles, grid)) * 4));
    uint32_t* const part = c.nb_part.as<uint32_t>();
    if ((tiled_first || tiled_next) && use_records) {
        PMS_TRY(c.nb_tcount.ensure(static_cast<size_t>(tiles) * 4));
        PMS_TRY(c.nb_toff.ensure(static_cast<size_t>(tiles + 1) * 4));
        PMS_TRY(c.nb_tcur.ensure(static_cast<size_t>(tiles) * 4));
        PMS_TRY(c.nb_rec.ensure(std::max<uint64_t>(records, 1) * 4));
    }
    const double pass_s = std::min(tiled_s(false), scatter_s(false));
    if (!tiled_next && n > 1) PMS_TRY(c.nb_b.ensure(words * 4));
    // PMS_TEST_NBHD_VERIFY_AFTER=<k> checks the survivors directly after k
    // passes whatever the cost model says (tests of both verify kernels).
    int32_t verify_after = 0;
    if (const char* v = getenv("PMS_TEST_NBHD_VERIFY_AFTER")) verify_after = atoi(v);
    uint64_t left = 0, visits = 0;
    int32_t scanned = 0;
    bool verified = false;
    for (int32_t i = 0; i < n; ++i) {
        PMS_HIP(pms::launch_fill(reinterpret_cast<uint32_t*>(cnt), 8, 0u, s));
        // M = B for the first sequence, M &= B after; cnt counts M's bits.
        const uint32_t* codes_i = c.nb_codes.as<uint32_t>() + static_cast<size_t>(i) * nw;
        if (i == 0 ? tiled_first : tiled_next) {
            const uint32_t* rec = nullptr;
            const uint32_t* rec_off = nullptr;
            if (use_records) {
                PMS_HIP(pms::launch_nbhd_records(codes_i, nw, c.nb_ne.as<uint32_t>(), c.nb_nne, T, tiles,
                                                 c.nb_tcount.as<uint32_t>(), c.nb_toff.as<uint32_t>(),
                                                 c.nb_tcur.as<uint32_t>(), c.nb_rec.as<uint32_t>(), grid,
                                                 s));
                rec = c.nb_rec.as<uint32_t>();
                rec_off = c.nb_toff.as<uint32_t>();
            }
            PMS_HIP(pms::launch_nbhd_tile(codes_i, nw, c.nb_deltas.as<uint32_t>(),
                                          c.nb_groups.as<uint32_t>(), rec, rec_off, T, tiles,
                                          tile_words, m, i == 0, part, s));
            PMS_HIP(pms::launch_nbhd_sum(part, tiles, cnt, s));
        } else {
            uint32_t* target = i == 0 ? m : c.nb_b.as<uint32_t>();
            PMS_HIP(pms::launch_nbhd_zero(target, words, grid, s));
            PMS_HIP(pms::launch_nbhd_scatter(codes_i, nw, c.nb_deltas.as<uint32_t>(), nd, target,
                                             i == 0 ? part : nullptr, grid, s));
            if (i > 0) PMS_HIP(pms::launch_nbhd_and(m, target, words, part, grid, s));
            PMS_HIP(pms::launch_nbhd_sum(part, grid, cnt, s));
        }
        PMS_HIP(hipMemcpyAsync(h_cnt, cnt, 8, hipMemcpyDeviceToHost, s));
        PMS_HIP(hipStreamSynchronize(s));
        left = h_cnt[0];
        ++scanned;
        if (left == 0 || i + 1 == n) break;
        const double verify_s = static_cast<double>(left) * nw * 1.1 / kComparesPerS;
        const bool forced = verify_after > 0 && scanned >= verify_after;
        if (!forced && verify_s > pass_s) continue;
        // The candidates left, then sequences i+1 .. n-1 checked directly.
        PMS_TRY(c.nb_cand.ensure(left * 4));
        PMS_TRY(c.nb_out.ensure(left * 4));
        PMS_HIP(pms::launch_fill(reinterpret_cast<uint32_t*>(cnt), 2, 0u, s));  // collect count
        PMS_HIP(pms::launch_nbhd_collect(m, words, c.nb_cand.as<uint32_t>(), left, cnt, grid, s));
        PMS_HIP(pms::launch_nbhd_verify(c.nb_cand.as<uint32_t>(), left, c.nb_codes.as<uint32_t>(), nw,
                                        i + 1, n, d, c.nb_out.as<uint32_t>(), left, cnt + 1, cnt + 2,
                                        grid, s));
        PMS_HIP(hipEventRecord(c.ev[2], s));
        PMS_HIP(hipMemcpyAsync(h_cnt, cnt, 24, hipMemcpyDeviceToHost, s));
        PMS_HIP(hipStreamSynchronize(s));
        if (h_cnt[0] != left) return fail(PMS_ERR_DEVICE, "collected count differs from the AND count");
        left = h_cnt[1];
        visits = h_cnt[2];
        verified = true;
        break;
    }
    if (!verified) {
        PMS_TRY(c.nb_out.ensure(std::max<uint64_t>(left, 1) * 4));
        PMS_HIP(pms::launch_fill(reinterpret_cast<uint32_t*>(cnt), 2, 0u, s));
        if (left)
            PMS_HIP(pms::launch_nbhd_collect(m, words, c.nb_out.as<uint32_t>(), left, cnt, grid, s));
        PMS_HIP(hipEventRecord(c.ev[2], s));
        PMS_HIP(hipMemcpyAsync(h_cnt, cnt, 8, hipMemcpyDeviceToHost, s));
        PMS_HIP(hipStreamSynchronize(s));
        if (left && h_cnt[0] != left)
            return fail(PMS_ERR_DEVICE, "collected count differs from the AND count");
    }
    const auto t_back = std::chrono::steady_clock::now();
    std::vector<uint32_t> codes(left);
    if (left)
        PMS_HIP(hipMemcpy(codes.data(), c.nb_out.p, left * 4, hipMemcpyDeviceToHost));
    std::vector<uint32_t> tmp;
    sort_codes(codes.data(), codes.size(), 2 * l, tmp);
    const uint64_t k = std::min<uint64_t>(cap, left);
    if (k) memcpy(out_motifs, codes.data(), k * 4);
    float ms = 0;
    PMS_HIP(hipEventElapsedTime(&ms, c.ev[0], c.ev[2]));
    c.last = pms_stats{};
    c.last.kernel_ms = ms;
    c.last.batches = static_cast<uint64_t>(scanned);
    c.last.window_compares = static_cast<uint64_t>(scanned) * nw * static_cast<uint64_t>(nd);
    c.last.seq_visits = visits;
    c.last.host_prep_ms = prep_ms;
    c.last.host_finish_ms = ms_since(t_back);
    c.last_pending = false;
    *out_count = left;
    return left > cap ? fail(PMS_ERR_OVERFLOW, "more motifs than capacity") : PMS_OK;
}

int pms_solve_many(const pms_instance* inst, int32_t count, pms_result* results) {
    const TraceRange trace_range("pms_solve_many");
    const auto t_call = std::chrono::steady_clock::now();
    g_last_error.clear();
    if (!inst || !results || count < 0) return fail(PMS_ERR_INVALID, "NULL batch or negative count");
    std::vector<Shape> shapes;
    std::vector<const char* const*> rows;
    std::vector<uint32_t*> outs;
    std::vector<uint64_t> caps;
    std::vector<int32_t> index;
    int first_bad = PMS_OK;
    std::string first_msg;
    for (int32_t i = 0; i < count; ++i) {
        results[i].status = PMS_OK;
        results[i].reserved = 0;
        results[i].count = 0;
        results[i].latency_ms = 0;
        const pms_instance& q = inst[i];
        int s = validate_shape(q.n, q.t, q.l, q.d);
        if (s == PMS_OK && q.capacity > 0 && !q.out_motifs)
            s = fail(PMS_ERR_INVALID, "out_motifs is NULL with capacity > 0");
        if (s == PMS_OK) s = validate_rows(q.seqs, q.n, q.t);
        if (s != PMS_OK) {
            results[i].status = s;
            if (first_bad == PMS_OK) {
                first_bad = s;
                first_msg = g_last_error;
            }
            continue;
        }
        shapes.push_back({q.n, q.t, q.l, q.d});
        rows.push_back(q.seqs);
        outs.push_back(q.out_motifs);
        caps.push_back(q.capacity);
        index.push_back(i);
    }
    if (shapes.empty()) {
        if (first_bad != PMS_OK) g_last_error = first_msg;
        return first_bad;
    }
    PMS_TRY(test_hook("pms_solve_many"));
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    PMS_TRY(init_ctx(g_ctx));
    g_ctx.t_call = t_call;
    std::vector<int> status;
    std::vector<uint64_t> counts;
    std::vector<double> lat;
    PMS_TRY(solve_instances(g_ctx, shapes, rows, outs, caps, status, counts, lat,
                            use_graph_default()));
    for (size_t j = 0; j < index.size(); ++j) {
        pms_result& r = results[index[j]];
        r.status = status[j];
        r.count = counts[j];
        r.latency_ms = lat[j];
    }
    int ret = PMS_OK;
    for (int32_t i = 0; i < count && ret == PMS_OK; ++i) ret = results[i].status;
    if (ret != PMS_OK && ret == first_bad && !first_msg.empty()) g_last_error = first_msg;
    return ret;
}

int pms_last_stats(pms_stats* out) {
    if (!out) return fail(PMS_ERR_INVALID, "out is NULL");
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    Ctx& c = g_ctx;
    if (c.last_pending) {
        // A device-level call: read its events and counters now.
        float w_ms = 0, k_ms = 0;
        PMS_HIP(hipEventSynchronize(c.ev[2]));
        PMS_HIP(hipEventElapsedTime(&w_ms, c.ev[0], c.ev[1]));
        PMS_HIP(hipEventElapsedTime(&k_ms, c.ev[1], c.ev[2]));
        c.last.windows_ms = w_ms;
        c.last.kernel_ms = k_ms;
        if (c.dv_counters) {
            PMS_HIP(hipEventSynchronize(c.dv_back));
            const pms_dev_state st = *c.hv_back.as<pms_dev_state>(c.dv_state_off);
            const pms_dev_counters ctr = *c.hv_back.as<pms_dev_counters>(c.dv_ctr_off);
            c.last.seq_visits = st.visits;
            c.last.window_compares = st.visits * static_cast<uint64_t>(c.dv_nw);
            c.last.batches = ctr.batches;
            c.last.single_batches = ctr.single_batches;
            c.last.filtered_batches = ctr.filtered_batches;
            c.last.filtered_groups = ctr.filtered_groups;
            c.last.candidate_slots = candidate_slots(ctr, c.dv_variant);
        }
        c.last_pending = false;
    }
    *out = c.last;
    return PMS_OK;
}

int pms_build_windows(const uint8_t* dev_seqs, int32_t n, int32_t t, int32_t l, int32_t layout,
                      uint32_t* dev_windows, uint32_t* dev_bad, void* stream) {
    const TraceRange trace_range("pms_build_windows");
    g_last_error.clear();
    if (!dev_seqs || !dev_windows) return fail(PMS_ERR_INVALID, "NULL device pointer");
    if (n < 1 || n > PMS_MAX_N || l < 1 || l > PMS_MAX_L || t < l || t > PMS_MAX_T)
        return fail(PMS_ERR_INVALID, "size out of range");
    if (layout != PMS_LAYOUT_PLANES && (layout != PMS_LAYOUT_BITSLICED || l < 2))
        return fail(PMS_ERR_INVALID, "bad layout (BITSLICED needs l >= 2)");
    PMS_TRY(test_hook("pms_build_windows"));
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    Ctx& c = g_ctx;
    PMS_TRY(init_ctx(c));
    hipStream_t s = static_cast<hipStream_t>(stream);
    static_assert(PMS_MAX_N * sizeof(pms_win_job) <= Ctx::kJobSlot, "job slot too small");
    PMS_TRY(c.bw_host.ensure(Ctx::kJobRing * Ctx::kJobSlot));
    PMS_TRY(c.bw_dev.ensure(Ctx::kJobRing * Ctx::kJobSlot));
    const int slot = c.bw_next;
    c.bw_next = (slot + 1) % Ctx::kJobRing;
    if (!c.bw_ev[slot]) PMS_HIP(hipEventCreateWithFlags(&c.bw_ev[slot], hipEventDisableTiming));
    if (c.bw_live[slot]) PMS_HIP(hipEventSynchronize(c.bw_ev[slot]));
    char* h = c.bw_host.as<char>(slot * Ctx::kJobSlot);
    char* dv = c.bw_dev.as<char>(slot * Ctx::kJobSlot);
    pms_win_job* jobs = reinterpret_cast<pms_win_job*>(h);
    const int32_t stride = window_stride(t, l, layout);
    for (int32_t r = 0; r < n; ++r)
        jobs[r] = {static_cast<uint64_t>(r) * t, static_cast<uint64_t>(r) * stride, t, l, stride, 0,
                   layout, 0};
    PMS_HIP(hipMemcpyAsync(dv, h, static_cast<size_t>(n) * sizeof(pms_win_job),
                           hipMemcpyHostToDevice, s));
    PMS_HIP(hipEventRecord(c.bw_ev[slot], s));
    c.bw_live[slot] = true;
    PMS_HIP(pms::launch_windows(reinterpret_cast<const pms_win_job*>(dv), n, t, dev_seqs,
                                dev_windows, dev_bad, s));
    return PMS_OK;
}

int pms_step_launch(const pms_dev_instance* dev_instances, int32_t n_inst, int32_t max_n,
                    const pms_work_item* dev_work, int32_t n_work, pms_dev_state* dev_state,
                    pms_dev_counters* dev_counters, const pms_config* cfg, void* stream) {
    const TraceRange trace_range("pms_step_launch");
    g_last_error.clear();
    if (!dev_instances || !dev_state || !dev_counters || (n_work > 0 && !dev_work))
        return fail(PMS_ERR_INVALID, "NULL device pointer");
    if (n_inst < 1 || n_work < 0 || max_n < 1 || max_n > PMS_MAX_N)
        return fail(PMS_ERR_INVALID, "table size out of range");
    PMS_TRY(test_hook("pms_step_launch"));
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    Ctx& c = g_ctx;
    PMS_TRY(init_ctx(c));
    const pms_config r = resolve(cfg, c.cfg);
    if (!config_ok(r)) return fail(PMS_ERR_INVALID, "configuration field out of range");
    const uint32_t variant = r.variant == PMS_VARIANT_AUTO ? PMS_VARIANT_GROUP64 : r.variant;
    Shape2 sh;
    PMS_TRY(launch_shape(c, r, max_n, variant, c.dv_gq, &sh));
    const uint32_t grid = sh.grid, waves = sh.waves;
    hipStream_t s = static_cast<hipStream_t>(stream);
    PMS_HIP(hipEventRecord(c.ev[0], s));
    PMS_HIP(hipEventRecord(c.ev[1], s));
    PMS_HIP(launch_variant(variant, launch_flags(r), dev_instances, dev_work, static_cast<uint32_t>(n_work), dev_state,
                           dev_counters, sh, s));
    PMS_HIP(hipEventRecord(c.ev[2], s));
    c.last = pms_stats{};
    c.last.grid = grid;
    c.last.wg_waves = waves;
    c.last.chunk = r.chunk;
    c.last.variant = variant;
    c.last.work_items = static_cast<uint32_t>(n_work);
    c.last_pending = true;
    c.dv_counters = false;
    return PMS_OK;
}

int pms_solve_dev(const uint8_t* dev_seqs, int32_t n, int32_t t, int32_t l, int32_t d,
                  uint32_t* dev_out, uint64_t capacity, uint64_t* dev_count, void* stream) {
    const TraceRange trace_range("pms_solve_dev");
    g_last_error.clear();
    if (!dev_seqs || !dev_count || (capacity > 0 && !dev_out))
        return fail(PMS_ERR_INVALID, "NULL device pointer");
    PMS_TRY(validate_shape(n, t, l, d));
    PMS_TRY(test_hook("pms_solve_dev"));
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    Ctx& c = g_ctx;
    PMS_TRY(init_ctx(c));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const pms_config cfg = c.cfg;
    std::ostringstream kss;
    kss << n << ':' << t << ':' << l << ':' << d << ':' << cfg.chunk << ':' << cfg.wg_waves << ':'
        << cfg.wgs_per_cu << ':' << cfg.tail_split << ':' << cfg.variant << ':' << cfg.filter << ':'
        << target_items(c, 1);
    const std::string key = kss.str();
    const bool reuse = c.dv_plan_valid && key == c.dv_key;
    if (!reuse) {
        c.dv_plan_valid = false;
        c.dv_plan = Batch{};
        c.dv_plan.shape = {Shape{n, t, l, d}};
        c.dv_plan.out_cap = {1};
        plan_batch(c.dv_plan, cfg, target_items(c, 1));
    }
    const Batch& b = c.dv_plan;
    Shape2 sh;
    PMS_TRY(launch_shape(c, cfg, b.max_n, b.variant, c.dv_gq, &sh));
    const uint32_t grid = sh.grid, waves = sh.waves;
    if (c.dv_copy_live) PMS_HIP(hipEventSynchronize(c.dv_copied));
    PMS_TRY(c.dv_win.ensure(std::max<size_t>(b.win_words * 4, 256)));
    PMS_TRY(c.dv_meta.ensure(b.meta_bytes));
    PMS_TRY(c.hv_meta.ensure(b.meta_bytes));
    char* hm = c.hv_meta.as<char>();
    char* dm = c.dv_meta.as<char>();
    // The per-call records (instance; state, counters, flags) are rewritten
    // every call; the window jobs and the work table only with a new plan.
    const bool whole = !reuse || c.dv_uploaded != c.dv_meta.p;
    memset(hm, 0, b.off_jobs);
    pms_dev_instance* in = reinterpret_cast<pms_dev_instance*>(hm + b.off_insts);
    in->windows = c.dv_win.as<uint32_t>();
    in->out = dev_out;
    in->out_cap = capacity;
    in->n = n;
    in->nw_stride = window_stride(
        t, l, b.variant == PMS_VARIANT_LANE ? PMS_LAYOUT_PLANES : PMS_LAYOUT_BITSLICED);
    in->l = l;
    in->d = d;
    reinterpret_cast<pms_dev_state*>(hm + b.off_state)->items_left = b.items_per_inst[0];
    if (whole) {
        memcpy(hm + b.off_jobs, b.jobs.data(), b.jobs.size() * sizeof(pms_win_job));
        memcpy(hm + b.off_work, b.work.data(), b.work.size() * sizeof(pms_work_item));
        PMS_HIP(hipMemcpyAsync(dm, hm, b.meta_bytes, hipMemcpyHostToDevice, s));
    } else {
        PMS_HIP(hipMemcpyAsync(dm, hm, b.off_jobs, hipMemcpyHostToDevice, s));
    }
    PMS_HIP(hipEventRecord(c.dv_copied, s));
    c.dv_copy_live = true;
    c.dv_key = key;
    c.dv_plan_valid = true;
    c.dv_uploaded = c.dv_meta.p;
    PMS_HIP(hipEventRecord(c.ev[0], s));
    PMS_HIP(pms::launch_windows(reinterpret_cast<const pms_win_job*>(dm + b.off_jobs), n, t,
                                dev_seqs, c.dv_win.as<uint32_t>(),
                                reinterpret_cast<uint32_t*>(dm + b.off_bad), s));
    PMS_HIP(hipEventRecord(c.ev[1], s));
    PMS_HIP(launch_variant(b.variant, b.flags, reinterpret_cast<const pms_dev_instance*>(dm + b.off_insts),
                           reinterpret_cast<const pms_work_item*>(dm + b.off_work),
                           static_cast<uint32_t>(b.work.size()),
                           reinterpret_cast<pms_dev_state*>(dm + b.off_state),
                           reinterpret_cast<pms_dev_counters*>(dm + b.off_ctr), sh, s));
    PMS_HIP(hipEventRecord(c.ev[2], s));
    PMS_HIP(hipMemcpyAsync(dev_count, dm + b.off_state + offsetof(pms_dev_state, count),
                           sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    // The state and counters for pms_last_stats, without a synchronous copy.
    PMS_TRY(c.hv_back.ensure(b.off_jobs));
    PMS_HIP(hipMemcpyAsync(c.hv_back.as<char>(b.off_state), dm + b.off_state, b.off_jobs - b.off_state,
                           hipMemcpyDeviceToHost, s));
    PMS_HIP(hipEventRecord(c.dv_back, s));
    c.last = pms_stats{};
    c.last.grid = grid;
    c.last.wg_waves = waves;
    c.last.chunk = cfg.chunk;
    c.last.variant = b.variant;
    c.last.work_items = static_cast<uint32_t>(b.work.size());
    c.last_pending = true;
    c.dv_counters = true;
    c.dv_variant = b.variant;
    c.dv_state_off = b.off_state;
    c.dv_ctr_off = b.off_ctr;
    c.dv_nw = t - l + 1;
    return PMS_OK;
}

int pms_shutdown(void) {
    const TraceRange trace_range("pms_shutdown");
    g_last_error.clear();
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    Ctx& c = g_ctx;
    if (!c.dev_ready) return PMS_OK;  // nothing was created
    int status = PMS_OK;
    auto note = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && status == PMS_OK)
            status = fail(PMS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    note(hipSetDevice(c.device), "hipSetDevice");
    // Device-level calls may still run on callers' streams with library
    // buffers: everything on the device completes first.
    note(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (c.gexec) note(hipGraphExecDestroy(c.gexec), "hipGraphExecDestroy");
    c.gexec = nullptr;
    c.gsig.clear();
    for (auto& e : c.ev) {
        if (e) note(hipEventDestroy(e), "hipEventDestroy");
        e = nullptr;
    }
    for (hipEvent_t* e : {&c.dv_copied, &c.dv_back}) {
        if (*e) note(hipEventDestroy(*e), "hipEventDestroy");
        *e = nullptr;
    }
    for (int i = 0; i < Ctx::kJobRing; ++i) {
        if (c.bw_ev[i]) note(hipEventDestroy(c.bw_ev[i]), "hipEventDestroy");
        c.bw_ev[i] = nullptr;
        c.bw_live[i] = false;
    }
    c.bw_next = 0;
    if (c.stream) note(hipStreamDestroy(c.stream), "hipStreamDestroy");
    c.stream = nullptr;
    for (DevBuf* b : {&c.d_raw, &c.d_win, &c.d_out, &c.d_meta, &c.d_gq, &c.d_gtab, &c.d_gather,
                      &c.dv_win, &c.dv_meta,
                      &c.dv_gq, &c.bw_dev, &c.nb_m, &c.nb_b, &c.nb_codes, &c.nb_deltas,
                      &c.nb_groups, &c.nb_ne, &c.nb_cand, &c.nb_out, &c.nb_count, &c.nb_tcount,
                      &c.nb_toff, &c.nb_tcur, &c.nb_rec, &c.nb_part})
        note(b->release(), "hipFree");
    for (HostBuf* b : {&c.h_raw, &c.h_meta, &c.h_back, &c.h_out, &c.h_gtab, &c.hv_meta, &c.hv_back,
                       &c.bw_host})
        note(b->release(), "hipHostFree");
    c.nb_ball_l = c.nb_ball_d = -1;
    c.nb_ball_size = c.nb_nne = 0;
    c.dv_plan_valid = false;
    c.dv_uploaded = nullptr;
    c.dv_copy_live = false;
    c.dv_counters = false;
    c.last_pending = false;
    c.shapes.clear();
    c.ready = false;
    c.dev_ready = false;
    c.scratch = nullptr;
    c.scratch_bytes = 0;
    return status;
}

int pms_solve_dev_noalloc(const uint8_t* dev_seqs, int32_t n, int32_t t, int32_t l, int32_t d,
                          uint32_t* dev_out, uint64_t capacity, uint64_t* dev_count,
                          void* stream) {
    const TraceRange trace_range("pms_solve_dev_noalloc");
    g_last_error.clear();
    if (!dev_seqs || !dev_count || (capacity > 0 && !dev_out))
        return fail(PMS_ERR_INVALID, "NULL device pointer");
    PMS_TRY(validate_shape(n, t, l, d));
    PMS_TRY(test_hook("pms_solve_dev_noalloc"));
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    Ctx& c = g_ctx;
    PMS_TRY(init_device(c));
    if (!c.scratch) return fail(PMS_ERR_DEVICE, "no scratch address for this device");
    const pms_config cfg = c.cfg;
    const Shape shape{n, t, l, d};
    const uint32_t variant = choose_variant({shape}, cfg.variant);
    const int32_t layout = variant == PMS_VARIANT_LANE ? PMS_LAYOUT_PLANES : PMS_LAYOUT_BITSLICED;
    // The same items the host planner makes for one instance.
    const ItemPlan ip = item_plan(shape, 1.0, cfg, target_items(c, 1));
    pms::NoallocLayout lay{};
    lay.n = n;
    lay.t = t;
    lay.l = l;
    lay.d = d;
    lay.layout = layout;
    lay.stride = window_stride(t, l, layout);
    lay.size = ip.size;
    lay.small = ip.small;
    const uint64_t n_head = ip.head_end ? (ip.head_end + ip.size - 1) / ip.size : 0;
    const uint64_t h = std::min(n_head * ip.size, ip.total);
    const uint64_t n_small = h < ip.total ? (ip.total - h + ip.small - 1) / ip.small : 0;
    lay.n_head = static_cast<uint32_t>(n_head);
    lay.n_items = static_cast<uint32_t>(n_head + n_small);
    size_t off = 0;
    lay.off_win = off;
    off = align_up(off + static_cast<size_t>(n) * lay.stride * 4, 256);
    lay.off_inst = off;
    off = align_up(off + sizeof(pms_dev_instance), 256);
    lay.off_state = off;
    off = align_up(off + sizeof(pms_dev_state), 256);
    lay.off_ctr = off;
    off = align_up(off + sizeof(pms_dev_counters), 256);
    lay.off_bad = off;
    off = align_up(off + sizeof(uint32_t), 256);
    lay.off_jobs = off;
    off = align_up(off + static_cast<size_t>(n) * sizeof(pms_win_job), 256);
    lay.off_work = off;
    off = align_up(off + static_cast<size_t>(lay.n_items) * sizeof(pms_work_item), 256);
    // PMS_TEST_NOALLOC_CAP=<bytes> lowers the usable size (tests of the
    // reduced grid and of the size error).
    size_t avail = c.scratch_bytes;
    if (const char* v = getenv("PMS_TEST_NOALLOC_CAP")) {
        const long long k = atoll(v);
        if (k > 0 && static_cast<size_t>(k) < avail) avail = static_cast<size_t>(k);
    }
    Shape2 sh;
    PMS_TRY(cached_shape(c, cfg, n, variant, &sh));
    const size_t per_wg = static_cast<size_t>(sh.waves) * sh.gq.gq_words * 4;
    if (off > avail || (per_wg && avail - off < per_wg))
        return fail(PMS_ERR_INVALID,
                    "tables of this size (" + std::to_string(off + per_wg) +
                        " bytes with one workgroup's stage queues) exceed the fixed scratch of " +
                        std::to_string(avail) + " bytes");
    if (per_wg) {
        // Stage queues beyond LDS for every workgroup; with less room, fewer
        // workgroups (the persistent search is exact with any grid).
        sh.grid = static_cast<uint32_t>(std::min<size_t>(sh.grid, (avail - off) / per_wg));
        sh.gq.gq = reinterpret_cast<uint32_t*>(static_cast<char*>(c.scratch) + off);
        off += per_wg * sh.grid;
    }
    lay.off_gq = off - per_wg * sh.grid;
    lay.bytes = off;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(c.scratch);
    PMS_HIP(pms::launch_noalloc_setup(base, lay, dev_out, capacity, s));
    PMS_HIP(pms::launch_windows(reinterpret_cast<const pms_win_job*>(base + lay.off_jobs), n, t,
                                dev_seqs, reinterpret_cast<uint32_t*>(base + lay.off_win),
                                reinterpret_cast<uint32_t*>(base + lay.off_bad), s));
    PMS_HIP(launch_variant(variant, launch_flags(cfg),
                           reinterpret_cast<const pms_dev_instance*>(base + lay.off_inst),
                           reinterpret_cast<const pms_work_item*>(base + lay.off_work),
                           lay.n_items, reinterpret_cast<pms_dev_state*>(base + lay.off_state),
                           reinterpret_cast<pms_dev_counters*>(base + lay.off_ctr), sh, s));
    PMS_HIP(pms::launch_noalloc_count(reinterpret_cast<const pms_dev_state*>(base + lay.off_state),
                                      dev_count, s));
    // No events or counters are kept for this call.
    c.last = pms_stats{};
    c.last.grid = sh.grid;
    c.last.wg_waves = sh.waves;
    c.last.chunk = cfg.chunk;
    c.last.variant = variant;
    c.last.work_items = lay.n_items;
    c.last_pending = false;
    c.dv_counters = false;
    return PMS_OK;
}

int pms_autotune(int32_t n, int32_t t, int32_t l, int32_t d, const char* cache_path,
                 pms_config* best) {
    const TraceRange trace_range("pms_autotune");
    g_last_error.clear();
    PMS_TRY(validate_shape(n, t, l, d));
    std::string path = cache_path ? cache_path : "";
    if (path.empty())
        if (const char* v = getenv("PMS_AUTOTUNE_CACHE")) path = v;
    std::unique_lock<std::mutex> lk(g_ctx.mu);
    Ctx& c = g_ctx;
    PMS_TRY(init_ctx(c));
    const std::string key = tune_key(c, n, t, l, d);
    pms_config found;
    if (!path.empty() && cache_lookup(path, key, &found)) {
        c.cfg = found;
        if (best) *best = found;
        return PMS_OK;
    }
    const std::vector<std::string> rows = synthetic_rows(n, t, l, d, 0x1403131300ull + l * 64 + d);
    std::vector<const char*> ptrs(n);
    for (int32_t i = 0; i < n; ++i) ptrs[i] = rows[i].data();
    pms_config best_cfg;
    PMS_TRY(tune_grid(c, {Shape{n, t, l, d}}, {ptrs.data()}, {c.cfg.variant}, 3, &best_cfg));
    c.cfg = best_cfg;
    if (!path.empty()) cache_store(path, key, best_cfg);
    if (best) *best = best_cfg;
    return PMS_OK;
}

int pms_autotune_many(const pms_instance* inst, int32_t count, const char* cache_path,
                      pms_config* best) {
    const TraceRange trace_range("pms_autotune_many");
    g_last_error.clear();
    if (!inst || count < 1) return fail(PMS_ERR_INVALID, "NULL batch or count < 1");
    std::vector<Shape> shapes;
    std::vector<const char* const*> rows;
    for (int32_t i = 0; i < count; ++i) {
        const pms_instance& q = inst[i];
        PMS_TRY(validate_shape(q.n, q.t, q.l, q.d));
        PMS_TRY(validate_rows(q.seqs, q.n, q.t));
        shapes.push_back({q.n, q.t, q.l, q.d});
        rows.push_back(q.seqs);
    }
    std::string path = cache_path ? cache_path : "";
    if (path.empty())
        if (const char* v = getenv("PMS_AUTOTUNE_CACHE")) path = v;
    std::unique_lock<std::mutex> lk(g_ctx.mu);
    Ctx& c = g_ctx;
    PMS_TRY(init_ctx(c));
    const std::string key = tune_key_many(c, shapes);
    pms_config found;
    if (!path.empty() && cache_lookup(path, key, &found)) {
        c.cfg = found;
        if (best) *best = found;
        return PMS_OK;
    }
    // The requested variant, and the 16-candidate kernel beside the
    // 64-candidate one when the choice is automatic: with low pass rates
    // the 64-candidate groups carry many dead members.
    std::vector<uint32_t> variants = {c.cfg.variant};
    if (c.cfg.variant == PMS_VARIANT_AUTO) variants.push_back(PMS_VARIANT_GROUP);
    pms_config best_cfg;
    PMS_TRY(tune_grid(c, shapes, rows, variants, 2, &best_cfg));
    c.cfg = best_cfg;
    if (!path.empty()) cache_store(path, key, best_cfg);
    if (best) *best = best_cfg;
    return PMS_OK;
}

int pms_valu_probe(int op, int32_t waves_per_simd, int32_t iters_in, pms_probe_result* out) {
    g_last_error.clear();
    if (!out || op < PMS_PROBE_XOR || op > PMS_PROBE_MOV64_S)
        return fail(PMS_ERR_INVALID, "bad probe op or NULL result");
    if (waves_per_simd < 0 || waves_per_simd > 16 || iters_in < 0 || iters_in > (1 << 24))
        return fail(PMS_ERR_INVALID, "probe size out of range");
    std::lock_guard<std::mutex> lk(g_ctx.mu);
    Ctx& c = g_ctx;
    PMS_TRY(init_ctx(c));
    // 256-thread blocks are 4 wavefronts, one per SIMD when spread evenly.
    const uint32_t blocks = static_cast<uint32_t>(c.cus) * (waves_per_simd ? waves_per_simd : 8);
    const uint32_t iters = iters_in ? static_cast<uint32_t>(iters_in) : 32768u;
    DevBuf sink, clocks;
    PMS_TRY(sink.ensure(static_cast<size_t>(blocks) * 256 * 4));
    PMS_TRY(clocks.ensure(16));
    float ms = 0;
    for (int rep = 0; rep < 2; ++rep) {  // the first launch warms up the clocks
        PMS_HIP(hipEventRecord(c.ev[0], c.stream));
        PMS_HIP(pms::valu_probe(op, blocks, iters, sink.as<uint32_t>(), clocks.as<uint64_t>(), c.stream));
        PMS_HIP(hipEventRecord(c.ev[1], c.stream));
        PMS_HIP(hipStreamSynchronize(c.stream));
        PMS_HIP(hipEventElapsedTime(&ms, c.ev[0], c.ev[1]));
    }
    uint64_t clk[2] = {0, 0};
    PMS_HIP(hipMemcpy(clk, clocks.p, 16, hipMemcpyDeviceToHost));
    (void)hipFree(sink.p);
    (void)hipFree(clocks.p);
    const double per_chain = op == PMS_PROBE_COMPARE ? 4.0 : 1.0;
    const double lane_ops = static_cast<double>(blocks) * 256.0 * iters * 16.0 * per_chain;
    out->ms = ms;
    out->lane_ops_per_s = lane_ops / (ms * 1e-3);
    out->sclk_mhz = clk[1] ? static_cast<double>(clk[0]) / (static_cast<double>(clk[1]) * 1e-8) / 1e6 : 0;
    out->compute_units = c.cus;
    out->reserved = 0;
    out->lane_ops_per_clk_per_cu =
        out->sclk_mhz > 0 ? out->lane_ops_per_s / (out->sclk_mhz * 1e6 * c.cus) : 0;
    return PMS_OK;
}

}  // extern "C"
