// pms_internal.h -- shared between the kernels and the host library (not
// part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pms.h"

// Stage-queue slots per sequence stage per wavefront.  At most one queue is
// ever at or above 64 entries and it is scanned before anything else is
// pushed, so every queue stays below 128.
#define PMS_QCAP 128u
// Single-candidate queue slots per stage (64-candidate kernel).  A singles
// scan pushes at most 64 onto a queue below 64; a group scan pushes sparse
// groups' members only while they fit.
#define PMS_SCAP 128u
// Per-wavefront staging slots for final survivors (flushed at > OUTBUF-64).
#define PMS_OUTBUF 256u
// Largest workgroup of the 64-candidates-per-lane kernel (4 wavefronts).
#define PMS_GROUP64_MAX_THREADS 256

// One row for the window-building kernel.
typedef struct {
    uint64_t src_off;  // byte offset of the row in the packed input
    uint64_t dst_off;  // uint32 offset of the row's windows
    int32_t t, l, stride, inst;  // t: this row's length
    int32_t layout, flags;        // flags: pms_input_flag bits
} pms_win_job;

namespace pms {

hipError_t launch_windows(const pms_win_job* jobs, int32_t rows, int32_t max_t,
                          const uint8_t* seqs, uint32_t* windows, uint32_t* bad,
                          hipStream_t stream);

hipError_t launch_search(const pms_dev_instance* insts, const pms_work_item* work,
                         uint32_t n_work, pms_dev_state* state, pms_dev_counters* ctr,
                         uint32_t q_words, uint32_t grid, uint32_t wg_waves, hipStream_t stream);

hipError_t launch_fill(uint32_t* p, uint64_t words, uint32_t v, hipStream_t stream);

// Copies, for each i < m, tab[3i+2] codes from src + tab[3i] to dst + tab[3i+1].
hipError_t launch_gather(const uint32_t* src, const uint64_t* tab, uint32_t m, uint32_t* dst,
                         hipStream_t stream);

// Neighbourhood-intersection method (pms_nbhd.hip).
hipError_t launch_nbhd_codes(const uint8_t* seqs, int32_t t, int32_t l, int32_t rows,
                             uint32_t* codes, hipStream_t stream);
// Bitmap lengths in words are multiples of 4 (16-byte vectors).
hipError_t launch_nbhd_zero(uint32_t* p, uint64_t words, uint32_t grid, hipStream_t stream);
// Pass counts come per workgroup (part[blockIdx]) and are summed by
// launch_nbhd_sum into one uint64.
hipError_t launch_nbhd_scatter(const uint32_t* codes, int32_t nw, const uint32_t* deltas,
                               int32_t nd, uint32_t* bitmap, uint32_t* fresh,
                               uint32_t grid, hipStream_t stream);
hipError_t launch_nbhd_and(uint32_t* m, const uint32_t* b, uint64_t words,
                           uint32_t* part, uint32_t grid, hipStream_t stream);
hipError_t launch_nbhd_sum(const uint32_t* part, uint32_t n, unsigned long long* total,
                           hipStream_t stream);
// One pass
// over a sequence: `tiles` workgroups of 2^T candidate bits (tile_words words
// each); group_off has tiles + 1 entries (masks sorted by their bits above T).
size_t nbhd_tile_lds_bytes(uint32_t tile_words);
// rec/rec_off (may be null): the tile's (window, group) records, as built by
// launch_nbhd_records; without them every tile looks up every window.
hipError_t launch_nbhd_tile(const uint32_t* codes, int32_t nw, const uint32_t* deltas,
                            const uint32_t* group_off, const uint32_t* rec,
                            const uint32_t* rec_off, int32_t T, uint32_t tiles,
                            uint32_t tile_words, uint32_t* m, bool first,
                            uint32_t* part, hipStream_t stream);
// Records of one pass: ne[0 .. nne) the non-empty mask groups; tcount and
// tcur hold tiles words, toff tiles + 1, rec nw x nne.
hipError_t launch_nbhd_records(const uint32_t* codes, int32_t nw, const uint32_t* ne, int32_t nne,
                               int32_t T, uint32_t tiles, uint32_t* tcount, uint32_t* toff,
                               uint32_t* tcur, uint32_t* rec, uint32_t grid, hipStream_t stream);
hipError_t launch_nbhd_collect(const uint32_t* m, uint64_t words, uint32_t* out, uint64_t cap,
                               unsigned long long* count, uint32_t grid, hipStream_t stream);
hipError_t launch_nbhd_verify(const uint32_t* cand, uint64_t count, const uint32_t* codes,
                              int32_t nw, int32_t s_begin, int32_t n, int32_t d, uint32_t* out,
                              uint64_t cap, unsigned long long* out_count,
                              unsigned long long* visits, uint32_t grid, hipStream_t stream);

const void* search_kernel_symbol();

// Where one pms_solve_dev_noalloc call keeps its tables inside the scratch
// (byte offsets from its start) and the work-item plan of its instance.
struct NoallocLayout {
    uint64_t off_win, off_inst, off_state, off_ctr, off_bad, off_jobs, off_work, off_gq, bytes;
    uint64_t size, small;       // candidates per head item / per tail item
    uint32_t n_head, n_items;   // head items; all items
    int32_t n, t, l, d, stride, layout;
};

// The scratch's device address and size (hipGetSymbolAddress; call with the
// device current).
hipError_t noalloc_scratch(void** ptr, size_t* bytes);
// Builds the call's records in the scratch (no host copy).
hipError_t launch_noalloc_setup(void* base, const NoallocLayout& lay, uint32_t* dev_out,
                                uint64_t capacity, hipStream_t stream);
// Copies the instance's motif count to *dev_count.
hipError_t launch_noalloc_count(const pms_dev_state* st, uint64_t* dev_count, hipStream_t stream);

// Launch flags of the grouped kernels.
#define PMS_LAUNCH_NO_FILTER 1u   // 64-candidate kernel: scan every window

// Where a grouped launch keeps its stage queues: the first lds_stages in LDS,
// the rest in gq (gq_words words per wavefront, grid x wg_waves wavefronts).
struct GroupQueues {
    uint32_t lds_stages;
    uint32_t* gq;
    uint32_t gq_words;
};

// suffix: 2 (16 candidates per lane) or 3 (64).
hipError_t launch_search_group(const pms_dev_instance* insts, const pms_work_item* work,
                               uint32_t n_work, pms_dev_state* state, pms_dev_counters* ctr,
                               const GroupQueues& q, uint32_t grid, uint32_t wg_waves,
                               hipStream_t stream, int suffix, uint32_t flags);

const void* search_group_kernel_symbol(int suffix);

hipError_t valu_probe(int op, uint32_t blocks, uint32_t iters, uint32_t* sink, uint64_t* clocks,
                      hipStream_t s);

// Words of one stage's queues per wavefront in the grouped kernels: suffix
// 2 keeps a uint32 prefix and a uint32 alive mask per group; suffix 3 a
// prefix and a uint64 mask per group, then PMS_SCAP single motif codes.
constexpr uint32_t stage_queue_words(int suffix) {
    return suffix == 3 ? 3u * PMS_QCAP + PMS_SCAP : 2u * PMS_QCAP;
}

// Suffix-vector table of the 64-candidate kernel's shared-prefix scans, per
// wavefront: 12 words per window group (4 mismatch vectors for each of the
// three suffix positions), so rows of up to 42 window groups use it.
#define PMS_SVT_WORDS 512u

// LDS words per wavefront of a grouped launch besides its stage queues:
// the survivor staging buffer and (suffix 3) the suffix-vector table.
constexpr uint32_t wave_fixed_words(int suffix) {
    return PMS_OUTBUF + (suffix == 3 ? PMS_SVT_WORDS : 0u);
}

// Words of stage queues one wavefront needs for instances of up to max_n
// sequences.  variant: LANE keeps one uint32 candidate per slot; the grouped
// variants as in stage_queue_words.
inline uint32_t queue_words(int32_t max_n, uint32_t variant) {
    const uint32_t stages = static_cast<uint32_t>(max_n > 1 ? max_n - 1 : 0);
    const uint32_t words = variant == PMS_VARIANT_GROUP64 ? stage_queue_words(3)
                           : variant == PMS_VARIANT_GROUP ? stage_queue_words(2)
                                                          : PMS_QCAP;
    return stages * words;
}

// Candidates per lane of a variant.
inline uint32_t candidates_per_lane(uint32_t variant) {
    return variant == PMS_VARIANT_GROUP64 ? 64u : variant == PMS_VARIANT_GROUP ? 16u : 1u;
}

}  // namespace pms
