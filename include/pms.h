/*
 * pms.h -- exact planted (l, d) motif search (Skip-Brute-Force) on one
 * AMD Instinct MI355X (gfx950).  C ABI: plain pointers and sizes.
 *
 * The operation (Section I.A, the planted (l, d) motif problem; Section
 * III.A, the enhanced brute force): given n DNA sequences of length t, the
 * result is every l-mer x over {A, C, G, T} such that every sequence has a
 * window (a length-l substring at any start 0 .. t-l, t-l+1 of them) within
 * Hamming distance d of x.  All 4^l l-mers are candidates; a candidate is
 * rejected at the first sequence that has no such window, and the remaining
 * sequences are not examined (the enhanced rule of Section III.A).  The
 * candidate space is split into numbered index ranges that workers claim and
 * generate on the fly (Section IV.A).
 *
 * Motif code: base p of the l-mer (p = 0 leftmost) occupies bits
 * [2(l-1-p), 2(l-1-p)+1], with A=0, C=1, G=2, T=3.  Ascending codes are the
 * dictionary order of the strings (A < C < G < T).  Codes fit in uint32
 * because l <= 16.
 *
 * Threading: every entry point may be called from several host threads; the
 * host-level calls serialise on one library lock per device.  Device-level
 * calls are asynchronous on the caller's stream.
 *
 * Errors: no entry point aborts or throws.  Each returns a pms_status; on a
 * non-OK status pms_last_error() returns a message for the calling thread.
 */
#ifndef PMS_H
#define PMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes returned by every entry point. */
enum pms_status {
    PMS_OK = 0,
    PMS_ERR_INVALID = 1,  /* bad argument; nothing was written except *count = 0 */
    PMS_ERR_OVERFLOW = 2, /* more motifs than capacity; see each entry point */
    PMS_ERR_NOMEM = 3,    /* device or pinned host memory could not be allocated */
    PMS_ERR_DEVICE = 4    /* a HIP runtime call failed; detail in pms_last_error() */
};

/* Limits checked by every entry point (PMS_ERR_INVALID beyond them).
 * l: codes are 32-bit.  n: per-wavefront stage bookkeeping holds one stage
 * per lane of a 64-wide wavefront.  t: one row, packed 16 bases per word,
 * is staged in the LDS of one workgroup. */
#define PMS_MAX_L 16
#define PMS_MAX_N 64
#define PMS_MAX_T (1 << 17)

/*
 * pms_solve -- one instance, host buffers in and out, synchronous.  The
 * problem of Section I.A solved by the enhanced brute force of Section III.A
 * (every l-mer a candidate; a candidate is dropped at the first sequence
 * without a window within d), the candidate numbers split into index ranges
 * as in Section IV.A.
 *
 *   seqs        n pointers, each to at least t bytes of A/C/G/T (either
 *               case); no terminator needed.  Read only; nothing retained.
 *   n, t, l, d  1 <= n <= PMS_MAX_N, 1 <= l <= PMS_MAX_L, l <= t <= PMS_MAX_T,
 *               0 <= d <= l.
 *   out_motifs  caller-owned array of *out_count (on entry) uint32 slots; may
 *               be NULL only when *out_count == 0 on entry.
 *   out_count   in: capacity of out_motifs.  out: |M|, the exact number of
 *               motifs (also on PMS_ERR_OVERFLOW; 0 on PMS_ERR_INVALID).
 *
 * On PMS_OK out_motifs[0 .. |M|) holds M ascending, without duplicates.
 * If |M| exceeds the capacity the smallest `capacity` motifs are written,
 * ascending, and PMS_ERR_OVERFLOW is returned; capacity 0 is a size query.
 * PMS_ERR_INVALID (NULL pointer, size out of range, a byte that is not a
 * base) writes nothing to out_motifs.
 */
int pms_solve(const char* const* seqs, int32_t n, int32_t t, int32_t l, int32_t d,
              uint32_t* out_motifs, uint64_t* out_count);

/*
 * pms_solve_ex -- pms_solve for sequences of their own lengths, with options
 * (pms_input_flag): seqs[i] has lengths[i] bytes, l <= lengths[i] <=
 * PMS_MAX_T.  The window set of sequence i is every length-l substring (none
 * holding N under PMS_INPUT_MASK_N), plus their reverse complements under
 * PMS_INPUT_BOTH_STRANDS; M is defined over these sets as for pms_solve.
 * A sequence with no window leaves M empty (PMS_OK, |M| = 0, no device
 * work).  Same output, capacity and error semantics as pms_solve; lengths
 * NULL or an unknown flag is PMS_ERR_INVALID.
 */
int pms_solve_ex(const char* const* seqs, int32_t n, const int32_t* lengths, int32_t l,
                 int32_t d, uint32_t flags, uint32_t* out_motifs, uint64_t* out_count);

/*
 * pms_solve_intersect -- the same result as pms_solve by a second exact
 * method: M is the intersection over sequences of the union of the
 * distance-d neighbourhoods (Hamming balls) of each sequence's windows, the
 * sample-driven form of the Planted Motif Search family that Section VI names
 * as future work.  The GPU keeps the candidate space as a 4^l-bit map
 * (2^(2l-3) bytes of device memory, 512 MiB at l = 16); per sequence each
 * workgroup sets the bits of every window's neighbours in one 2^18-bit tile
 * of it in LDS and ANDs the tile into the map, and the passes stop early when
 * no candidate is left.  Work per sequence: (t-l+1) x
 * |Ball| bit sets, |Ball| = sum_{k<=d} C(l,k) 3^k; far less than the sweep
 * when d is small against l, far more when it is not.  Arguments, output and
 * errors as for pms_solve; PMS_ERR_INVALID also when |Ball| exceeds
 * PMS_NBHD_MAX_BALL.  Once the candidates left are few enough that checking
 * them against the remaining sequences costs less than another bitmap pass,
 * they are checked directly (with the enhanced rule).  pms_last_stats
 * reports the device time (kernel_ms), the bitmap passes (batches), the bits
 * set (window_compares) and the direct (candidate, sequence) checks
 * (seq_visits).
 */
#define PMS_NBHD_MAX_BALL (1u << 24)
int pms_solve_intersect(const char* const* seqs, int32_t n, int32_t t, int32_t l, int32_t d,
                        uint32_t* out_motifs, uint64_t* out_count);

/* One instance of a batched solve (host buffers). */
typedef struct {
    const char* const* seqs; /* n pointers to >= t bytes each, as for pms_solve */
    int32_t n, t, l, d;
    uint32_t* out_motifs;    /* caller-owned, `capacity` slots; NULL iff capacity 0 */
    uint64_t capacity;
} pms_instance;

/* Per-instance outcome of a batched solve. */
typedef struct {
    int32_t status;    /* pms_status of this instance */
    int32_t reserved;
    uint64_t count;    /* |M| (exact, also on PMS_ERR_OVERFLOW) */
    double latency_ms; /* device time from the launch's first claim to this
                          instance's last work item retiring */
} pms_result;

/*
 * pms_solve_many -- many independent instances of uneven (l, d, n, t) in one
 * persistent launch, each solved by the method of Section III.A as in
 * pms_solve (the paper runs one instance per program run; sharing one launch
 * among many is this library's) (replayed from a captured HIP graph when the batch has
 * the same layout as the previous call).  Same per-instance semantics as
 * pms_solve.  An invalid instance gets PMS_ERR_INVALID and does not stop the
 * others.  Returns PMS_OK when every instance is OK, else the first non-OK
 * instance status (PMS_ERR_INVALID for bad `inst`/`count`/`results`).
 */
int pms_solve_many(const pms_instance* inst, int32_t count, pms_result* results);

/* Writes the l characters of motif `code` to out (no terminator); the code's
 * base order A < C < G < T is the dictionary order of the strings (the paper
 * fixes no encoding). */
void pms_decode(uint32_t code, int32_t l, char* out);

/* Sorts `count` motif codes of length l ascending in place (step a7 for
 * codes a device-level caller copied back unsorted; a least-significant-digit
 * radix sort over the codes' 2l bits above 4096 codes).  PMS_ERR_INVALID for
 * l out of range, NULL codes with count > 0 or a code with bits above 2l
 * (nothing is reordered then); PMS_ERR_DEVICE if two codes are equal (a
 * motif set has none; the codes are sorted all the same). */
int pms_sort_codes(uint32_t* codes, uint64_t count, int32_t l);

/* Static text for a status code. */
const char* pms_status_string(int status);

/* Message for the calling thread's last non-OK status ("" if none). */
const char* pms_last_error(void);

/* ------------------------------------------------------------------------ *
 * Launch configuration and tuning
 * ------------------------------------------------------------------------ */

/* Search kernel variants (pms_config.variant). */
enum pms_variant {
    PMS_VARIANT_AUTO = 0,   /* GROUP64 when every instance of a launch has l >= 3, else GROUP
                               when every instance has l >= 2, else LANE */
    PMS_VARIANT_LANE = 1,   /* one candidate per lane; per window v_xor + v_or_b32_sdwa +
                               v_bcnt + v_min3 (bit-plane window layout) */
    PMS_VARIANT_GROUP = 2,  /* 16 candidates sharing l-2 bases per lane; 32 windows per
                               register, carry-save counts (bit-sliced layout); l >= 2 */
    PMS_VARIANT_GROUP64 = 3 /* 64 candidates sharing l-3 bases per lane (bit-sliced
                               layout); l >= 3 */
};

/* Window table layouts (pms_build_windows). */
enum pms_layout {
    PMS_LAYOUT_PLANES = 0,    /* [row][window] uint32: high plane << 16 | low plane */
    PMS_LAYOUT_BITSLICED = 1  /* [row][group of 32 windows][2l] uint32: word p has bit j =
                                 high bit of base p of window 32g+j, word l+p the low bit */
};

/* Input options of pms_solve_ex (bit flags).  The reading of the
 * real-sequence future work of Section VI:
 *   PMS_INPUT_MASK_N        bytes N/n are allowed; a window holding one is
 *                           not a window of its sequence.
 *   PMS_INPUT_BOTH_STRANDS  a sequence's windows also include the reverse
 *                           complement of each of its windows (read
 *                           backwards, A<->T, C<->G). */
enum pms_input_flag {
    PMS_INPUT_MASK_N = 1,
    PMS_INPUT_BOTH_STRANDS = 2
};

/* Window filter of the 64-candidate kernel (pms_config.filter).  When the
 * live groups of a sequence scan all share their first l-6 bases, a window
 * whose mismatches on those bases already exceed d cannot match any of their
 * candidates; the filter scans only the other windows (re-sliced into dense
 * 32-window groups).  Exact: the same motifs, the same sequence visits.  An
 * extension of the enhanced rule of Section III.A, not part of the paper's
 * method; OFF gives the unfiltered scan for comparison. */
enum pms_filter {
    PMS_FILTER_DEFAULT = 0, /* ON */
    PMS_FILTER_ON = 1,
    PMS_FILTER_OFF = 2
};

/* Shape of the persistent search launch.  Zero fields mean "default". */
typedef struct {
    uint32_t chunk;        /* least candidates per work item (multiple of 64; default
                              4096); items are rounded up to multiples of 4096 candidates
                              for l >= 6, and a launch cuts each instance into items in
                              proportion to its work, about 8 per resident wavefront for
                              one instance and 32 for a batch */
    uint32_t wg_waves;     /* 64-lane wavefronts per workgroup (1..16) */
    uint32_t wgs_per_cu;   /* resident workgroups per compute unit (0 = as many as fit) */
    uint32_t tail_split;   /* work items of the last tail_split/64 of each instance are
                              cut 4x smaller, so the launch ends evenly (0..64; the
                              default, 0, splits nothing) */
    uint32_t variant;      /* pms_variant */
    uint32_t filter;       /* pms_filter: window filter of the 64-candidate kernel */
} pms_config;

/* Sets the configuration used by later calls that pass no configuration
 * (NULL restores the defaults).  PMS_ERR_INVALID for out-of-range fields.
 * The launch shape is this library's; the paper's one knob is the number of
 * threads that share the index ranges (Section IV.A). */
int pms_set_config(const pms_config* cfg);
int pms_get_config(pms_config* cfg);

/*
 * pms_autotune -- (launch shape, not part of the paper's method) times the
 * candidate-chunk x workgroup-shape grid on one
 * instance shape (FM synthetic data drawn inside the library from a fixed
 * seed) and makes the fastest the current configuration.  The result is
 * cached in the JSON file named by cache_path (or $PMS_AUTOTUNE_CACHE when
 * cache_path is NULL; no caching when both are absent), keyed by GPU
 * architecture, compute-unit count and shape bucket.  best may be NULL.
 */
int pms_autotune(int32_t n, int32_t t, int32_t l, int32_t d, const char* cache_path,
                 pms_config* best);

/*
 * pms_autotune_many -- (launch shape, not part of the paper's method) times
 * the same grid on a batch itself (its own instances, eager launches), with
 * the 16-candidate kernel beside the 64-candidate one when the current
 * variant is AUTO, and makes the fastest the current configuration, for
 * pms_solve_many on that batch.  Cached as for pms_autotune under a key made
 * of the build, the device and a hash of the instances' shapes.  Instances
 * as for pms_solve_many (capacities unused); PMS_ERR_INVALID for an invalid
 * one.  best may be NULL.
 */
int pms_autotune_many(const pms_instance* inst, int32_t count, const char* cache_path,
                      pms_config* best);

/* Counters of the last solve on this device.  seq_visits counts the
 * (candidate, sequence) scans that the enhanced rule of Section III.A makes,
 * the method's own work; the others describe this library's launches.  After a device-level call
 * (pms_solve_dev, pms_step_launch) pms_last_stats waits for that call's
 * kernels and for its counters, which pms_solve_dev copies to pinned host
 * memory on the caller's stream right after the search. */
typedef struct {
    double kernel_ms;        /* search kernel, HIP events on its own stream */
    double windows_ms;       /* window-building kernel, HIP events */
    uint64_t seq_visits;     /* (candidate, sequence) scans = algorithmic work of the
                                enhanced rule; times the window count it is the
                                algorithmic window-compare count */
    uint64_t batches;        /* wavefront sequence scans executed */
    uint64_t window_compares;/* sum over instances of seq_visits x (t-l+1) */
    uint64_t candidate_slots;/* candidate scan slots executed: 64 per lane-candidate of
                                each batch (1, 16 or 64 per lane; 1 in GROUP64's
                                single-candidate scans) */
    uint32_t grid;           /* workgroups launched */
    uint32_t wg_waves;
    uint32_t chunk;
    uint32_t reruns;         /* relaunches caused by device output overflow */
    uint32_t variant;        /* pms_variant actually launched (LANE, GROUP or GROUP64) */
    uint32_t work_items;     /* work items in the launch's table (the claims it makes) */
    double host_prep_ms;     /* host-level calls: validation, planning and staging before
                                the launch (0 for device-level calls) */
    double host_finish_ms;   /* host-level calls: copy-back, sort and capacity handling
                                after the launch, reruns included (0 for device-level) */
    uint64_t single_batches; /* of `batches`: GROUP64 scans of one candidate per lane */
    uint64_t filtered_batches; /* of `batches`: group scans through the window filter
                                  (pms_filter); the rest of those batches' windows
                                  were skipped */
    uint64_t filtered_groups;  /* dense 32-window groups the filtered scans ran */
} pms_stats;

int pms_last_stats(pms_stats* out);

/* ------------------------------------------------------------------------ *
 * Measurement
 * ------------------------------------------------------------------------ */

/* Instruction kinds timed by pms_valu_probe. */
enum pms_probe_op {
    PMS_PROBE_XOR = 0,     /* v_xor_b32 */
    PMS_PROBE_BCNT = 1,    /* v_bcnt_u32_b32 */
    PMS_PROBE_MIN3 = 2,    /* v_min3_u32 */
    PMS_PROBE_OR_SDWA = 3, /* v_or_b32_sdwa (16-bit halves) */
    PMS_PROBE_ADD = 4,     /* v_add_u32 */
    PMS_PROBE_FMA_F32 = 5, /* v_fma_f32, for comparison with the published fp32 rate */
    PMS_PROBE_XOR_VV = 6,  /* v_xor_b32 with two VGPR sources */
    PMS_PROBE_COMPARE = 7, /* the search loop's compare: xor, or_sdwa, bcnt, min3 (4 ops) */
    PMS_PROBE_MOV_S = 8,   /* v_mov_b32 from an SGPR */
    PMS_PROBE_MOV64_S = 9  /* v_mov_b64 from an SGPR pair (one op per 64-bit move) */
};

typedef struct {
    double lane_ops_per_s;           /* achieved lane-operations per second, whole GPU */
    double ms;                       /* probe kernel time (HIP events) */
    double sclk_mhz;                 /* engine clock during the run (shader-clock counter
                                        over the 100 MHz real-time counter) */
    double lane_ops_per_clk_per_cu;  /* lane_ops_per_s / (sclk * compute units) */
    int32_t compute_units;
    int32_t reserved;
} pms_probe_result;

/*
 * pms_valu_probe -- issue rate of one VALU instruction kind: every lane of
 * `waves_per_simd` x 4 wavefronts per compute unit runs 16 independent chains
 * of the instruction for `iters` iterations (0 = defaults 8 and 32768).  Used to state the integer VALU roofline of the
 * search kernel from measurement rather than assumption.
 */
int pms_valu_probe(int op, int32_t waves_per_simd, int32_t iters, pms_probe_result* out);

/* ------------------------------------------------------------------------ *
 * Device level: device pointers, caller's stream (hipStream_t as void*; NULL
 * is the null stream).  Asynchronous: results are valid once the stream is
 * synchronised.  The caller owns every buffer passed in.
 * ------------------------------------------------------------------------ */

/* Number of uint32 words per sequence row of a window table for length t,
 * motif length l and `layout`: PLANES, t-l+1 rounded up to a multiple of 16;
 * BITSLICED, 2l per group of 32 windows (0 for invalid sizes, and for
 * BITSLICED with l < 2). */
int32_t pms_window_stride(int32_t t, int32_t l, int32_t layout);

/*
 * pms_build_windows -- steps a1+a2, the windows of every sequence that
 * Section III.A extracts before the comparisons: encodes n rows of t bytes
 * (row-major at dev_seqs, device memory) into 2-bit codes, stages each row
 * in LDS, and writes every window of length l to
 * dev_windows[n][pms_window_stride(t, l, layout)].  PLANES: window j is (high-bit plane of base p in bit 16+l-1-p,
 * low-bit plane in bit l-1-p).  BITSLICED: see pms_layout.  Window slots past
 * t-l+1 repeat window 0.  Bytes that are not A/C/G/T (either case) set
 * *dev_bad (device uint32) to 1; dev_bad may be NULL.  Asynchronous on
 * `stream`; the call does not wait for work already queued there (its job
 * table goes through one of 8 staging slots that are reused in turn).
 */
int pms_build_windows(const uint8_t* dev_seqs, int32_t n, int32_t t, int32_t l, int32_t layout,
                      uint32_t* dev_windows, uint32_t* dev_bad, void* stream);

/* Device-resident description of one instance for pms_step_launch. */
typedef struct {
    const uint32_t* windows; /* [n][nw_stride] from pms_build_windows, in the layout of
                                the launch's variant (LANE: PLANES, GROUP: BITSLICED) */
    uint32_t* out;           /* motif codes, unsorted, up to out_cap of them */
    uint64_t out_cap;
    int32_t n, nw_stride, l, d;
} pms_dev_instance;

/* One work item: candidates [begin, begin+len) of instance `inst`.  LANE
 * numbers candidates in bit-plane order (candidate k has high plane k >> l and
 * low plane k & (2^l - 1)); GROUP and GROUP64 in dictionary order (k is the
 * motif code), and there begin and len must be multiples of 16 and 64.  Either way the items of
 * an instance must cover [0, 4^l) once.  len is at most 2^31. */
typedef struct {
    uint64_t begin;
    uint32_t len;
    uint32_t inst;
} pms_work_item;

/* Per-instance device state.  Before a launch: count = visits = t_done = 0
 * and items_left = number of work items of the instance in the launch. */
typedef struct {
    uint64_t count;      /* motifs found (keeps counting past out_cap) */
    uint64_t visits;     /* (candidate, sequence) scans */
    uint64_t t_done;     /* device realtime stamp (100 MHz) when items_left hit 0 */
    uint32_t items_left;
    uint32_t reserved;
} pms_dev_state;

/* Launch-wide device counters; all zero before a launch. */
typedef struct {
    uint32_t next_item;  /* work-claim counter */
    uint32_t error;      /* set to 1 if an instance had n > max_n (its items are skipped) */
    uint64_t batches;    /* 64-lane sequence scans executed */
    uint64_t t_start;    /* realtime stamp of the first claim */
    uint64_t single_batches; /* of those, scans of one candidate per lane (GROUP64) */
    uint64_t filtered_batches; /* of those, group scans through the window filter */
    uint64_t filtered_groups;  /* dense 32-window groups those scans ran */
} pms_dev_counters;

/*
 * pms_step_launch -- steps a3-a6 of the sweep of Section III.A (candidates
 * generated from their index numbers, compared window by window, dropped at
 * the first sequence without a match, survivors output) over caller-built
 * index ranges as in Section IV.A: one persistent search launch over the
 * work items dev_work[0 .. n_work).  Each instance's survivors are appended
 * (unsorted, as motif codes) to its `out`; its state counts them.  cfg may be
 * NULL (current configuration); its variant selects the kernel and so the
 * window layout the instances must have (AUTO means GROUP64 here).
 * n_inst/n_work are the table lengths; max_n is the largest n over the
 * instances the items reference (it sizes LDS; an instance with more
 * sequences is refused and sets the counters' error flag).
 */
int pms_step_launch(const pms_dev_instance* dev_instances, int32_t n_inst, int32_t max_n,
                    const pms_work_item* dev_work, int32_t n_work,
                    pms_dev_state* dev_state, pms_dev_counters* dev_counters,
                    const pms_config* cfg, void* stream);

/*
 * pms_fill_work_items -- host helper for callers that build the work tables
 * of pms_step_launch themselves (index ranges of Section IV.A): writes the
 * items covering candidates [begin, begin + count) of instance `inst`, in
 * ranges of item_len candidates (the last one shorter), to out[0 ..),
 * stopping after max_items.  Returns the number of items written; the
 * candidates they cover are min(count, items x item_len).  -1 (nothing
 * written) for item_len 0, NULL out with max_items > 0, or a range that
 * passes 2^32 candidates.
 */
int32_t pms_fill_work_items(uint64_t begin, uint64_t count, uint32_t item_len, uint32_t inst,
                            pms_work_item* out, int32_t max_items);

/*
 * pms_solve_dev -- the whole device part of one solve (Section III.A's method
 * on device buffers) on the caller's stream:
 * builds windows, lays out work items, and runs the search.  dev_seqs holds
 * n*t bytes row-major on the device.  Motif codes are appended, unsorted, to
 * dev_out (capacity `capacity`); *dev_count (device uint64) receives |M|
 * (exact, also when it exceeds capacity).  Workspace is owned by the library
 * and reused; the call is asynchronous.  Calls must be ordered: on one
 * stream, or a later call on another stream only after the earlier one has
 * completed.  A call with the same shape and configuration as the previous
 * one reuses its window jobs and work table on the device and uploads only
 * the per-call records.  Invalid bytes are not checked here (use
 * pms_build_windows's flag or the host-level calls).
 */
int pms_solve_dev(const uint8_t* dev_seqs, int32_t n, int32_t t, int32_t l, int32_t d,
                  uint32_t* dev_out, uint64_t capacity, uint64_t* dev_count, void* stream);

/*
 * pms_shutdown -- releases every device and pinned-host resource the library
 * holds for the device (stream, events, the captured graph, workspaces,
 * staging buffers; the fixed scratch of pms_solve_dev_noalloc is a static
 * array and stays), after waiting for all work on the device, including
 * device-level calls still running on callers' streams.  A later call
 * creates them again.  Meant for the end of a process (the Python binding
 * registers it to run at interpreter exit), so that no library-owned HIP
 * object outlives the HIP runtime's own teardown; no other thread may be
 * inside the library meanwhile.  PMS_OK, or PMS_ERR_DEVICE with the first
 * failing release named in pms_last_error() (the rest are still released).
 * Makes no HIP call when the library never touched a device.
 */
int pms_shutdown(void);

/*
 * pms_solve_dev_noalloc -- pms_solve_dev for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and ordering
 * rules as pms_solve_dev; the caller still owns dev_seqs, dev_out and
 * dev_count.  Everything else the solve needs (window table, instance and
 * work records, stage-queue workspace) lives in one fixed array of
 * PMS_NOALLOC_SCRATCH_BYTES per device, held by the library until the process
 * ends; the records are rebuilt and the counters cleared on the device by
 * every call, so the call makes no hipMalloc, hipFree, host-to-device copy or
 * memset.  All calls on one device share that array: calls that overlap on
 * the device (two streams, or two threads without ordering) race and give
 * wrong results.  When the stage queues of a full-occupancy launch do not fit
 * beside the tables, fewer workgroups are launched (same result, slower);
 * PMS_ERR_INVALID when the tables and one workgroup's queues exceed the array
 * (not reachable within PMS_MAX_N / PMS_MAX_T today).  pms_last_stats reports
 * only the launch shape after this call (no timings or counters).
 */
#define PMS_NOALLOC_SCRATCH_BYTES (128u << 20)
int pms_solve_dev_noalloc(const uint8_t* dev_seqs, int32_t n, int32_t t, int32_t l, int32_t d,
                          uint32_t* dev_out, uint64_t capacity, uint64_t* dev_count,
                          void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PMS_H */
