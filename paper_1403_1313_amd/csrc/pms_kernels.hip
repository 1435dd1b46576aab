// pms_kernels.hip -- gfx950 kernels of the planted (l, d) motif search.
//
// Two kernels make up one solve:
//
//   pms_windows_kernel  (steps a1 + a2)  One workgroup per sequence row.  The
//       row's bytes are encoded to 2-bit codes (A=0 C=1 G=2 T=3), packed 16
//       bases per 32-bit word into LDS, and every window of length l (the t-l+1
//       substrings of Section III.A) is written out in bit-plane form:
//       bit 16 + (l-1-p) holds the high bit of base p and bit (l-1-p) its low
//       bit.  Rows are padded to a multiple of 16 windows with copies of
//       window 0 (a repeated window cannot change a minimum).
//
//   pms_search_kernel   (steps a3 - a6)  Persistent workgroups; every 64-lane
//       wavefront works on its own.  It claims numbered work items (index
//       ranges of candidate l-mers, Section IV.A) with one global atomic and
//       generates the candidates of a range on the fly.  A wavefront always
//       scans 64 candidates against ONE sequence s at a time, so the window
//       index and the sequence are wave-uniform and every window arrives through
//       the scalar data cache as an SGPR operand: one compare is
//       v_xor (candidate ^ window), v_or_b32_sdwa (merge the two bit planes),
//       v_bcnt (mismatching positions) and half a v_min3 (running minimum).
//       Candidates whose minimum over the windows of s exceeds d are dropped
//       on the spot and never see sequences s+1.. (the enhanced rule of
//       Section III.A, applied per lane); the others are appended to an LDS
//       queue for stage s+1 through a wavefront ballot + mbcnt prefix.  A
//       queue that reaches 64 entries is scanned next, deepest stage first,
//       so the queues stay below 128 entries and no lane idles on a candidate
//       that already failed.  Candidates that pass the last sequence are
//       converted to motif codes and staged in a per-wavefront LDS buffer
//       that is flushed with a single global atomicAdd per flush.
//
// Candidates are numbered in bit-plane order inside the kernel: candidate k
// has high plane k >> l and low plane k & (2^l - 1).  This enumerates the same
// set as the dictionary order; survivors are converted to the dictionary code
// (bit 2q+1 = high-plane bit q, bit 2q = low-plane bit q) when written out.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pms.h"
#include "pms_device.h"
#include "pms_internal.h"

namespace {

using namespace pms_dev;

// (x >> 16) | (x & 0xffff) in one instruction: the OR of the two bit planes
// of an XOR difference marks every mismatching base position.
__device__ __forceinline__ uint32_t or_planes(uint32_t x) {
    uint32_t r;
    asm("v_or_b32_sdwa %0, %1, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 "
        "src1_sel:WORD_0"
        : "=v"(r)
        : "v"(x));
    return r;
}

__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Inserts a zero bit above every bit of a 16-bit value.
__device__ __forceinline__ uint32_t spread16(uint32_t x) {
    x &= 0xffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

// Bit-plane candidate -> motif code (first base in the top digit).
__device__ __forceinline__ uint32_t plane_to_code(uint32_t c) {
    return (spread16(c >> 16) << 1) | spread16(c);
}

// Smallest mismatch count between `cand` and the windows W[0 .. 16*groups).
// W is wave-uniform, so its words are scalar loads.
__device__ __forceinline__ uint32_t scan_sequence(cu32* W, uint32_t groups, uint32_t cand) {
    uint32_t a0 = 0xffu, a1 = 0xffu;
    for (uint32_t g = 0; g < groups; ++g, W += 16) {
#pragma unroll
        for (int k = 0; k < 16; k += 4) {
            const uint32_t m0 = __builtin_popcount(or_planes(cand ^ W[k + 0]));
            const uint32_t m1 = __builtin_popcount(or_planes(cand ^ W[k + 1]));
            const uint32_t m2 = __builtin_popcount(or_planes(cand ^ W[k + 2]));
            const uint32_t m3 = __builtin_popcount(or_planes(cand ^ W[k + 3]));
            a0 = min3u(a0, m0, m1);
            a1 = min3u(a1, m2, m3);
        }
    }
    return a0 < a1 ? a0 : a1;
}

}  // namespace

// --------------------------------------------------------------------------
// Steps a1 + a2: encode, pack into LDS, write the window table.
//
// Window slots of a row: slot w < nw = t-l+1 is the window starting at w;
// with both strands, slot nw + k is the reverse complement of window k (read
// backwards, base b -> 3 - b); remaining slots up to the table's stride
// repeat the row's first window.  With N masking a window holding an N is
// not a window: its slot repeats the first N-free window instead.  A repeated
// window cannot change a minimum, so the table holds exactly the row's window
// set.  (A row with no N-free window is never launched: its instance has no
// motifs.)
// --------------------------------------------------------------------------
namespace {

// Bits [j, j+l) of the N map are all clear (l <= 16; the map has a spare
// word past the row).
__device__ __forceinline__ bool n_free(const uint32_t* nbits, int j, int l) {
    const uint64_t two = (static_cast<uint64_t>(nbits[(j >> 5) + 1]) << 32) | nbits[j >> 5];
    return ((two >> (j & 31)) & ((1ull << l) - 1)) == 0;
}

// Source of window slot w: its start and whether it is read as a reverse
// complement.
__device__ __forceinline__ void slot_source(int w, int nw, int j0, bool mask_n, bool both,
                                            const uint32_t* nbits, int l, int& start, bool& rc) {
    start = j0;
    rc = false;
    if (w < nw) {
        if (!mask_n || n_free(nbits, w, l)) start = w;
    } else if (both && w < 2 * nw) {
        const int k = w - nw;
        if (!mask_n || n_free(nbits, k, l)) {
            start = k;
            rc = true;
        }
    }
}

// Base p of the window starting at `start` (reverse complement when rc).
__device__ __forceinline__ uint32_t slot_base(const uint32_t* packed, int start, bool rc, int p,
                                              int l) {
    const int pos = rc ? start + (l - 1 - p) : start + p;
    const uint32_t b = (packed[pos >> 4] >> (2 * (pos & 15))) & 3u;
    return rc ? (b ^ 3u) : b;
}

}  // namespace

extern "C" __global__ void __launch_bounds__(256)
pms_windows_kernel(const pms_win_job* __restrict__ jobs, const uint8_t* __restrict__ seqs,
                   uint32_t* __restrict__ windows, uint32_t* __restrict__ bad) {
    extern __shared__ uint32_t packed[];
    const pms_win_job job = jobs[blockIdx.x];
    const uint8_t* row = seqs + job.src_off;
    const int t = job.t, l = job.l, stride = job.stride;
    const bool mask_n = (job.flags & PMS_INPUT_MASK_N) != 0;
    const bool both = (job.flags & PMS_INPUT_BOTH_STRANDS) != 0;
    const int words = (t + 15) >> 4;
    const int nwords = (t + 31) >> 5;
    uint32_t* const nbits = packed + words + 1;                      // bit q: base q is N
    int* const first = reinterpret_cast<int*>(nbits + nwords + 1);  // first N-free window
    const int nw = t - l + 1;

    for (int i = threadIdx.x; i <= nwords; i += blockDim.x) nbits[i] = 0;
    if (threadIdx.x == 0) {
        packed[words] = 0;  // a window may read one word past the row
        *first = nw;
    }
    __syncthreads();

    // a1: 16 bases per word, base q of the word in bits [2q, 2q+1].
    bool saw_bad = false;
    for (int w = threadIdx.x; w < words; w += blockDim.x) {
        uint32_t v = 0, nb = 0;
        const int q_end = min(16, t - 16 * w);
        for (int q = 0; q < q_end; ++q) {
            const uint32_t c = row[16 * w + q] | 0x20u;  // fold upper case onto lower
            uint32_t code;
            if (c == 'a') code = 0;
            else if (c == 'c') code = 1;
            else if (c == 'g') code = 2;
            else if (c == 't') code = 3;
            else if (c == 'n' && mask_n) { code = 0; nb |= 1u << q; }
            else { code = 0; saw_bad = true; }
            v |= code << (2 * q);
        }
        packed[w] = v;
        if (nb) atomicOr(&nbits[w >> 1], nb << (16 * (w & 1)));
    }
    if (saw_bad && bad) bad[job.inst] = 1u;
    __syncthreads();
    if (mask_n) {
        for (int j = threadIdx.x; j < nw; j += blockDim.x)
            if (n_free(nbits, j, l)) {
                atomicMin(first, j);
                break;
            }
        __syncthreads();
    }
    const int j0 = *first < nw ? *first : 0;

    // a2: the window slots of the row.
    uint32_t* dst = windows + job.dst_off;
    if (job.layout == PMS_LAYOUT_PLANES) {
        for (int j = threadIdx.x; j < stride; j += blockDim.x) {
            int start;
            bool rc;
            slot_source(j, nw, j0, mask_n, both, nbits, l, start, rc);
            uint32_t hi = 0, lo = 0;
            for (int p = 0; p < l; ++p) {
                const uint32_t b = slot_base(packed, start, rc, p, l);
                hi |= (b >> 1) << (l - 1 - p);
                lo |= (b & 1u) << (l - 1 - p);
            }
            dst[j] = (hi << 16) | lo;
        }
    } else {
        // Bit-sliced: word (g, p) bit j is the high bit of base p of window
        // slot 32g+j, word (g, l+p) the low bit.  Each lane takes one window
        // slot and builds its code; per base and plane one ballot over the
        // wavefront's 64 slots gives the words of its two window groups,
        // which writelane gathers into lanes 0..2l-1 of two registers.
        const int groups = stride / (2 * l);
        const int lane = static_cast<int>(threadIdx.x & 63u);
        const int waves = static_cast<int>(blockDim.x >> 6);
        for (int g2 = static_cast<int>(threadIdx.x >> 6); 2 * g2 < groups; g2 += waves) {
            const int w = 64 * g2 + lane;
            int start;
            bool rc;
            slot_source(w, nw, j0, mask_n, both, nbits, l, start, rc);
            uint32_t code = 0;
            for (int p = 0; p < l; ++p) code = (code << 2) | slot_base(packed, start, rc, p, l);
            int lo = 0, hi = 0;
            for (int p = 0; p < l; ++p) {
                const int sh = 2 * (l - 1 - p);
                const uint64_t bh = __builtin_amdgcn_ballot_w64(((code >> (sh + 1)) & 1u) != 0u);
                const uint64_t bl = __builtin_amdgcn_ballot_w64(((code >> sh) & 1u) != 0u);
                lo = pms_dev::write_lane(static_cast<int>(static_cast<uint32_t>(bh)), p, lo);
                hi = pms_dev::write_lane(static_cast<int>(static_cast<uint32_t>(bh >> 32)), p, hi);
                lo = pms_dev::write_lane(static_cast<int>(static_cast<uint32_t>(bl)), l + p, lo);
                hi = pms_dev::write_lane(static_cast<int>(static_cast<uint32_t>(bl >> 32)), l + p, hi);
            }
            if (lane < 2 * l) {
                dst[(2 * g2) * 2 * l + lane] = static_cast<uint32_t>(lo);
                if (2 * g2 + 1 < groups) dst[(2 * g2 + 1) * 2 * l + lane] = static_cast<uint32_t>(hi);
            }
        }
    }
}

// --------------------------------------------------------------------------
// Steps a3 - a6: persistent candidate sweep.
// --------------------------------------------------------------------------
extern "C" __global__ void __launch_bounds__(1024)
pms_search_kernel(const pms_dev_instance* __restrict__ insts,
                  const pms_work_item* __restrict__ work, uint32_t n_work,
                  pms_dev_state* __restrict__ state, pms_dev_counters* __restrict__ ctr,
                  uint32_t q_words) {
    extern __shared__ uint32_t lds[];
    constexpr uint32_t kNone = 0xffffffffu;
    const uint32_t lane = lane_id();
    const uint32_t wave = uni(threadIdx.x >> 6);
    uint32_t* const q = lds + wave * (q_words + PMS_OUTBUF);  // stage queues
    uint32_t* const ob = q + q_words;                         // survivor staging

    uint32_t cur = kNone;     // instance whose candidates the queues hold
    uint32_t pending = 0;     // claimed items of `cur` not yet retired
    uint32_t stash = kNone;   // claimed item of another instance, waiting
    bool more = true;         // the work table may still have items
    uint64_t next = 0, end = 0;
    uint64_t visits = 0, batches = 0;
    uint32_t nob = 0;         // entries in ob
    uint32_t counts = 0;      // lane s: candidates queued for stage s

    cu32* W = nullptr;
    uint32_t* out = nullptr;
    uint64_t cap = 0;
    uint32_t n = 0, nwp = 0, l = 0, d = 0, lmask = 0;

    for (;;) {
        uint32_t s, cand = 0;
        bool active;
        const uint64_t full = ballot(counts >= 64u);
        if (full) {
            // Deepest full queue first: pop its newest 64 entries.
            s = 63u - static_cast<uint32_t>(__builtin_clzll(full));
            const uint32_t c = __builtin_amdgcn_readlane(counts, s);
            cand = q[(s - 1) * PMS_QCAP + c - 64u + lane];
            active = true;
            if (lane == s) counts -= 64u;
        } else if (next < end) {
            // Stage 0: the next 64 candidate numbers of the claimed range.
            s = 0;
            const uint64_t k = next + lane;
            active = k < end;
            const uint32_t kk = static_cast<uint32_t>(k);
            cand = ((kk >> l) << 16) | (kk & lmask);
            next += 64;
        } else {
            if (stash == kNone && more) {
                uint32_t item = 0;
                if (lane == 0) item = atomicAdd(&ctr->next_item, 1u);
                item = uni(item);
                if (item == 0 && lane == 0) ctr->t_start = wall_clock64();
                if (item >= n_work) {
                    more = false;
                } else {
                    const pms_work_item wi = load_uniform(work + item);
                    if (wi.inst == cur) {
                        ++pending;
                        next = wi.begin;
                        end = wi.begin + wi.len;
                    } else {
                        stash = item;
                    }
                }
                continue;
            }
            const uint64_t nz = ballot(counts > 0u);
            if (nz == 0) {
                // Queues empty: every candidate of `cur` this wave claimed is done.
                if (cur != kNone) {
                    if (nob) {
                        uint64_t base = 0;
                        if (lane == 0)
                            base = atomicAdd(reinterpret_cast<unsigned long long*>(&state[cur].count),
                                             static_cast<unsigned long long>(nob));
                        base = uni64(base);
                        for (uint32_t i = lane; i < nob; i += 64u)
                            if (base + i < cap) out[base + i] = ob[i];
                        nob = 0;
                    }
                    if (lane == 0) {
                        atomicAdd(reinterpret_cast<unsigned long long*>(&state[cur].visits),
                                  static_cast<unsigned long long>(visits));
                        const uint32_t old = atomicSub(&state[cur].items_left, pending);
                        if (old == pending) state[cur].t_done = wall_clock64();
                    }
                    visits = 0;
                    pending = 0;
                    cur = kNone;
                }
                if (stash == kNone) break;
                const pms_work_item wi = load_uniform(work + stash);
                const pms_dev_instance in = load_uniform(insts + wi.inst);
                stash = kNone;
                if (in.n < 1 || (static_cast<uint32_t>(in.n) - 1u) * PMS_QCAP > q_words) {
                    // More stages than the launch's LDS queues hold: refuse the item.
                    if (lane == 0) atomicOr(&ctr->error, 1u);
                    continue;
                }
                cur = wi.inst;
                W = (cu32*)(in.windows);
                out = in.out;
                cap = in.out_cap;
                n = static_cast<uint32_t>(in.n);
                nwp = static_cast<uint32_t>(in.nw_stride);
                l = static_cast<uint32_t>(in.l);
                d = static_cast<uint32_t>(in.d);
                lmask = (1u << l) - 1u;
                pending = 1;
                next = wi.begin;
                end = wi.begin + wi.len;
                continue;
            }
            // Drain: the shallowest non-empty queue (fewer than 64 entries).
            s = static_cast<uint32_t>(__builtin_ctzll(nz));
            const uint32_t c = __builtin_amdgcn_readlane(counts, s);
            active = lane < c;
            if (active) cand = q[(s - 1) * PMS_QCAP + lane];
            if (lane == s) counts = 0;
        }

        // One sequence scan for the 64 lanes.
        const uint32_t best = scan_sequence(W + s * nwp, nwp >> 4, cand);
        const bool pass = active && best <= d;
        visits += __builtin_popcountll(ballot(active));
        ++batches;
        const uint64_t pm = ballot(pass);
        if (pm) {
            const uint32_t r = rank_below(pm);
            const uint32_t np = static_cast<uint32_t>(__builtin_popcountll(pm));
            if (s + 1 < n) {
                const uint32_t base = __builtin_amdgcn_readlane(counts, s + 1);
                if (pass) q[s * PMS_QCAP + base + r] = cand;
                if (lane == s + 1) counts += np;
            } else {
                if (pass) ob[nob + r] = plane_to_code(cand);
                nob += np;
                if (nob > PMS_OUTBUF - 64u) {
                    uint64_t base = 0;
                    if (lane == 0)
                        base = atomicAdd(reinterpret_cast<unsigned long long*>(&state[cur].count),
                                         static_cast<unsigned long long>(nob));
                    base = uni64(base);
                    for (uint32_t i = lane; i < nob; i += 64u)
                        if (base + i < cap) out[base + i] = ob[i];
                    nob = 0;
                }
            }
        }
    }
    if (lane == 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(&ctr->batches),
                  static_cast<unsigned long long>(batches));
}

// --------------------------------------------------------------------------
// Small helpers used by the host library.
// --------------------------------------------------------------------------

// Clears `words` 32-bit words (used instead of a memset so that the same
// sequence can be captured into a graph).
extern "C" __global__ void pms_fill_kernel(uint32_t* __restrict__ p, uint64_t words, uint32_t v) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < words;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

// Step a7 for a batch: copies the codes of instance blockIdx.x from its
// reserved output range to its place in one contiguous array, so that one
// copy brings every instance's codes to the host.  tab[3i], tab[3i+1],
// tab[3i+2]: source offset, destination offset, count (in codes).
extern "C" __global__ void __launch_bounds__(256)
pms_gather_kernel(const uint32_t* __restrict__ src, const uint64_t* __restrict__ tab, uint32_t m,
                  uint32_t* __restrict__ dst) {
    const uint32_t i = blockIdx.x;
    if (i >= m) return;
    const uint64_t from = tab[3 * static_cast<uint64_t>(i)];
    const uint64_t to = tab[3 * static_cast<uint64_t>(i) + 1];
    const uint64_t k = tab[3 * static_cast<uint64_t>(i) + 2];
    for (uint64_t j = threadIdx.x; j < k; j += blockDim.x) dst[to + j] = src[from + j];
}

namespace pms {

hipError_t launch_gather(const uint32_t* src, const uint64_t* tab, uint32_t m, uint32_t* dst,
                         hipStream_t stream) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(pms_gather_kernel, dim3(m), dim3(256), 0, stream, src, tab, m, dst);
    return hipGetLastError();
}

hipError_t launch_windows(const pms_win_job* jobs, int32_t rows, int32_t max_t,
                          const uint8_t* seqs, uint32_t* windows, uint32_t* bad,
                          hipStream_t stream) {
    if (rows <= 0) return hipSuccess;
    // packed row + spare word, N map + spare word, first N-free window
    const size_t lds = (static_cast<size_t>((max_t + 15) / 16) + 1 +
                        static_cast<size_t>((max_t + 31) / 32) + 1 + 1) * sizeof(uint32_t);
    hipLaunchKernelGGL(pms_windows_kernel, dim3(rows), dim3(256), lds, stream, jobs, seqs,
                       windows, bad);
    return hipGetLastError();
}

hipError_t launch_search(const pms_dev_instance* insts, const pms_work_item* work,
                         uint32_t n_work, pms_dev_state* state, pms_dev_counters* ctr,
                         uint32_t q_words, uint32_t grid, uint32_t wg_waves, hipStream_t stream) {
    const size_t lds = static_cast<size_t>(wg_waves) * (q_words + PMS_OUTBUF) * sizeof(uint32_t);
    hipLaunchKernelGGL(pms_search_kernel, dim3(grid), dim3(64 * wg_waves), lds, stream, insts,
                       work, n_work, state, ctr, q_words);
    return hipGetLastError();
}

hipError_t launch_fill(uint32_t* p, uint64_t words, uint32_t v, hipStream_t stream) {
    if (words == 0) return hipSuccess;
    const uint64_t blocks64 = (words + 255) / 256;
    const uint32_t blocks = static_cast<uint32_t>(blocks64 < 1024 ? blocks64 : 1024);
    hipLaunchKernelGGL(pms_fill_kernel, dim3(blocks), dim3(256), 0, stream, p, words, v);
    return hipGetLastError();
}

const void* search_kernel_symbol() { return reinterpret_cast<const void*>(&pms_search_kernel); }

}  // namespace pms
