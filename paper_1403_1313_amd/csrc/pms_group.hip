// pms_group.hip -- grouped bit-sliced search kernel (steps a3 - a6).
//
// The same enumeration and the same enhanced rule as pms_search_kernel, with
// the window index bit-sliced instead of the candidate:
//
//  * A lane owns a *group*: the 16 candidates that share their first l-2
//    bases (the prefix).  Candidate c of the group has bases c >> 2 and c & 3
//    at positions l-2 and l-1, so its motif code is (group << 4) | c and
//    groups are numbered in dictionary order.
//  * Windows are processed 32 at a time: for each position p the window table
//    holds two words whose bit j is the high / low bit of the base at
//    position p of window j (pms_windows_kernel, bit-sliced layout).  A
//    mismatch vector is (WH ^ CH) | (WL ^ CL) with CH, CL all-ones or all-zero
//    masks of the lane's prefix base.
//  * The prefix positions' mismatch vectors are added by a carry-save tree
//    into a 4-bit bit-sliced count c (32 windows per register).  Shared by the
//    16 candidates of the group, that count is computed once.  The last two
//    positions contribute s in {0, 1, 2} mismatches, a wave-uniform function of
//    the window and the candidate's two bases, so with u = [s >= 1],
//    v = [s >= 2] (scalar ALU) and T_k = [c <= d - k] a window is within d of
//    candidate c exactly when  T_2 | (T_1 & ~v) | (T_0 & ~u).  Per candidate
//    and per 32 windows that is two v_and_or_b32.
//  * The enhanced rule: after the windows of sequence s, a candidate with no
//    window within d leaves the group's alive mask and is never examined for
//    sequences s+1..; a group whose mask is empty is dropped, and the others
//    go to an LDS queue for stage s+1 (ballot + mbcnt), deepest full queue
//    first, exactly as in the per-lane kernel.
//  * Candidates alive after the last sequence are staged in LDS and flushed
//    with one global atomicAdd per flush.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pms.h"
#include "pms_device.h"
#include "pms_internal.h"

namespace {

using namespace pms_dev;

// Full adder on 32 bit-lanes: a + b + c = s + 2 * carry.
__device__ __forceinline__ void full_add(uint32_t a, uint32_t b, uint32_t c, uint32_t& s,
                                         uint32_t& carry) {
    const uint32_t t = a ^ b;
    s = t ^ c;
    carry = (a & b) | (t & c);
}

// Bit-sliced count of P one-bit vectors: count = c1 + 2 c2 + 4 c4 + 8 c8
// (P <= 15).  Column compression by full and half adders; every loop bound
// and index is a compile-time constant once P is fixed.
template <int P>
__device__ __forceinline__ void count_bits(const uint32_t (&m)[P > 0 ? P : 1], uint32_t& c1,
                                           uint32_t& c2, uint32_t& c4, uint32_t& c8) {
    uint32_t w[4][16];
    int nw[4] = {P, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < P; ++i) w[0][i] = m[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            if (nw[k] >= 3) {
                uint32_t s, cy;
                full_add(w[k][nw[k] - 3], w[k][nw[k] - 2], w[k][nw[k] - 1], s, cy);
                nw[k] -= 2;
                w[k][nw[k] - 1] = s;
                if (k < 3) w[k + 1][nw[k + 1]++] = cy;
            } else if (nw[k] == 2 && k < 3) {
                const uint32_t a = w[k][0], b = w[k][1];
                w[k][0] = a ^ b;
                nw[k] = 1;
                w[k + 1][nw[k + 1]++] = a & b;
            } else if (nw[k] == 2) {
                // weight 8: two ones here would mean a count >= 16 > P
                w[k][0] |= w[k][1];
                nw[k] = 1;
            }
        }
    }
    c1 = nw[0] ? w[0][0] : 0u;
    c2 = nw[1] ? w[1][0] : 0u;
    c4 = nw[2] ? w[2][0] : 0u;
    c8 = nw[3] ? w[3][0] : 0u;
}

// Bit-sliced [count <= k] for a wave-uniform k.
__device__ __forceinline__ uint32_t count_le(uint32_t c1, uint32_t c2, uint32_t c4, uint32_t c8,
                                             int k) {
    if (k < 0) return 0u;
    if (k >= 15) return ~0u;
    uint32_t gt = 0u, eq = ~0u;
    if (k & 8) { eq &= c8; } else { gt |= eq & c8; eq &= ~c8; }
    if (k & 4) { eq &= c4; } else { gt |= eq & c4; eq &= ~c4; }
    if (k & 2) { eq &= c2; } else { gt |= eq & c2; eq &= ~c2; }
    if (k & 1) { /* eq &= c1; not needed */ } else { gt |= eq & c1; }
    return ~gt;
}

// One sequence scan for the lane's group: returns the 16-bit mask of
// candidates with a window within d, restricted to `alive`.
// W: the sequence's bit-sliced row (groups x 2L words), wave-uniform.
template <int P>
__device__ __forceinline__ uint32_t scan_group(cu32* W, uint32_t groups, uint32_t prefix,
                                               int d, uint32_t alive) {
    constexpr int L = P + 2;
    uint32_t ch[P > 0 ? P : 1], cl[P > 0 ? P : 1];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t b = (prefix >> (2 * (P - 1 - p))) & 3u;
        ch[p] = 0u - (b >> 1);
        cl[p] = 0u - (b & 1u);
    }
    uint32_t found[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) found[c] = 0u;
    uint32_t found_all = 0u;
    for (uint32_t gi = 0; gi < groups; ++gi, W += 2 * L) {
        uint32_t m[P > 0 ? P : 1];
#pragma unroll
        for (int p = 0; p < P; ++p) m[p] = (W[p] ^ ch[p]) | (W[L + p] ^ cl[p]);
        uint32_t c1 = 0, c2 = 0, c4 = 0, c8 = 0;
        if (P > 0) count_bits<P>(m, c1, c2, c4, c8);
        const uint32_t t0 = count_le(c1, c2, c4, c8, d);
        const uint32_t t1 = count_le(c1, c2, c4, c8, d - 1);
        const uint32_t t2 = count_le(c1, c2, c4, c8, d - 2);
        found_all |= t2;
        // Mismatch of each base at the last two positions (wave-uniform):
        // base 0 (A=00) mismatches where hi|lo, C=01 where hi|~lo, G=10 where
        // ~hi|lo, T=11 where ~(hi&lo).
        const uint32_t ha = W[P], la = W[L + P], hb = W[P + 1], lb = W[L + P + 1];
        const uint32_t sa[4] = {ha | la, ha | ~la, ~ha | la, ~(ha & la)};
        const uint32_t sb[4] = {hb | lb, hb | ~lb, ~hb | lb, ~(hb & lb)};
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const uint32_t nu = ~(sa[c >> 2] | sb[c & 3]);  // no suffix mismatch
            const uint32_t nv = ~(sa[c >> 2] & sb[c & 3]);  // at most one
            found[c] |= t1 & nv;
            found[c] |= t0 & nu;
        }
    }
    uint32_t pass = 0u;
#pragma unroll
    for (int c = 0; c < 16; ++c) pass |= ((found[c] | found_all) != 0u ? 1u : 0u) << c;
    return pass & alive;
}

// Dispatch on the number of prefix positions (wave-uniform).
__device__ __forceinline__ uint32_t scan_group_any(uint32_t P, cu32* W, uint32_t groups,
                                                   uint32_t prefix, int d, uint32_t alive) {
    switch (P) {
        case 0: return scan_group<0>(W, groups, prefix, d, alive);
        case 1: return scan_group<1>(W, groups, prefix, d, alive);
        case 2: return scan_group<2>(W, groups, prefix, d, alive);
        case 3: return scan_group<3>(W, groups, prefix, d, alive);
        case 4: return scan_group<4>(W, groups, prefix, d, alive);
        case 5: return scan_group<5>(W, groups, prefix, d, alive);
        case 6: return scan_group<6>(W, groups, prefix, d, alive);
        case 7: return scan_group<7>(W, groups, prefix, d, alive);
        case 8: return scan_group<8>(W, groups, prefix, d, alive);
        case 9: return scan_group<9>(W, groups, prefix, d, alive);
        case 10: return scan_group<10>(W, groups, prefix, d, alive);
        case 11: return scan_group<11>(W, groups, prefix, d, alive);
        case 12: return scan_group<12>(W, groups, prefix, d, alive);
        case 13: return scan_group<13>(W, groups, prefix, d, alive);
        default: return scan_group<14>(W, groups, prefix, d, alive);
    }
}

}  // namespace

extern "C" __global__ void __launch_bounds__(1024)
pms_search_group_kernel(const pms_dev_instance* __restrict__ insts,
                        const pms_work_item* __restrict__ work, uint32_t n_work,
                        pms_dev_state* __restrict__ state, pms_dev_counters* __restrict__ ctr,
                        uint32_t q_words) {
    extern __shared__ uint32_t lds[];
    constexpr uint32_t kNone = 0xffffffffu;
    const uint32_t lane = lane_id();
    const uint32_t wave = uni(threadIdx.x >> 6);
    // Per wavefront: queue prefixes [stages][QCAP] u32, queue masks
    // [stages][QCAP] u16, survivor staging [OUTBUF] u32.
    uint32_t* const qp = lds + wave * (q_words + PMS_OUTBUF);
    const uint32_t stages_cap = q_words / (PMS_QCAP + PMS_QCAP / 2);
    uint16_t* const qm = reinterpret_cast<uint16_t*>(qp + stages_cap * PMS_QCAP);
    uint32_t* const ob = qp + q_words;

    uint32_t cur = kNone, pending = 0, stash = kNone;
    bool more = true;
    uint64_t next = 0, end = 0;     // group numbers
    uint64_t batches = 0;
    uint64_t visits = 0;            // per lane
    uint32_t nob = 0;
    uint32_t counts = 0;            // lane s: groups queued for stage s

    cu32* W = nullptr;
    uint32_t* out = nullptr;
    uint64_t cap = 0;
    uint32_t n = 0, row = 0, groups = 0, P = 0;
    int d = 0;

    for (;;) {
        uint32_t s, prefix = 0, alive = 0;
        const uint64_t full = ballot(counts >= 64u);
        if (full) {
            s = 63u - static_cast<uint32_t>(__builtin_clzll(full));
            const uint32_t c = __builtin_amdgcn_readlane(counts, s);
            const uint32_t at = (s - 1) * PMS_QCAP + c - 64u + lane;
            prefix = qp[at];
            alive = qm[at];
            if (lane == s) counts -= 64u;
        } else if (next < end) {
            s = 0;
            const uint64_t g = next + lane;
            prefix = static_cast<uint32_t>(g);
            alive = g < end ? 0xffffu : 0u;
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
                        next = wi.begin >> 4;
                        end = (wi.begin + wi.len) >> 4;
                    } else {
                        stash = item;
                    }
                }
                continue;
            }
            const uint64_t nz = ballot(counts > 0u);
            if (nz == 0) {
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
                    // Sum the lanes' visit counts, then one atomic per wavefront.
                    unsigned long long v = visits;
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                    if (lane == 0 && v)
                        atomicAdd(reinterpret_cast<unsigned long long*>(&state[cur].visits), v);
                    visits = 0;
                    if (lane == 0) {
                        const uint32_t old = atomicSub(&state[cur].items_left, pending);
                        if (old == pending) state[cur].t_done = wall_clock64();
                    }
                    pending = 0;
                    cur = kNone;
                }
                if (stash == kNone) break;
                const pms_work_item wi = load_uniform(work + stash);
                const pms_dev_instance in = load_uniform(insts + wi.inst);
                stash = kNone;
                if (in.n < 1 || in.l < 2 || (static_cast<uint32_t>(in.n) - 1u) > stages_cap) {
                    if (lane == 0) atomicOr(&ctr->error, 1u);
                    continue;
                }
                cur = wi.inst;
                W = (cu32*)(in.windows);
                out = in.out;
                cap = in.out_cap;
                n = static_cast<uint32_t>(in.n);
                row = static_cast<uint32_t>(in.nw_stride);
                P = static_cast<uint32_t>(in.l) - 2u;
                groups = row / (2u * (P + 2u));
                d = in.d;
                pending = 1;
                next = wi.begin >> 4;
                end = (wi.begin + wi.len) >> 4;
                continue;
            }
            s = static_cast<uint32_t>(__builtin_ctzll(nz));
            const uint32_t c = __builtin_amdgcn_readlane(counts, s);
            if (lane < c) {
                prefix = qp[(s - 1) * PMS_QCAP + lane];
                alive = qm[(s - 1) * PMS_QCAP + lane];
            }
            if (lane == s) counts = 0;
        }

        // One sequence scan for 64 groups (up to 1024 candidates).
        const uint32_t pass = scan_group_any(P, W + s * row, groups, prefix, d, alive);
        visits += static_cast<uint32_t>(__builtin_popcount(alive));
        ++batches;
        const bool keep = pass != 0u;
        const uint64_t pm = ballot(keep);
        if (pm) {
            if (s + 1 < n) {
                const uint32_t base = __builtin_amdgcn_readlane(counts, s + 1);
                const uint32_t r = rank_below(pm);
                if (keep) {
                    qp[s * PMS_QCAP + base + r] = prefix;
                    qm[s * PMS_QCAP + base + r] = static_cast<uint16_t>(pass);
                }
                if (lane == s + 1) counts += static_cast<uint32_t>(__builtin_popcountll(pm));
            } else {
                // Survivors: one code per alive candidate, compacted by ballot.
                for (uint32_t c = 0; c < 16u; ++c) {
                    const bool hit = (pass >> c) & 1u;
                    const uint64_t hm = ballot(hit);
                    if (!hm) continue;
                    if (hit) ob[nob + rank_below(hm)] = (prefix << 4) | c;
                    nob += static_cast<uint32_t>(__builtin_popcountll(hm));
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
    }
    if (lane == 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(&ctr->batches),
                  static_cast<unsigned long long>(batches));
}

namespace pms {

hipError_t launch_search_group(const pms_dev_instance* insts, const pms_work_item* work,
                               uint32_t n_work, pms_dev_state* state, pms_dev_counters* ctr,
                               uint32_t q_words, uint32_t grid, uint32_t wg_waves,
                               hipStream_t stream) {
    const size_t lds = static_cast<size_t>(wg_waves) * (q_words + PMS_OUTBUF) * sizeof(uint32_t);
    hipLaunchKernelGGL(pms_search_group_kernel, dim3(grid), dim3(64 * wg_waves), lds, stream, insts,
                       work, n_work, state, ctr, q_words);
    return hipGetLastError();
}

const void* search_group_kernel_symbol() {
    return reinterpret_cast<const void*>(&pms_search_group_kernel);
}

}  // namespace pms
