// pms_group.hip -- grouped bit-sliced search kernel (steps a3 - a6).
//
// The same enumeration and the same enhanced rule as pms_search_kernel, with
// the window index bit-sliced instead of the candidate:
//
//  * A lane owns a *group*: the 4^S candidates that share their first
//    P = l - S bases (the prefix); S = 2 (16 per group) or S = 3 (64).
//    Candidate c of the group has the base-4 digits of c at the last S
//    positions, so its motif code is (group << 2S) | c and groups are
//    numbered in dictionary order.
//  * Windows are processed 32 at a time: for each position p the window table
//    holds two words whose bit j is the high / low bit of the base at
//    position p of window j (pms_windows_kernel, bit-sliced layout).  A
//    mismatch vector is (WH ^ CH) | (WL ^ CL) with CH, CL all-ones or all-zero
//    masks of the lane's prefix base.
//  * The prefix positions' mismatch vectors are added by a carry-save tree
//    into a 4-bit bit-sliced count c (32 windows per register), computed once
//    for the whole group, and compared with the thresholds T_k = [c <= d - k].
//    The suffix positions' mismatch vectors depend only on the window, so
//    they are wave-uniform (scalar unit); a selection tree over them decides
//    [c + suffix mismatches <= d] for all 4^S candidates with plain
//    and/or/not forms (scan_group).
//  * The enhanced rule: after the windows of sequence s, a candidate with no
//    window within d leaves the group's alive mask and is never examined for
//    sequences s+1..; a group whose mask is empty is dropped, and the others
//    go to a queue for stage s+1 (ballot + mbcnt), deepest full queue first,
//    exactly as in the per-lane kernel.
//  * Candidates alive after the last sequence are staged in LDS and flushed
//    with one global atomicAdd per flush.
//  * S = 3 only: groups with at most two live members go on as single
//    candidates (scan_single, 64 singles per wavefront); group and single
//    batches whose candidates fall into a few blocks of 4096 scan only the
//    windows within d of the blocks' shared first l - 6 bases (the window
//    filter: filter_windows, then scan_filtered or scan_filtered_single).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pms.h"
#include "pms_device.h"
#include "pms_internal.h"

namespace {

using namespace pms_dev;

// Three-input bit functions as single v_bitop3_b32 instructions.  The
// compiler would otherwise pick v_bfi / v_or3 / v_and_or forms for some of
// them, which issue at half the rate of v_bitop3 on gfx950.  Truth-table
// index: (a << 2) | (b << 1) | c.
template <uint32_t TT>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}
constexpr uint32_t kXor3 = 0x96;     // a ^ b ^ c
constexpr uint32_t kMaj = 0xE8;      // at least two of a, b, c
constexpr uint32_t kMux = 0xCA;      // a ? b : c
constexpr uint32_t kOrAndN = 0xF4;   // a | (b & ~c)
constexpr uint32_t kOr3 = 0xFE;      // a | b | c
constexpr uint32_t kAnd3 = 0x80;     // a & b & c
constexpr uint32_t kNandOr = 0x1F;   // ~(a & (b | c))
constexpr uint32_t kNorAnd = 0x07;   // ~(a | (b & c))
constexpr uint32_t kOrXor = 0xF6;    // a | (b ^ c)
constexpr uint32_t kAndN = 0x30;     // a & ~b

// Bit-sliced sum of P one-bit vectors plus a wave-uniform bias B < 32 given
// as five all-ones / all-zero masks bias[i] = bit i of B:
//   sum = c[0] + 2 c[1] + 4 c[2] + 8 c[3] + 16 c[4]   (P + B < 32).
// Column compression by full adders (xor3 + majority) and half adders; every
// loop bound and index is a compile-time constant once P is fixed.
template <int P>
__device__ __forceinline__ void count_bits(const uint32_t (&m)[P > 0 ? P : 1],
                                           const uint32_t (&bias)[5], uint32_t (&c)[5]) {
    uint32_t w[5][18];
    int nw[5] = {P + 1, 1, 1, 1, 1};
#pragma unroll
    for (int i = 0; i < P; ++i) w[0][i] = m[i];
    w[0][P] = bias[0];
#pragma unroll
    for (int k = 1; k < 5; ++k) w[k][0] = bias[k];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
#pragma unroll
        for (int it = 0; it < 18; ++it) {
            if (nw[k] >= 3) {
                const uint32_t x = w[k][nw[k] - 3], y = w[k][nw[k] - 2], z = w[k][nw[k] - 1];
                nw[k] -= 2;
                w[k][nw[k] - 1] = bop3<kXor3>(x, y, z);
                if (k < 4) w[k + 1][nw[k + 1]++] = bop3<kMaj>(x, y, z);
            } else if (nw[k] == 2 && k < 4) {
                const uint32_t x = w[k][0], y = w[k][1];
                w[k][0] = x ^ y;
                nw[k] = 1;
                w[k + 1][nw[k + 1]++] = x & y;
            } else if (nw[k] == 2) {
                // weight 16: both set would mean a sum >= 32
                w[k][0] |= w[k][1];
                nw[k] = 1;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) c[k] = nw[k] ? w[k][0] : 0u;
}


// A wave-uniform value copied into a VGPR.  VALU instructions that read an
// SGPR issue at half rate on gfx950; the selection tree below reads these
// copies instead, so it runs at full rate.
__device__ __forceinline__ uint32_t to_vgpr(uint32_t x) {
    uint32_t r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

// Alive / pass masks: 16 candidates per group (S = 2) or 64 (S = 3).
template <int S> struct MaskOf { typedef uint32_t type; };
template <> struct MaskOf<3> { typedef uint64_t type; };

// Suffix mismatch vectors of one 32-window group for suffix position q:
// base 0 = A = 00 mismatches where hi|lo, C = 01 where hi|~lo, G = 10 where
// ~hi|lo, T = 11 where ~(hi&lo).  Computed on the scalar unit, copied to VGPRs.
__device__ __forceinline__ void suffix_vectors(uint32_t h, uint32_t lo, uint32_t (&sv)[4]) {
    sv[0] = to_vgpr(h | lo);
    sv[1] = to_vgpr(h | ~lo);
    sv[2] = to_vgpr(~h | lo);
    sv[3] = to_vgpr(~(h & lo));
}

// Selection tree over the S suffix positions for one 32-window group, given
// the thresholds t[k] = [mismatches before the suffix <= d - k], k = 0..S:
//   U_1[b1][k]    = s_1[b1] ? t[k+1] : t[k]                 k = 0..S-1
//   U_j[..bj][k]  = s_j[bj] ? U_{j-1}[..][k+1] : U_{j-1}[..][k]
// U_j[..][k] = [mismatches + s_1 + .. + s_j <= d - k].  The last level is
// folded into the accumulators: a candidate has a good window where
//   U_{S-1}[..][1]  |  (~s_S[bS] & U_{S-1}[..][0]).
template <int S, bool First = false>
__device__ __forceinline__ void select_accumulate(const uint32_t (&t)[4], const uint32_t (&sv)[S][4],
                                                  uint32_t (&found)[1 << (2 * S)],
                                                  uint32_t (&top)[1 << (2 * S - 2)]) {
    constexpr int N1 = 1 << (2 * S - 2);
    uint32_t u[N1][2];
    if constexpr (S == 2) {
#pragma unroll
        for (int b1 = 0; b1 < 4; ++b1) {
            const uint32_t sm = sv[0][b1];
            u[b1][0] = bop3<kMux>(sm, t[1], t[0]);
            u[b1][1] = bop3<kMux>(sm, t[2], t[1]);
        }
    } else {
#pragma unroll
        for (int b1 = 0; b1 < 4; ++b1) {
            const uint32_t sm = sv[0][b1];
            uint32_t v1[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) v1[k] = bop3<kMux>(sm, t[k + 1], t[k]);
#pragma unroll
            for (int b2 = 0; b2 < 4; ++b2) {
                const uint32_t sn = sv[S - 2][b2];
                u[b1 * 4 + b2][0] = bop3<kMux>(sn, v1[1], v1[0]);
                u[b1 * 4 + b2][1] = bop3<kMux>(sn, v1[2], v1[1]);
            }
        }
    }
#pragma unroll
    for (int n = 0; n < N1; ++n) {
        if constexpr (First) {
            // The first window group sets the accumulators (no zeroing).
            top[n] = u[n][1];
#pragma unroll
            for (int b = 0; b < 4; ++b) found[n * 4 + b] = bop3<kAndN>(u[n][0], sv[S - 1][b], 0u);
        } else {
            top[n] |= u[n][1];
#pragma unroll
            for (int b = 0; b < 4; ++b)
                found[n * 4 + b] = bop3<kOrAndN>(found[n * 4 + b], u[n][0], sv[S - 1][b]);
        }
    }
}

// Pass mask of a group: candidate c has a window within d.
//  * 16 candidates: a plain OR of shifted flags.
//  * 64 candidates: 32 bits at a time as acc = 2 acc + [x_c != 0] from the
//    highest candidate down, each step one v_cmp (into VCC) and one
//    v_addc_co_u32 that adds acc to itself with VCC as the carry in.  This
//    keeps the epilogue to two instructions per candidate and, unlike the
//    select-and-merge code the compiler forms for the flags, holds few
//    registers at once, which lets the kernel fit three wavefronts per SIMD.
template <int S>
__device__ __forceinline__ typename MaskOf<S>::type group_pass(const uint32_t (&found)[1 << (2 * S)],
                                                               const uint32_t (&top)[1 << (2 * S - 2)]) {
    typedef typename MaskOf<S>::type Mask;
    constexpr int K = 1 << (2 * S);
    Mask pass = 0;
    if constexpr (S == 2) {
#pragma unroll
        for (int c = 0; c < K; ++c)
            pass |= static_cast<Mask>((found[c] | top[c >> 2]) != 0u ? 1u : 0u) << c;
    } else {
#pragma unroll
        for (int h = K / 32 - 1; h >= 0; --h) {
            uint32_t acc = 0;
#pragma unroll
            for (int c = h * 32 + 31; c >= h * 32; --c) {
                const uint32_t x = found[c] | top[c >> 2];
                asm("v_cmp_ne_u32_e32 vcc, 0, %1\n\tv_addc_co_u32_e32 %0, vcc, %0, %0, vcc"
                    : "+v"(acc)
                    : "v"(x)
                    : "vcc");
            }
            pass = (pass << 32) | acc;
        }
    }
    return pass;
}

// One sequence scan for the lane's group of 4^S candidates that share the
// P = l - S prefix bases `prefix`: returns the mask of candidates with a
// window within d, restricted to `alive`.  W: the sequence's bit-sliced row
// (groups x 2l words), wave-uniform.
//
// Per 32 windows: the prefix mismatch count plus the bias 16 - d,
// c' = c + 16 - d (< 32), so that the thresholds T_k = [c <= d - k] are
// comparisons of c' with the constants 16 - k:
//   T_0 = ~(c'16 & (c'8 | c'4 | c'2 | c'1)),  T_1 = ~c'16,
//   T_2 = ~(c'16 | c'8 c'4 c'2 c'1),           T_3 = ~(c'16 | c'8 c'4 c'2),
// then a selection tree over the suffix positions: with s_q[b] = mismatch of
// base b at suffix position q,
//   U_1[b1][k]    = s_1[b1] ? T[k+1] : T[k]                 k = 0..S-1
//   U_j[..bj][k]  = s_j[bj] ? U_{j-1}[..][k+1] : U_{j-1}[..][k]
// U_j[..][k] = [c + s_1 + .. + s_j <= d - k].  The last level is folded into
// the accumulators: a candidate has a good window where
//   U_{S-1}[..][1]  |  (~s_S[bS] & U_{S-1}[..][0]).
template <int P, int S>
__device__ __forceinline__ typename MaskOf<S>::type scan_group(
        cu32* W, uint32_t groups, uint32_t prefix, int d, typename MaskOf<S>::type alive) {
    typedef typename MaskOf<S>::type Mask;
    constexpr int L = P + S;
    constexpr int K = 1 << (2 * S);    // candidates per group
    constexpr int N1 = K / 4;          // nodes of the next-to-last level
    uint32_t ch[P > 0 ? P : 1], cl[P > 0 ? P : 1];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t b = (prefix >> (2 * (P - 1 - p))) & 3u;
        ch[p] = 0u - (b >> 1);
        cl[p] = 0u - (b & 1u);
    }
    const uint32_t bias_value = static_cast<uint32_t>(16 - d);
    uint32_t bias[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) bias[i] = to_vgpr(0u - ((bias_value >> i) & 1u));
    uint32_t found[K], top[N1];
#pragma unroll
    for (int c = 0; c < K; ++c) found[c] = 0u;
#pragma unroll
    for (int c = 0; c < N1; ++c) top[c] = 0u;
    // The words of one group of 32 windows live in SGPRs.  The next group's
    // words are requested as soon as the current ones have been consumed
    // (prefix count and suffix vectors), so the scalar loads are in flight
    // while the selection tree runs.
    // (The first group is read through a volatile pointer so that the
    // compiler does not merge these loads with the loop's and move them to
    // the loop head.)
    uint32_t w[2 * L];
#pragma unroll
    for (int i = 0; i < 2 * L; ++i) w[i] = ((__attribute__((address_space(4))) const volatile uint32_t*)W)[i];
    for (uint32_t gi = 0; gi < groups; ++gi) {
        uint32_t m[P > 0 ? P : 1];
#pragma unroll
        for (int p = 0; p < P; ++p) m[p] = (w[p] ^ ch[p]) | (w[L + p] ^ cl[p]);
        uint32_t c[5];
        count_bits<P>(m, bias, c);
        uint32_t t[4];
        t[0] = bop3<kNandOr>(c[4], bop3<kOr3>(c[3], c[2], c[1]), c[0]);
        t[1] = ~c[4];
        const uint32_t a = bop3<kAnd3>(c[3], c[2], c[1]);
        t[2] = bop3<kNorAnd>(c[4], a, c[0]);
        t[3] = ~(c[4] | a);
        uint32_t sv[S][4];
#pragma unroll
        for (int q = 0; q < S; ++q) suffix_vectors(w[P + q], w[L + P + q], sv[q]);
        // The thresholds are complete here: pin them before the next loads.
#pragma unroll
        for (int k = 0; k <= S; ++k) asm volatile("" : "+v"(t[k]));
        // Last group: the same words again (read, never used).  The empty asm
        // keeps the loads below this point.
        W += gi + 1 < groups ? 2 * L : 0;
        asm volatile("" : "+s"(W));
#pragma unroll
        for (int i = 0; i < 2 * L; ++i) w[i] = W[i];
        select_accumulate<S>(t, sv, found, top);
    }
    return group_pass<S>(found, top) & alive;
}

// Dispatch on the number of prefix positions (wave-uniform).
template <int S>
__device__ __forceinline__ typename MaskOf<S>::type scan_group_any(
        uint32_t P, cu32* W, uint32_t groups, uint32_t prefix, int d,
        typename MaskOf<S>::type alive) {
    switch (P) {
        case 0: return scan_group<0, S>(W, groups, prefix, d, alive);
        case 1: return scan_group<1, S>(W, groups, prefix, d, alive);
        case 2: return scan_group<2, S>(W, groups, prefix, d, alive);
        case 3: return scan_group<3, S>(W, groups, prefix, d, alive);
        case 4: return scan_group<4, S>(W, groups, prefix, d, alive);
        case 5: return scan_group<5, S>(W, groups, prefix, d, alive);
        case 6: return scan_group<6, S>(W, groups, prefix, d, alive);
        case 7: return scan_group<7, S>(W, groups, prefix, d, alive);
        case 8: return scan_group<8, S>(W, groups, prefix, d, alive);
        case 9: return scan_group<9, S>(W, groups, prefix, d, alive);
        case 10: return scan_group<10, S>(W, groups, prefix, d, alive);
        case 11: return scan_group<11, S>(W, groups, prefix, d, alive);
        case 12: return scan_group<12, S>(W, groups, prefix, d, alive);
        case 13: return scan_group<13, S>(W, groups, prefix, d, alive);
        default: return scan_group<(S == 2 ? 14 : 13), S>(W, groups, prefix, d, alive);
    }
}

// Scan of 64 groups whose prefixes fall into at most 64 / groups blocks of
// 64 consecutive groups: the groups of one block share their first Q = P - 3
// bases (the block number, prefix >> 6) and differ only in the last three
// (prefix & 63).  A stage-0 batch aligned to 64 groups is one block; a
// stage-1 batch, the top of a queue fed by consecutive stage-0 batches,
// usually two or three.
//  * Once per call, table lane b*groups + j (block b, window group j) counts
//    the block's shared-position mismatches for window group j (carry-save,
//    bias 19 - d, c' = c + 19 - d < 32) and keeps the thresholds
//    U_k = [c <= d - k], k = 0..6, as comparisons of c' with the constants
//    19 - k.  Lanes j < groups also write window group j's suffix mismatch
//    vectors into the wavefront's LDS table `svt`.
//  * Per 32 windows every lane fetches U_0..U_6 of the current window group
//    from its block's table lane (ds_bpermute) and walks them through its
//    own three prefix positions with the selection recursion of the suffix:
//      V_1[k] = m_1 ? U[k+1] : U[k]    (k = 0..5)
//      V_2[k] = m_2 ? V_1[k+1] : V_1[k] (k = 0..4)
//      T[k]   = m_3 ? V_2[k+1] : V_2[k] (k = 0..3)
//    so T[k] = [mismatches over the whole prefix <= d - k], as in scan_group.
// The prefix count over Q positions is thus done once per call and block
// instead of once per window group per lane, no word of the shared positions
// is read per iteration, and the suffix vectors come from LDS (three
// broadcast reads straight into VGPRs) instead of being moved from SGPRs.
// Arguments, per lane: kv, tj = the block and window group this lane builds
// thresholds for (tj >= groups: none); src = first table lane of the lane's
// own block; low = prefix & 63.  Requires 3 <= P <= 13 and 12 * groups <=
// PMS_SVT_WORDS.
template <int P>
__device__ __forceinline__ uint64_t scan_group_shared(cu32* W, uint32_t groups, uint32_t kv,
                                                      uint32_t tj, uint32_t src, uint32_t low,
                                                      int d, uint64_t alive,
                                                      uint32_t* __restrict__ svt) {
    constexpr int S = 3;
    constexpr int L = P + S;
    constexpr int Q = P - 3;           // shared prefix positions
    constexpr int K = 64;
    constexpr int N1 = K / 4;
    // The lane index is rebuilt per call: hoisted out of the persistent
    // loop, values derived from it would hold registers through every other
    // path as well.
    uint32_t ln = lane_id();
    asm volatile("" : "+v"(ln));
    uint32_t u[7];
    {
        const uint32_t bias_value = static_cast<uint32_t>(19 - d);
        uint32_t bias[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) bias[i] = 0u - ((bias_value >> i) & 1u);
        uint32_t m[Q > 0 ? Q : 1];
#pragma unroll
        for (int p = 0; p < (Q > 0 ? Q : 1); ++p) m[p] = 0u;
        if (tj < groups) {
            const uint32_t* row = (const uint32_t*)(W) + tj * (2u * L);
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const uint32_t b = (kv >> (2 * (Q - 1 - p))) & 3u;
                m[p] = (row[p] ^ (0u - (b >> 1))) | (row[L + p] ^ (0u - (b & 1u)));
            }
        }
        if (ln < groups) {
            // This window group's suffix mismatch vectors (A, C, G, T at
            // each suffix position) into the wavefront's table.
            const uint32_t* row = (const uint32_t*)(W) + ln * (2u * L);
            uint4* dst = reinterpret_cast<uint4*>(svt + ln * 12u);
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const uint32_t h = row[P + q], lo = row[L + P + q];
                dst[q] = make_uint4(h | lo, h | ~lo, ~h | lo, ~(h & lo));
            }
        }
        uint32_t c[5];
        count_bits<Q>(m, bias, c);
        u[0] = ~(c[4] & (c[3] | c[2]));
        u[1] = ~(c[4] & (c[3] | c[2] | (c[1] & c[0])));
        u[2] = ~(c[4] & (c[3] | c[2] | c[1]));
        u[3] = ~(c[4] & (c[3] | c[2] | c[1] | c[0]));
        u[4] = ~c[4];
        u[5] = ~(c[4] | (c[3] & c[2] & c[1] & c[0]));
        u[6] = ~(c[4] | (c[3] & c[2] & c[1]));
    }
    // The lane's own last three prefix bases.
    uint32_t ch[3], cl[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const uint32_t b = (low >> (2 * (2 - q))) & 3u;
        ch[q] = 0u - (b >> 1);
        cl[q] = 0u - (b & 1u);
    }
    uint32_t found[K], top[N1];
#pragma unroll
    for (int c = 0; c < K; ++c) found[c] = 0u;
#pragma unroll
    for (int c = 0; c < N1; ++c) top[c] = 0u;
    // Per window group the loop reads the lane positions' words (3 high, 3
    // low plane, in SGPRs, the next group's loaded while the selection tree
    // runs, as in scan_group) and the suffix vectors from the table (three
    // broadcast LDS reads straight into VGPRs: no v_mov from SGPRs).
    uint32_t w[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        w[i] = ((__attribute__((address_space(4))) const volatile uint32_t*)W)[Q + i];
        w[3 + i] = ((__attribute__((address_space(4))) const volatile uint32_t*)W)[L + Q + i];
    }
    const uint4* sp = reinterpret_cast<const uint4*>(svt);
    for (uint32_t gi = 0; gi < groups; ++gi) {
        // LDS traffic first (thresholds, suffix vectors): LDS and scalar
        // loads share one counter, so these must be complete before the
        // next group's scalar loads are issued below, or the wait for them
        // would also wait for those loads.
        uint32_t uu[7];
#pragma unroll
        for (int k = 0; k < 7; ++k)
            uu[k] = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(
                static_cast<int>((src + gi) << 2), static_cast<int>(u[k])));
        uint32_t sv[S][4];
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const uint4 v = sp[gi * 3u + q];
            sv[q][0] = v.x;
            sv[q][1] = v.y;
            sv[q][2] = v.z;
            sv[q][3] = v.w;
        }
        uint32_t m[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) m[q] = (w[q] ^ ch[q]) | (w[3 + q] ^ cl[q]);
        uint32_t v1[6], v2[5], t[4];
#pragma unroll
        for (int k = 0; k < 6; ++k) v1[k] = bop3<kMux>(m[0], uu[k + 1], uu[k]);
#pragma unroll
        for (int k = 0; k < 5; ++k) v2[k] = bop3<kMux>(m[1], v1[k + 1], v1[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k) t[k] = bop3<kMux>(m[2], v2[k + 1], v2[k]);
#pragma unroll
        for (int k = 0; k <= S; ++k) asm volatile("" : "+v"(t[k]));
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
            for (int b = 0; b < 4; ++b) asm volatile("" : "+v"(sv[q][b]));
        W += gi + 1 < groups ? 2 * L : 0;
        asm volatile("" : "+s"(W));
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            w[i] = W[Q + i];
            w[3 + i] = W[L + Q + i];
        }
        select_accumulate<S>(t, sv, found, top);
    }
    return group_pass<S>(found, top) & alive;
}

// Dispatch on P (wave-uniform, 3..13).
__device__ __forceinline__ uint64_t scan_group_shared_any(uint32_t P, cu32* W, uint32_t groups,
                                                          uint32_t kv, uint32_t tj, uint32_t src,
                                                          uint32_t low, int d, uint64_t alive,
                                                          uint32_t* svt) {
    switch (P) {
        case 3: return scan_group_shared<3>(W, groups, kv, tj, src, low, d, alive, svt);
        case 4: return scan_group_shared<4>(W, groups, kv, tj, src, low, d, alive, svt);
        case 5: return scan_group_shared<5>(W, groups, kv, tj, src, low, d, alive, svt);
        case 6: return scan_group_shared<6>(W, groups, kv, tj, src, low, d, alive, svt);
        case 7: return scan_group_shared<7>(W, groups, kv, tj, src, low, d, alive, svt);
        case 8: return scan_group_shared<8>(W, groups, kv, tj, src, low, d, alive, svt);
        case 9: return scan_group_shared<9>(W, groups, kv, tj, src, low, d, alive, svt);
        case 10: return scan_group_shared<10>(W, groups, kv, tj, src, low, d, alive, svt);
        case 11: return scan_group_shared<11>(W, groups, kv, tj, src, low, d, alive, svt);
        case 12: return scan_group_shared<12>(W, groups, kv, tj, src, low, d, alive, svt);
        default: return scan_group_shared<13>(W, groups, kv, tj, src, low, d, alive, svt);
    }
}

// Window filter for a batch of 64 groups whose live lanes fall into nb
// blocks of 64 consecutive groups (each block shares its first Q = P - 3
// bases).  A window whose mismatch count over a block's shared bases exceeds
// d is farther than d from every candidate of that block; a window farther
// for every block of the batch cannot change any candidate's result, so only
// the windows with U_0 = [shared count <= d] set for some block are scanned
// (an exact filter on top of the enhanced rule, which it leaves unchanged:
// the same candidates reach the same sequences).
//
// filter_windows builds the blocks' thresholds in the table lanes of
// scan_group_shared (lane b * groups + j: block b, window group j; U_0..U_6)
// with the window group's plane words of the six unshared positions (3 lane,
// 3 suffix; high plane, then low), and re-slices the windows that pass into
// dense 32-window groups in the wavefront's LDS table `svt`, 12 + 8 nb words
// each: the 12 plane words, then U_0..U_6 (and one spare word) per block.
//  * The union mask of each window group is collected in lane j (one
//    ds_bpermute per block); the lanes' offsets in the list of passing
//    windows come from an inclusive sum of their counts over the lanes,
//    and each lane writes the numbers of its passing windows into a
//    64-position LDS list, 64 list positions at a time.
//  * 64 listed windows (or the rest, at the end) are re-sliced: each lane
//    fetches its window's words from the table lanes (ds_bpermute) and one
//    ballot per word forms the new bit-sliced words.  Lanes past the listed
//    count give all-zero words: U_0 = 0 there, which no candidate passes.
// Returns the number of dense groups, or kNoFit when they would not fit in
// the table (the caller then scans every window).  No per-candidate state
// is live here, which keeps the register budget of scan_filtered's loop.
// Requires 3 <= P <= 13, nb * groups <= 64 and nb <= kFilterBlocks.
constexpr uint32_t kNoFit = 0xffffffffu;

// Inclusive sum of v over the 64 lanes (every lane active): within each
// row of 16 lanes, the values 1, 2, 4 and 8 lanes below are added in turn
// (row_shr; a lane with no such neighbour in its row adds 0), then row 0's
// total is added to row 1 and row 2's to row 3 (row_bcast:15 on rows 1 and
// 3), then the total of rows 0-1 to rows 2 and 3 (row_bcast:31 on rows 2
// and 3).
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xa, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xc, 0xf, false));
    return v;
}
constexpr uint32_t kListWords = 65u;   // 64 list positions and a spare entry
constexpr uint32_t kFilterBlocks = 4u;

template <int P>
__device__ __forceinline__ uint32_t filter_windows(cu32* W, uint32_t groups, uint32_t nb,
                                                   uint32_t kv, uint32_t tj, int d,
                                                   uint32_t* __restrict__ svt) {
    constexpr int L = P + 3;
    constexpr int Q = P - 3;
    uint32_t ln = lane_id();
    asm volatile("" : "+v"(ln));
    uint32_t u[7], pw[12];
    {
        const uint32_t bias_value = static_cast<uint32_t>(19 - d);
        uint32_t bias[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) bias[i] = 0u - ((bias_value >> i) & 1u);
        uint32_t m[Q > 0 ? Q : 1];
#pragma unroll
        for (int p = 0; p < (Q > 0 ? Q : 1); ++p) m[p] = 0u;
#pragma unroll
        for (int i = 0; i < 12; ++i) pw[i] = 0u;
        const bool table = tj < groups;
        if (table) {
            const uint32_t* row = (const uint32_t*)(W) + tj * (2u * L);
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const uint32_t b = (kv >> (2 * (Q - 1 - p))) & 3u;
                m[p] = (row[p] ^ (0u - (b >> 1))) | (row[L + p] ^ (0u - (b & 1u)));
            }
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                pw[i] = row[Q + i];
                pw[6 + i] = row[L + Q + i];
            }
        }
        uint32_t c[5];
        count_bits<Q>(m, bias, c);
        // Lanes that are no table lane hold no windows.
        const uint32_t on = table ? ~0u : 0u;
        u[0] = on & ~(c[4] & (c[3] | c[2]));
        u[1] = on & ~(c[4] & (c[3] | c[2] | (c[1] & c[0])));
        u[2] = on & ~(c[4] & (c[3] | c[2] | c[1]));
        u[3] = on & ~(c[4] & (c[3] | c[2] | c[1] | c[0]));
        u[4] = on & ~c[4];
        u[5] = on & ~(c[4] | (c[3] & c[2] & c[1] & c[0]));
        u[6] = on & ~(c[4] | (c[3] & c[2] & c[1]));
    }
    // Lane j < groups: the windows of window group j that pass for some block.
    uint32_t um = 0;
    for (uint32_t b = 0; b < nb; ++b)
        um |= static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(
            static_cast<int>((b * groups + ln) << 2), static_cast<int>(u[0])));
    um = ln < groups ? um : 0u;
    // Total and each lane's offset in the list: an inclusive sum of the
    // counts over the lanes.
    const uint32_t pc = static_cast<uint32_t>(__builtin_popcount(um));
    const uint32_t incl = wave_inclusive_sum(pc);
    const uint32_t total = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(incl), 63));
    const uint32_t off = incl - pc;
    const uint32_t stride = 12u + 8u * nb;
    const uint32_t dense = (total + 31u) >> 5;
    if (dense * stride + kListWords > PMS_SVT_WORDS) return kNoFit;
    uint32_t* const list = svt + (PMS_SVT_WORDS - kListWords);
    uint32_t nv = 0;
    for (uint32_t base = 0; base < total; base += 64u) {
        // List positions [base, base + 64): each lane writes its passing
        // windows' numbers in order, one per round while some lane has one
        // left below base + 64; a lane with none in range writes the spare
        // entry 64 instead, so every round is one store with no branch.
        {
            uint32_t mm = um, at = off;
            const uint32_t lim = base + 64u;
            while (ballot(mm != 0u && at < lim) != 0u) {
                const bool put = mm != 0u && at - base < 64u;
                const uint32_t bit = static_cast<uint32_t>(__builtin_ffs(static_cast<int>(mm))) - 1u;
                list[put ? at - base : 64u] = 32u * ln + bit;
                mm &= mm - 1u;
                ++at;
            }
        }
        __builtin_amdgcn_wave_barrier();
        const uint32_t cnt = total - base < 64u ? total - base : 64u;
        const bool valid = ln < cnt;
        const uint32_t wi = valid ? list[ln] : 0u;
        __builtin_amdgcn_wave_barrier();
        const uint32_t g = wi >> 5;
        // The lane's bit in the words it fetches (none past the list's end),
        // so that each ballot below is one compare.
        const uint32_t sel = valid ? 1u << (wi & 31u) : 0u;
        uint32_t lo = 0, hi = 0;
        // Plane words: from lane g (block 0's table lane of window group g).
        uint32_t x[12];
#pragma unroll
        for (int i = 0; i < 12; ++i)
            x[i] = static_cast<uint32_t>(
                __builtin_amdgcn_ds_bpermute(static_cast<int>(g << 2), static_cast<int>(pw[i])));
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const uint64_t bm = ballot((x[i] & sel) != 0u);
            lo = static_cast<uint32_t>(write_lane(static_cast<int>(static_cast<uint32_t>(bm)), i,
                                                  static_cast<int>(lo)));
            hi = static_cast<uint32_t>(write_lane(static_cast<int>(static_cast<uint32_t>(bm >> 32)),
                                                  i, static_cast<int>(hi)));
        }
        // Thresholds of each block: from lane b * groups + g.
        for (uint32_t b = 0; b < nb; ++b) {
            const int src = static_cast<int>((b * groups + g) << 2);
            uint32_t y[7];
#pragma unroll
            for (int k = 0; k < 7; ++k)
                y[k] = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(src, static_cast<int>(u[k])));
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                const uint64_t bm = ballot((y[k] & sel) != 0u);
                const int at = static_cast<int>(12u + 8u * b) + k;
                lo = static_cast<uint32_t>(write_lane(static_cast<int>(static_cast<uint32_t>(bm)), at,
                                                      static_cast<int>(lo)));
                hi = static_cast<uint32_t>(write_lane(
                    static_cast<int>(static_cast<uint32_t>(bm >> 32)), at, static_cast<int>(hi)));
            }
        }
        if (ln < stride) {
            svt[nv * stride + ln] = lo;
            if (cnt > 32u) svt[(nv + 1u) * stride + ln] = hi;
        }
        nv += cnt > 32u ? 2u : 1u;
    }
    __builtin_amdgcn_wave_barrier();
    return nv;
}

// The most blocks (up to kFilterBlocks) over which the window filter is
// expected to keep at most the fraction `pass_max` of the windows, so that it
// pays for its re-slicing: a random window is within d of a block's Q shared
// bases with probability p = sum_{k<=d} C(Q,k) 3^k / 4^Q, and of some block's
// of nb with 1 - (1-p)^nb.  0 when even one block keeps more.  Group batches
// take 1/2; single-candidate batches, whose own scan costs about 0.4 of a
// group scan per window group, take 1/6.
__device__ __forceinline__ uint32_t filter_block_limit(uint32_t Q, int d, double pass_max) {
    double ball = 0.0, c = 1.0, p3 = 1.0;
    for (uint32_t k = 0; k <= Q && static_cast<int>(k) <= d; ++k) {
        ball += c * p3;
        c = c * static_cast<double>(Q - k) / static_cast<double>(k + 1);
        p3 *= 3.0;
    }
    const double keep = 1.0 - ball / ldexp(1.0, 2 * static_cast<int>(Q));
    double r = 1.0;
    uint32_t nb = 0;
    for (uint32_t b = 1; b <= kFilterBlocks; ++b) {
        r *= keep;
        if (r >= 1.0 - pass_max) nb = b;
    }
    return nb;
}

// Dispatch on P (wave-uniform, 3..13).
__device__ __forceinline__ uint32_t filter_windows_any(uint32_t P, cu32* W, uint32_t groups,
                                                       uint32_t nb, uint32_t kv, uint32_t tj,
                                                       int d, uint32_t* svt) {
    switch (P) {
        case 3: return filter_windows<3>(W, groups, nb, kv, tj, d, svt);
        case 4: return filter_windows<4>(W, groups, nb, kv, tj, d, svt);
        case 5: return filter_windows<5>(W, groups, nb, kv, tj, d, svt);
        case 6: return filter_windows<6>(W, groups, nb, kv, tj, d, svt);
        case 7: return filter_windows<7>(W, groups, nb, kv, tj, d, svt);
        case 8: return filter_windows<8>(W, groups, nb, kv, tj, d, svt);
        case 9: return filter_windows<9>(W, groups, nb, kv, tj, d, svt);
        case 10: return filter_windows<10>(W, groups, nb, kv, tj, d, svt);
        case 11: return filter_windows<11>(W, groups, nb, kv, tj, d, svt);
        case 12: return filter_windows<12>(W, groups, nb, kv, tj, d, svt);
        default: return filter_windows<13>(W, groups, nb, kv, tj, d, svt);
    }
}

// Window filter attempt for a group batch (64-candidate kernel): counts the
// live lanes' blocks of 64 consecutive groups (key = the group's first l - 6
// bases), and when they are at most `lim` and fit the table lanes (`tab`
// blocks, 64 / groups), runs filter_windows.  `one`: the batch's block when
// the caller knows it is a single one (64 consecutive groups from the start
// of a block), else kNoKey.  Returns the dense group count (kNoFit
// otherwise) with the block count and the lane's block.
constexpr uint32_t kNoKey = 0xffffffffu;

__device__ __forceinline__ uint32_t try_filter(uint32_t lim, uint32_t tab, uint32_t one, uint32_t key,
                                               bool live, uint32_t P, cu32* W, uint32_t groups,
                                               int d, uint32_t* svt, uint32_t& fblk, uint32_t& fmyb) {
    fblk = 0;
    fmyb = 0;
    if (lim == 0u || P < 3u || groups > 64u) return kNoFit;
    const uint32_t lane = lane_id();
    if (one != kNoKey) {
        fblk = 1;
        return filter_windows_any(P, W, groups, 1u, one, lane < groups ? lane : 64u, d, svt);
    }
    const uint32_t kmax = tab < lim ? tab : lim;
    uint64_t todo = ballot(live);
    for (; todo != 0 && fblk <= kmax; ++fblk) {
        const uint32_t v = static_cast<uint32_t>(__builtin_amdgcn_readlane(
            static_cast<int>(key), static_cast<int>(__builtin_ctzll(todo))));
        todo &= ~ballot(key == v);
    }
    if (todo != 0 || fblk < 1u || fblk > kmax) return kNoFit;
    uint32_t kv = 0, tj = 64u;
    todo = ballot(live);
    for (uint32_t k = 0; todo != 0; ++k) {
        const uint32_t v = static_cast<uint32_t>(__builtin_amdgcn_readlane(
            static_cast<int>(key), static_cast<int>(__builtin_ctzll(todo))));
        const bool mine = key == v;
        todo &= ~ballot(mine);
        const uint32_t b = k * groups;
        if (mine) fmyb = k;
        if (lane - b < groups) {
            kv = v;
            tj = lane - b;
        }
    }
    return filter_windows_any(P, W, groups, fblk, kv, tj, d, svt);
}

// Scan of the nv dense window groups filter_windows left in `svt` (stride
// words each) for the lane's group of 64 candidates: myb = the lane's block
// in the batch, low = its last three prefix bases.  Per group the block's
// thresholds U_k walk through the lane's three prefix positions (as in
// scan_group_shared) and the selection tree runs over the three suffix
// positions.  Every word comes from LDS (the plane words by broadcast reads,
// the thresholds from the lane's block), so the loop issues no instruction
// with an SGPR operand.
__device__ __forceinline__ uint64_t scan_filtered(uint32_t nv, uint32_t stride, uint32_t myb,
                                                  const uint32_t* __restrict__ svt, uint32_t low,
                                                  uint64_t alive) {
    constexpr int S = 3;
    constexpr int K = 64;
    constexpr int N1 = K / 4;
    if (nv == 0) return 0;
    uint32_t ch[3], cl[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const uint32_t b = (low >> (2 * (2 - q))) & 3u;
        ch[q] = 0u - (b >> 1);
        cl[q] = 0u - (b & 1u);
    }
    uint32_t found[K], top[N1];
    const uint4* sp = reinterpret_cast<const uint4*>(svt);
    const uint32_t ub = (12u + 8u * myb) >> 2;   // the lane's thresholds, in uint4 units
    for (uint32_t g = 0; g < nv; ++g) {
        const uint32_t at = g * (stride >> 2);
        uint32_t x[12], uu[8];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const uint4 v = sp[at + i];
            x[4 * i] = v.x;
            x[4 * i + 1] = v.y;
            x[4 * i + 2] = v.z;
            x[4 * i + 3] = v.w;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const uint4 v = sp[at + ub + i];
            uu[4 * i] = v.x;
            uu[4 * i + 1] = v.y;
            uu[4 * i + 2] = v.z;
            uu[4 * i + 3] = v.w;
        }
        // x: 0..5 high plane of positions Q..Q+5, 6..11 low plane.
        uint32_t m[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) m[q] = bop3<kOrXor>(x[q] ^ ch[q], x[6 + q], cl[q]);
        uint32_t v1[6], v2[5], t[4];
#pragma unroll
        for (int k = 0; k < 6; ++k) v1[k] = bop3<kMux>(m[0], uu[k + 1], uu[k]);
#pragma unroll
        for (int k = 0; k < 5; ++k) v2[k] = bop3<kMux>(m[1], v1[k + 1], v1[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k) t[k] = bop3<kMux>(m[2], v2[k + 1], v2[k]);
        uint32_t sv[S][4];
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const uint32_t h = x[3 + q], lo = x[9 + q];
            sv[q][0] = bop3<0xFC>(h, lo, 0u);   // h | lo
            sv[q][1] = bop3<0xF3>(h, lo, 0u);   // h | ~lo
            sv[q][2] = bop3<0xCF>(h, lo, 0u);   // ~h | lo
            sv[q][3] = bop3<0x3F>(h, lo, 0u);   // ~(h & lo)
        }
        if (g == 0)
            select_accumulate<S, true>(t, sv, found, top);
        else
            select_accumulate<S>(t, sv, found, top);
    }
    return group_pass<S>(found, top) & alive;
}

// Scan of the nv dense window groups filter_windows left in `svt` for the
// lane's single candidate: myb = its block in the batch, low6 = its last six
// bases (2 bits each, the first of them most significant).  Per dense group
// the block's thresholds U_0..U_6 walk through the six unshared positions,
// U_k <- mismatch ? U_{k+1} : U_k, and what is left, U_0, marks the windows
// within d of the whole l-mer (33 VALU per dense group).
__device__ __forceinline__ bool scan_filtered_single(uint32_t nv, uint32_t stride, uint32_t myb,
                                                     const uint32_t* __restrict__ svt, uint32_t low6) {
    if (nv == 0) return false;
    uint32_t ch[6], cl[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const uint32_t b = (low6 >> (2 * (5 - q))) & 3u;
        ch[q] = 0u - (b >> 1);
        cl[q] = 0u - (b & 1u);
    }
    uint32_t found = 0;
    const uint4* sp = reinterpret_cast<const uint4*>(svt);
    const uint32_t ub = (12u + 8u * myb) >> 2;   // the block's thresholds, in uint4 units
    for (uint32_t g = 0; g < nv; ++g) {
        const uint32_t at = g * (stride >> 2);
        uint32_t x[12], v[8];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const uint4 w = sp[at + i];
            x[4 * i] = w.x;
            x[4 * i + 1] = w.y;
            x[4 * i + 2] = w.z;
            x[4 * i + 3] = w.w;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const uint4 w = sp[at + ub + i];
            v[4 * i] = w.x;
            v[4 * i + 1] = w.y;
            v[4 * i + 2] = w.z;
            v[4 * i + 3] = w.w;
        }
        // x: 0..5 high plane of positions Q..Q+5, 6..11 low plane.
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const uint32_t m = bop3<kOrXor>(x[q] ^ ch[q], x[6 + q], cl[q]);
#pragma unroll
            for (int k = 0; k < 6 - q; ++k) v[k] = bop3<kMux>(m, v[k + 1], v[k]);
        }
        found |= v[0];
    }
    return found != 0u;
}

// One sequence scan for one candidate per lane: whether some window is
// within d of the l-mer `code` (motif code).  All L positions are counted
// per lane by the carry-save tree of scan_group, with no selection tree; the
// bias is 15 - d, so c' = c + 15 - d < 32 and [c <= d] is ~c'16.  Used for
// the live members of groups that have few left: per 32 windows it costs
// about a third of a group scan.
template <int L>
__device__ __forceinline__ bool scan_single(cu32* W, uint32_t groups, uint32_t code, int d) {
    uint32_t ch[L], cl[L];
#pragma unroll
    for (int p = 0; p < L; ++p) {
        const uint32_t b = (code >> (2 * (L - 1 - p))) & 3u;
        ch[p] = 0u - (b >> 1);
        cl[p] = 0u - (b & 1u);
    }
    const uint32_t bias_value = static_cast<uint32_t>(15 - d);
    uint32_t bias[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) bias[i] = to_vgpr(0u - ((bias_value >> i) & 1u));
    uint32_t found = 0u;
    uint32_t w[2 * L];
#pragma unroll
    for (int i = 0; i < 2 * L; ++i) w[i] = ((__attribute__((address_space(4))) const volatile uint32_t*)W)[i];
    for (uint32_t gi = 0; gi < groups; ++gi) {
        uint32_t m[L];
#pragma unroll
        for (int p = 0; p < L; ++p) m[p] = (w[p] ^ ch[p]) | (w[L + p] ^ cl[p]);
        // The mismatch vectors are complete here: the next group's words
        // load while they are counted.
#pragma unroll
        for (int p = 0; p < L; ++p) asm volatile("" : "+v"(m[p]));
        W += gi + 1 < groups ? 2 * L : 0;
        asm volatile("" : "+s"(W));
#pragma unroll
        for (int i = 0; i < 2 * L; ++i) w[i] = W[i];
        uint32_t c[5];
        count_bits<L>(m, bias, c);
        found |= ~c[4];
    }
    return found != 0u;
}

// Dispatch on l (wave-uniform, 3 <= l <= 16).  d >= l: every window is
// within d.
__device__ __forceinline__ bool scan_single_any(uint32_t L, cu32* W, uint32_t groups, uint32_t code,
                                                int d) {
    if (d >= static_cast<int>(L)) return true;
    switch (L) {
        case 3: return scan_single<3>(W, groups, code, d);
        case 4: return scan_single<4>(W, groups, code, d);
        case 5: return scan_single<5>(W, groups, code, d);
        case 6: return scan_single<6>(W, groups, code, d);
        case 7: return scan_single<7>(W, groups, code, d);
        case 8: return scan_single<8>(W, groups, code, d);
        case 9: return scan_single<9>(W, groups, code, d);
        case 10: return scan_single<10>(W, groups, code, d);
        case 11: return scan_single<11>(W, groups, code, d);
        case 12: return scan_single<12>(W, groups, code, d);
        case 13: return scan_single<13>(W, groups, code, d);
        case 14: return scan_single<14>(W, groups, code, d);
        case 15: return scan_single<15>(W, groups, code, d);
        default: return scan_single<16>(W, groups, code, d);
    }
}

// Persistent grouped search; S = 2 (16 candidates per lane) or 3 (64).
// Per stage s = 1..n-1 a wavefront has a queue of groups (prefix and alive
// mask) and, for S = 3, a queue of single candidates (motif codes): a group
// that keeps at most kSparse live members after a sequence hands them on as
// singles, which cost a fraction of a group scan.  Stage queues for stages
// 1..lds_stages live in LDS; deeper stages live in a per-wavefront region of
// the global workspace `gq` (gq_words words per wavefront), which leaves room
// in LDS for more resident wavefronts.  Per stage, in both places: group
// prefixes [QCAP] u32, masks [QCAP] Mask, then (S = 3) singles [SCAP] u32.
template <int S>
__device__ __forceinline__ void search_groups(const pms_dev_instance* __restrict__ insts,
                                              const pms_work_item* __restrict__ work,
                                              uint32_t n_work, pms_dev_state* __restrict__ state,
                                              pms_dev_counters* __restrict__ ctr,
                                              uint32_t lds_stages, uint32_t* __restrict__ gq,
                                              uint32_t gq_words, uint32_t flags) {
    typedef typename MaskOf<S>::type Mask;
    constexpr int K = 1 << (2 * S);
    constexpr uint32_t kNone = 0xffffffffu;
    constexpr Mask kAll = static_cast<Mask>(~static_cast<Mask>(0)) >> (8 * sizeof(Mask) - K);
    constexpr uint32_t kEntryWords = 1 + sizeof(Mask) / 4;
    constexpr bool kSingles = S == 3;
    // A group with at most this many live members splits into singles (one
    // fewer where d >= 4, the singles' window filter is on and the filter's
    // table holds two blocks or more: there a filtered group scan of two
    // members costs less than their two single scans).  1 or 2 only: the singles push below writes a group's lowest
    // and highest live codes, so a third member would be lost.
    constexpr uint32_t kSparse = 2;
    constexpr uint32_t kStageWords = pms::stage_queue_words(S);
    constexpr uint32_t kSingleOff = kEntryWords * PMS_QCAP;
    extern __shared__ uint32_t lds[];
    const uint32_t lane = lane_id();
    const uint32_t wave = uni(threadIdx.x >> 6);
    uint32_t* const qp = lds + wave * (lds_stages * kStageWords + pms::wave_fixed_words(S));
    uint32_t* const ob = qp + lds_stages * kStageWords;
    uint32_t* const svt = ob + PMS_OUTBUF;   // S = 3: shared-prefix scans' suffix vectors
    const uint32_t gwave = blockIdx.x * uni(blockDim.x >> 6) + wave;
    uint32_t* const gw = gq + static_cast<size_t>(gwave) * gq_words;
    const uint32_t stages_cap = lds_stages + gq_words / kStageWords;
    const bool filter = (flags & PMS_LAUNCH_NO_FILTER) == 0u;

    uint32_t cur = kNone, pending = 0, stash = kNone;
    bool more = true;
    uint32_t next = 0, end = 0;     // group numbers (below 2^28)
    // Launch statistics, one per lane of one register: lane 0 batches, 1
    // single-candidate batches, 2 filtered group batches, 3 their dense
    // groups (kept out of the scalar registers, which the loop fills).
    uint32_t stat = 0;
    uint64_t visits = 0;            // per lane
    uint32_t nob = 0;
    // Lane s: groups queued for stage s (low 16 bits) and singles (high 16).
    uint32_t qc = 0;

    // The current instance's parameters.  Its output pointer and capacity
    // are read from its record at each flush of the survivor buffer (rare)
    // instead: the loop's scalar registers are full, and every one taken
    // out of them removed spills to vector lanes.
    cu32* W = nullptr;
    uint32_t n = 0, row = 0, groups = 0, P = 0;
    uint32_t fmax = 0;    // window filter: most blocks per batch (0: off)
    uint32_t sfmax = 0;   // the same for single-candidate batches
    uint32_t tab = 0;     // blocks whose window groups fit the table lanes: 64 / groups
    int d = 0;

    // Wave priority: raised for the bookkeeping between scans (queue pops and
    // pushes, claims, the window filter's phase 1), which is a chain of
    // dependent LDS, ballot and scalar steps, and lowered for the scans,
    // which are long runs of independent VALU work.  A wavefront waiting on
    // its chain then issues as soon as its operands arrive, and the scans of
    // the other wavefronts on the SIMD fill the issue slots between.
    constexpr int kPrioChain = 2, kPrioScan = 0;
    __builtin_amdgcn_s_setprio(kPrioChain);
    for (;;) {
        // prefix: a group's prefix, or a single's motif code.
        uint32_t s, prefix = 0;
        Mask alive = 0;
        bool single = false;
        uint32_t one = kNoKey;   // the batch's block, when it is known to be a single one
        const uint64_t full = ballot((qc & 0xffffu) >= 64u);
        const uint64_t sfull = kSingles ? ballot(qc >= (64u << 16)) : 0;
        if (full | sfull) {
            // The deepest full queue: at most one queue is ever full, and
            // scanning it pushes no more than 64 groups, or 64 singles, or
            // as many singles as fit, onto the next stage's queues.
            const int sg = full ? 63 - __builtin_clzll(full) : -1;
            const int ss = sfull ? 63 - __builtin_clzll(sfull) : -1;
            single = ss > sg;
            s = static_cast<uint32_t>(single ? ss : sg);
            const uint32_t cw = __builtin_amdgcn_readlane(qc, s);
            const uint32_t at = (single ? cw >> 16 : cw & 0xffffu) - 64u + lane;
            const uint32_t r = s - 1;
            if (r < lds_stages) {
                const uint32_t* q = qp + r * kStageWords;
                if (single) {
                    prefix = q[kSingleOff + at];
                    alive = 1;
                } else {
                    prefix = q[at];
                    alive = reinterpret_cast<const Mask*>(q + PMS_QCAP)[at];
                }
            } else {
                const uint32_t* g = gw + (r - lds_stages) * kStageWords;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                if (single) {
                    prefix = g[kSingleOff + at];
                    alive = 1;
                } else {
                    prefix = g[at];
                    alive = reinterpret_cast<const Mask*>(g + PMS_QCAP)[at];
                }
            }
            if (lane == s) qc -= single ? (64u << 16) : 64u;
        } else if (next < end) {
            s = 0;
            const uint32_t g = next + lane;
            prefix = static_cast<uint32_t>(g);
            alive = g < end ? kAll : static_cast<Mask>(0);
            if constexpr (S == 3)
                if ((next & 63u) == 0u) one = static_cast<uint32_t>(next >> 6);
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
                        next = static_cast<uint32_t>(wi.begin >> (2 * S));
                        end = static_cast<uint32_t>((wi.begin + wi.len) >> (2 * S));
                    } else {
                        stash = item;
                    }
                }
                continue;
            }
            const uint64_t nz = ballot((qc & 0xffffu) > 0u);
            const uint64_t snz = kSingles ? ballot(qc > 0xffffu) : 0;
            if ((nz | snz) == 0) {
                if (cur != kNone) {
                    if (nob) {
                        uint64_t base = 0;
                        if (lane == 0)
                            base = atomicAdd(reinterpret_cast<unsigned long long*>(&state[cur].count),
                                             static_cast<unsigned long long>(nob));
                        base = uni64(base);
                        const pms_dev_instance ci = load_uniform(insts + cur);
                        for (uint32_t i = lane; i < nob; i += 64u)
                            if (base + i < ci.out_cap) ci.out[base + i] = ob[i];
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
                if (in.n < 1 || in.l < S || (static_cast<uint32_t>(in.n) - 1u) > stages_cap) {
                    if (lane == 0) atomicOr(&ctr->error, 1u);
                    continue;
                }
                cur = wi.inst;
                W = (cu32*)(in.windows);
                n = static_cast<uint32_t>(in.n);
                row = static_cast<uint32_t>(in.nw_stride);
                P = static_cast<uint32_t>(in.l) - S;
                groups = row / (2u * (P + S));
                d = in.d;
                if constexpr (S == 3) {
                    fmax = filter && P >= 3u ? uni(filter_block_limit(P - 3u, d, 0.5)) : 0u;
                    sfmax = filter && P >= 3u ? uni(filter_block_limit(P - 3u, d, 1.0 / 6.0)) : 0u;
                    tab = groups ? uni(64u / groups) : 0u;
                }
                pending = 1;
                next = static_cast<uint32_t>(wi.begin >> (2 * S));
                end = static_cast<uint32_t>((wi.begin + wi.len) >> (2 * S));
                continue;
            }
            // No queue is full and no new work: drain the shallowest queue.
            const int sg = nz ? __builtin_ctzll(nz) : 64;
            const int ss = snz ? __builtin_ctzll(snz) : 64;
            single = ss < sg;
            s = static_cast<uint32_t>(single ? ss : sg);
            const uint32_t cw = __builtin_amdgcn_readlane(qc, s);
            const uint32_t c = single ? cw >> 16 : cw & 0xffffu;
            const uint32_t r = s - 1;
            if (r < lds_stages) {
                const uint32_t* q = qp + r * kStageWords;
                if (lane < c) {
                    if (single) {
                        prefix = q[kSingleOff + lane];
                        alive = 1;
                    } else {
                        prefix = q[lane];
                        alive = reinterpret_cast<const Mask*>(q + PMS_QCAP)[lane];
                    }
                }
            } else {
                const uint32_t* g = gw + (r - lds_stages) * kStageWords;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                if (lane < c) {
                    if (single) {
                        prefix = g[kSingleOff + lane];
                        alive = 1;
                    } else {
                        prefix = g[lane];
                        alive = reinterpret_cast<const Mask*>(g + PMS_QCAP)[lane];
                    }
                }
            }
            if (lane == s) qc &= single ? 0xffffu : 0xffff0000u;
        }

        if (kSingles && single) {
            // One sequence scan for up to 64 single candidates: through the
            // window filter when their codes fall into at most sfmax blocks
            // of 4096 candidates (block key: the first l - 6 bases), else
            // every window.
            const bool live = alive != 0;
            uint32_t fblk, fmyb;
            const uint32_t nv = try_filter(sfmax, tab, kNoKey, prefix >> 12, live, P, W + s * row,
                                           groups, d, svt, fblk, fmyb);
            bool ok;
            __builtin_amdgcn_s_setprio(kPrioScan);
            if (nv != kNoFit)
                ok = live && scan_filtered_single(nv, 12u + 8u * fblk, fmyb, svt, prefix & 0xfffu);
            else
                ok = live && scan_single_any(P + S, W + s * row, groups, prefix, d);
            __builtin_amdgcn_s_setprio(kPrioChain);
            visits += live ? 1u : 0u;
            stat += lane < 2u ? 1u : 0u;
            const uint64_t pm = ballot(ok);
            if (pm) {
                const uint32_t rk = rank_below(pm);
                if (s + 1 < n) {
                    const uint32_t base = __builtin_amdgcn_readlane(qc, s + 1) >> 16;
                    const uint32_t r = s;
                    if (r < lds_stages) {
                        if (ok) qp[r * kStageWords + kSingleOff + base + rk] = prefix;
                    } else {
                        uint32_t* g = gw + (r - lds_stages) * kStageWords;
                        if (ok) g[kSingleOff + base + rk] = prefix;
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    }
                    if (lane == s + 1) qc += static_cast<uint32_t>(__builtin_popcountll(pm)) << 16;
                } else {
                    if (ok) ob[nob + rk] = prefix;
                    nob += static_cast<uint32_t>(__builtin_popcountll(pm));
                    if (nob > PMS_OUTBUF - 64u) {
                        uint64_t base = 0;
                        if (lane == 0)
                            base = atomicAdd(reinterpret_cast<unsigned long long*>(&state[cur].count),
                                             static_cast<unsigned long long>(nob));
                        base = uni64(base);
                        const pms_dev_instance ci = load_uniform(insts + cur);
                        for (uint32_t i = lane; i < nob; i += 64u)
                            if (base + i < ci.out_cap) ci.out[base + i] = ob[i];
                        nob = 0;
                    }
                }
            }
            continue;
        }

        // One sequence scan for 64 groups.
        Mask pass;
        if constexpr (S == 3) {
            // The window filter's dense groups when it ran; otherwise, when
            // the live lanes' blocks of 64 consecutive groups all fit the
            // table lanes, the shared-prefix scan of every window.  (Counted
            // first with wave-uniform values only, then the per-lane block
            // data inside the branch that uses it: computed ahead of the
            // branch, it cost the general scan registers.)
            bool done = false;
            uint32_t fblk, fmyb;
            const uint32_t nv = try_filter(fmax, tab, one, prefix >> 6, alive != 0, P, W + s * row,
                                           groups, d, svt, fblk, fmyb);
            if (nv != kNoFit) {
                __builtin_amdgcn_s_setprio(kPrioScan);
                pass = scan_filtered(nv, 12u + 8u * fblk, fmyb, svt, prefix & 63u, alive);
                __builtin_amdgcn_s_setprio(kPrioChain);
                stat += lane == 2u ? 1u : (lane == 3u ? nv : 0u);
                done = true;
            } else if (P >= 3u && groups * 12u <= PMS_SVT_WORDS) {
                uint32_t nblk = 0;
                uint64_t todo = one != kNoKey ? 0u : ballot(alive != 0);
                for (; todo != 0 && nblk <= tab; ++nblk) {
                    const uint32_t v = static_cast<uint32_t>(__builtin_amdgcn_readlane(
                        static_cast<int>(prefix >> 6), static_cast<int>(__builtin_ctzll(todo))));
                    todo &= ~ballot((prefix >> 6) == v);
                }
                if (todo == 0 && nblk <= tab) {
                    const uint32_t hi = prefix >> 6;
                    uint32_t kv = one != kNoKey ? one : 0u;
                    uint32_t tj = one != kNoKey && lane < groups ? lane : 64u, myb = 0;
                    todo = one != kNoKey ? 0u : ballot(alive != 0);
                    for (uint32_t k = 0; todo != 0; ++k) {
                        const uint32_t v = static_cast<uint32_t>(__builtin_amdgcn_readlane(
                            static_cast<int>(hi), static_cast<int>(__builtin_ctzll(todo))));
                        const bool mine = hi == v;
                        todo &= ~ballot(mine);
                        const uint32_t b = k * groups;
                        if (mine) myb = k;
                        if (lane - b < groups) {
                            kv = v;
                            tj = lane - b;
                        }
                    }
                    __builtin_amdgcn_s_setprio(kPrioScan);
                    pass = scan_group_shared_any(P, W + s * row, groups, kv, tj, myb * groups,
                                                 prefix & 63u, d, alive, svt);
                    __builtin_amdgcn_s_setprio(kPrioChain);
                    done = true;
                }
            }
            if (!done) {
                __builtin_amdgcn_s_setprio(kPrioScan);
                pass = scan_group_any<S>(P, W + s * row, groups, prefix, d, alive);
                __builtin_amdgcn_s_setprio(kPrioChain);
            }
        } else {
            __builtin_amdgcn_s_setprio(kPrioScan);
            pass = scan_group_any<S>(P, W + s * row, groups, prefix, d, alive);
            __builtin_amdgcn_s_setprio(kPrioChain);
        }
        visits += static_cast<uint32_t>(__builtin_popcountll(static_cast<uint64_t>(alive)));
        stat += lane == 0u ? 1u : 0u;
        const bool keep = pass != 0;
        const uint64_t pm = ballot(keep);
        if (pm) {
            if (s + 1 < n) {
                const uint32_t live = static_cast<uint32_t>(__builtin_popcountll(static_cast<uint64_t>(pass)));
                const bool sparse = kSingles && keep &&
                                    live <= kSparse - (d >= 4 && sfmax != 0u && tab >= 2u ? 1u : 0u);
                const uint64_t dm = kSingles ? ballot(keep && !sparse) : pm;
                const uint32_t r = s;
                if (dm) {
                    const uint32_t base = __builtin_amdgcn_readlane(qc, s + 1) & 0xffffu;
                    const uint32_t rk = rank_below(dm);
                    const bool dense = keep && !sparse;
                    if (r < lds_stages) {
                        uint32_t* q = qp + r * kStageWords;
                        if (dense) {
                            q[base + rk] = prefix;
                            reinterpret_cast<Mask*>(q + PMS_QCAP)[base + rk] = pass;
                        }
                    } else {
                        uint32_t* g = gw + (r - lds_stages) * kStageWords;
                        if (dense) {
                            g[base + rk] = prefix;
                            reinterpret_cast<Mask*>(g + PMS_QCAP)[base + rk] = pass;
                        }
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    }
                    if (lane == s + 1) qc += static_cast<uint32_t>(__builtin_popcountll(dm));
                }
                if constexpr (kSingles) {
                    // Sparse groups: their one or two live members as
                    // singles, in lane order while the singles queue has
                    // room; the rest (rarely any) go on as groups after all.
                    const uint64_t b1 = ballot(sparse && live == 1u);
                    const uint64_t b2 = ballot(sparse && live == 2u);
                    if (b1 | b2) {
                        const uint32_t sbase = __builtin_amdgcn_readlane(qc, s + 1) >> 16;
                        const uint32_t at = sbase + rank_below(b1) + 2u * rank_below(b2);
                        uint32_t total = static_cast<uint32_t>(__builtin_popcountll(b1) + 2 * __builtin_popcountll(b2));
                        bool fits = sparse;
                        uint64_t over = 0;
                        if (sbase + total > PMS_SCAP) {
                            fits = sparse && at + live <= PMS_SCAP;
                            over = ballot(sparse && !fits);
                            total = static_cast<uint32_t>(__builtin_popcountll(ballot(fits && live == 1u)) +
                                                          2 * __builtin_popcountll(ballot(fits && live == 2u)));
                        }
                        const uint64_t pw = static_cast<uint64_t>(pass);
                        const uint32_t lo = (prefix << (2 * S)) | static_cast<uint32_t>(__builtin_ctzll(pw));
                        const uint32_t hi = (prefix << (2 * S)) | static_cast<uint32_t>(63 - __builtin_clzll(pw));
                        if (r < lds_stages) {
                            uint32_t* q = qp + r * kStageWords + kSingleOff;
                            if (fits) {
                                q[at] = lo;
                                if (live == 2u) q[at + 1] = hi;
                            }
                        } else {
                            uint32_t* g = gw + (r - lds_stages) * kStageWords + kSingleOff;
                            if (fits) {
                                g[at] = lo;
                                if (live == 2u) g[at + 1] = hi;
                            }
                            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                        }
                        if (lane == s + 1) qc += total << 16;
                        if (over) {
                            // Groups whose members did not fit: group queue
                            // (with the dense ones, at most 64 pushed).
                            const uint32_t base = __builtin_amdgcn_readlane(qc, s + 1) & 0xffffu;
                            const uint32_t rk = rank_below(over);
                            const bool push = sparse && !fits;
                            if (r < lds_stages) {
                                uint32_t* q = qp + r * kStageWords;
                                if (push) {
                                    q[base + rk] = prefix;
                                    reinterpret_cast<Mask*>(q + PMS_QCAP)[base + rk] = pass;
                                }
                            } else {
                                uint32_t* g = gw + (r - lds_stages) * kStageWords;
                                if (push) {
                                    g[base + rk] = prefix;
                                    reinterpret_cast<Mask*>(g + PMS_QCAP)[base + rk] = pass;
                                }
                                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                            }
                            if (lane == s + 1) qc += static_cast<uint32_t>(__builtin_popcountll(over));
                        }
                    }
                }
            } else {
                // Survivors: each lane writes its alive candidates in turn;
                // every round compacts one code per lane by ballot.
                Mask left = pass;
                for (;;) {
                    const bool hit = left != 0;
                    const uint64_t hm = ballot(hit);
                    if (!hm) break;
                    if (hit) {
                        const uint32_t c = static_cast<uint32_t>(__builtin_ctzll(static_cast<uint64_t>(left)));
                        ob[nob + rank_below(hm)] = (prefix << (2 * S)) | c;
                        left &= left - 1;
                    }
                    nob += static_cast<uint32_t>(__builtin_popcountll(hm));
                    if (nob > PMS_OUTBUF - 64u) {
                        uint64_t base = 0;
                        if (lane == 0)
                            base = atomicAdd(reinterpret_cast<unsigned long long*>(&state[cur].count),
                                             static_cast<unsigned long long>(nob));
                        base = uni64(base);
                        const pms_dev_instance ci = load_uniform(insts + cur);
                        for (uint32_t i = lane; i < nob; i += 64u)
                            if (base + i < ci.out_cap) ci.out[base + i] = ob[i];
                        nob = 0;
                    }
                }
            }
        }
    }
    if (lane < 4u && stat != 0u) {
        uint64_t* const dst = lane == 0u ? &ctr->batches
                              : lane == 1u ? &ctr->single_batches
                              : lane == 2u ? &ctr->filtered_batches : &ctr->filtered_groups;
        atomicAdd(reinterpret_cast<unsigned long long*>(dst), static_cast<unsigned long long>(stat));
    }
}

}  // namespace

// At most 5 wavefronts per SIMD: with the register budget that leaves, the
// prefix masks stay in registers instead of being rebuilt every iteration.
extern "C" __global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(1, 5)))
pms_search_group_kernel(const pms_dev_instance* __restrict__ insts,
                        const pms_work_item* __restrict__ work, uint32_t n_work,
                        pms_dev_state* __restrict__ state, pms_dev_counters* __restrict__ ctr,
                        uint32_t lds_stages, uint32_t* __restrict__ gq, uint32_t gq_words,
                        uint32_t flags) {
    search_groups<2>(insts, work, n_work, state, ctr, lds_stages, gq, gq_words, flags);
}

// At most 4 wavefronts per workgroup: the 64 accumulators per lane need more
// than the 128 VGPRs a 16-wavefront workgroup could give each lane.  At least
// three wavefronts per SIMD (at most 168 VGPRs): issue rates with two are far
// lower, and left to itself the scheduler would trade the third for registers.
extern "C" __global__ void __launch_bounds__(PMS_GROUP64_MAX_THREADS)
__attribute__((amdgpu_waves_per_eu(3)))
pms_search_group64_kernel(const pms_dev_instance* __restrict__ insts,
                          const pms_work_item* __restrict__ work, uint32_t n_work,
                          pms_dev_state* __restrict__ state, pms_dev_counters* __restrict__ ctr,
                          uint32_t lds_stages, uint32_t* __restrict__ gq, uint32_t gq_words,
                          uint32_t flags) {
    search_groups<3>(insts, work, n_work, state, ctr, lds_stages, gq, gq_words, flags);
}

namespace pms {

hipError_t launch_search_group(const pms_dev_instance* insts, const pms_work_item* work,
                               uint32_t n_work, pms_dev_state* state, pms_dev_counters* ctr,
                               const GroupQueues& q, uint32_t grid, uint32_t wg_waves,
                               hipStream_t stream, int suffix, uint32_t flags) {
    const size_t lds = static_cast<size_t>(wg_waves) *
                       (q.lds_stages * stage_queue_words(suffix) + wave_fixed_words(suffix)) *
                       sizeof(uint32_t);
    if (suffix == 3)
        hipLaunchKernelGGL(pms_search_group64_kernel, dim3(grid), dim3(64 * wg_waves), lds, stream,
                           insts, work, n_work, state, ctr, q.lds_stages, q.gq, q.gq_words, flags);
    else
        hipLaunchKernelGGL(pms_search_group_kernel, dim3(grid), dim3(64 * wg_waves), lds, stream,
                           insts, work, n_work, state, ctr, q.lds_stages, q.gq, q.gq_words, flags);
    return hipGetLastError();
}

const void* search_group_kernel_symbol(int suffix) {
    return suffix == 3 ? reinterpret_cast<const void*>(&pms_search_group64_kernel)
                       : reinterpret_cast<const void*>(&pms_search_group_kernel);
}

}  // namespace pms
