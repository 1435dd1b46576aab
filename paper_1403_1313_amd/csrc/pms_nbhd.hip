// pms_nbhd.hip -- neighbourhood-intersection kernels (a second exact method).
//
// The motif set is also the intersection over sequences of the union of the
// distance-d neighbourhoods (Hamming balls) of each sequence's windows:
//     M = AND_i  OR_{w in W_i}  Ball(w, d).
// This is the sample-driven form of the Planted Motif Search family that
// Section VI names as future work.  With candidates numbered as motif codes
// (base p in bits [2(l-1-p), 2(l-1-p)+1]), the neighbours of a window code w
// are w ^ delta for the XOR masks delta that change at most d of the l 2-bit
// digits, each to a different base.  The candidate space is a bitmap of 4^l
// bits in device memory:
//
//   pms_nbhd_codes_kernel    window codes of every row (one thread a window)
//   pms_nbhd_scatter_kernel  sets bit (w ^ delta) of a row's bitmap for every
//                            window w and mask delta (global atomicOr)
//   pms_nbhd_and_kernel      M &= B over the bitmaps, counting the bits left
//   pms_nbhd_collect_kernel  motif codes of the set bits of M (one global
//                            atomicAdd per wavefront)
//   pms_nbhd_verify_kernel   once few candidates are left, checks them against
//                            the remaining sequences directly
//
// Bound: the scatter issues nw x |Ball| atomics per sequence into a bitmap
// that stays in the on-chip caches for l <= 15; zeroing, AND and collection
// stream the bitmaps in 16-byte vectors.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pms.h"
#include "pms_device.h"
#include "pms_internal.h"

using namespace pms_dev;

// Window codes: thread j of row r writes code of bases j .. j+l-1 of the
// row (first base in the top digit).  Rows are n x t bytes, already checked.
extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_codes_kernel(const uint8_t* __restrict__ seqs, int32_t t, int32_t l, int32_t nw,
                      int32_t rows, uint32_t* __restrict__ codes) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= static_cast<int64_t>(rows) * nw) return;
    const int32_t r = static_cast<int32_t>(k / nw), j = static_cast<int32_t>(k % nw);
    const uint8_t* s = seqs + static_cast<int64_t>(r) * t + j;
    uint32_t code = 0;
    for (int p = 0; p < l; ++p) {
        const uint32_t c = s[p] | 0x20u;
        const uint32_t b = c == 'a' ? 0u : c == 'c' ? 1u : c == 'g' ? 2u : 3u;
        code = (code << 2) | b;
    }
    codes[k] = code;
}

// Bitmaps are handled as whole 16-byte vectors: their length in words is a
// multiple of 4 (the words past 4^l bits stay zero).

// Zeroes `vecs` 16-byte vectors.
extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_zero_kernel(uint4* __restrict__ p, uint64_t vecs) {
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t k = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < vecs; k += step)
        p[k] = make_uint4(0u, 0u, 0u, 0u);
}

// Every (window, mask) pair of one row: a grid-stride loop over the pairs,
// mask index fastest, so a wavefront reads consecutive masks and one window.
// `fresh` (optional) counts the bits this pass set that were clear, from the
// values the atomics return (one atomicAdd per wavefront).
extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_scatter_kernel(const uint32_t* __restrict__ codes, int32_t nw,
                        const uint32_t* __restrict__ deltas, int32_t nd,
                        uint32_t* __restrict__ bitmap, unsigned long long* __restrict__ fresh) {
    const int64_t pairs = static_cast<int64_t>(nw) * nd;
    const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
    uint32_t set = 0;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < pairs;
         k += step) {
        const int32_t j = static_cast<int32_t>(k / nd), q = static_cast<int32_t>(k % nd);
        const uint32_t x = codes[j] ^ deltas[q];
        const uint32_t bit = 1u << (x & 31u);
        set += (atomicOr(bitmap + (x >> 5), bit) & bit) ? 0u : 1u;
    }
    if (fresh) {
        unsigned long long v = set;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane_id() == 0 && v) atomicAdd(fresh, v);
    }
}

// M &= B over `vecs` 16-byte vectors; `count` accumulates the bits left (one
// atomic per wavefront).
extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_and_kernel(uint4* __restrict__ m, const uint4* __restrict__ b, uint64_t vecs,
                    unsigned long long* __restrict__ count) {
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    uint32_t bits = 0;
    for (uint64_t k = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < vecs;
         k += step) {
        const uint4 x = m[k], y = b[k];
        const uint4 v = make_uint4(x.x & y.x, x.y & y.y, x.z & y.z, x.w & y.w);
        m[k] = v;
        bits += static_cast<uint32_t>(__builtin_popcount(v.x) + __builtin_popcount(v.y) +
                                      __builtin_popcount(v.z) + __builtin_popcount(v.w));
    }
    unsigned long long v = bits;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane_id() == 0 && v) atomicAdd(count, v);
}

// Codes of the set bits of M (`vecs` 16-byte vectors), unsorted, at most
// `cap` written; *count receives the number of set bits.  Each lane has
// kCollectBatch vectors in flight per round (a sparse map is almost all
// zeros, so the loop is otherwise bound by load latency).  A round that
// finds bits reserves room for all of them with one atomic per wavefront
// and an inclusive scan of the lanes' counts, so the shared counter sees a
// single atomic per round however many bits there are.
constexpr int kCollectBatch = 8;

extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_collect_kernel(const uint4* __restrict__ m, uint64_t vecs, uint32_t* __restrict__ out,
                        uint64_t cap, unsigned long long* __restrict__ count) {
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    const uint32_t lane = lane_id();
    // Whole wavefronts iterate together so the ballots and shuffles see every lane.
    const uint64_t first = static_cast<uint64_t>(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u);
    for (uint64_t k0 = first; k0 < vecs; k0 += step * kCollectBatch) {
        uint4 x[kCollectBatch];
#pragma unroll
        for (int u = 0; u < kCollectBatch; ++u) {
            const uint64_t k = k0 + u * step + lane;
            x[u] = k < vecs ? m[k] : make_uint4(0u, 0u, 0u, 0u);
        }
        uint32_t mine = 0;
#pragma unroll
        for (int u = 0; u < kCollectBatch; ++u)
            mine += static_cast<uint32_t>(__builtin_popcount(x[u].x) + __builtin_popcount(x[u].y) +
                                          __builtin_popcount(x[u].z) + __builtin_popcount(x[u].w));
        if (!ballot(mine != 0u)) continue;
        uint32_t incl = mine;  // inclusive scan of the lanes' counts
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t v = __shfl_up(incl, off, 64);
            if (lane >= static_cast<uint32_t>(off)) incl += v;
        }
        const uint32_t total = __shfl(incl, 63, 64);
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(count, static_cast<unsigned long long>(total));
        base = uni64(base);
        uint64_t at = base + (incl - mine);
#pragma unroll
        for (int u = 0; u < kCollectBatch; ++u) {
            const uint64_t k = k0 + u * step + lane;
            const uint32_t w4[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                for (uint32_t v = w4[e]; v; v &= v - 1, ++at)
                    if (at < cap) out[at] = static_cast<uint32_t>((4 * k + e) * 32 + __builtin_ctz(v));
            }
        }
    }
}

// Survivors of the bitmap passes checked against sequences s_begin .. n-1
// directly: lane k takes survivor k; the wavefront scans one sequence at a
// time (window codes wave-uniform), a lane whose smallest distance exceeds d
// drops out, and the wavefront stops at the first sequence no lane passes
// (the enhanced rule of Section III.A).  Distance of codes x, w: the 2-bit
// digits that differ, popcount(((x ^ w) | (x ^ w) >> 1) & 0x55555555).
// Passing codes are appended to `out` (at most `cap`), *out_count counts
// them all; *visits counts (survivor, sequence) scans.
__device__ __forceinline__ uint32_t digit_mismatches(uint32_t x, uint32_t w) {
    const uint32_t y = x ^ w;
    return static_cast<uint32_t>(__builtin_popcount((y | (y >> 1)) & 0x55555555u));
}

extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_verify_kernel(const uint32_t* __restrict__ cand, uint64_t count,
                       const uint32_t* __restrict__ codes, int32_t nw, int32_t s_begin, int32_t n,
                       int32_t d, uint32_t* __restrict__ out, uint64_t cap,
                       unsigned long long* __restrict__ out_count,
                       unsigned long long* __restrict__ visits) {
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    const uint64_t first = static_cast<uint64_t>(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u);
    unsigned long long seen = 0;
    for (uint64_t k0 = first; k0 < count; k0 += step) {
        const uint64_t k = k0 + lane_id();
        bool alive = k < count;
        const uint32_t x = alive ? cand[k] : 0u;
        for (int32_t s = s_begin; s < n; ++s) {
            const uint64_t live = ballot(alive);
            if (!live) break;
            seen += static_cast<unsigned long long>(__builtin_popcountll(live));
            // Wave-uniform row: scalar loads, 16 window codes per request.
            cu32* w = (cu32*)(codes + static_cast<int64_t>(s) * nw);
            uint32_t best = 32u;
            int32_t j = 0;
            for (; j + 16 <= nw; j += 16) {
                uint32_t c[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) c[u] = w[j + u];
#pragma unroll
                for (int u = 0; u < 16; ++u) best = min(best, digit_mismatches(x, c[u]));
            }
            for (; j < nw; ++j) best = min(best, digit_mismatches(x, w[j]));
            alive = alive && best <= static_cast<uint32_t>(d);
        }
        const uint64_t pass = ballot(alive);
        if (pass) {
            unsigned long long base = 0;
            if (lane_id() == 0)
                base = atomicAdd(out_count, static_cast<unsigned long long>(__builtin_popcountll(pass)));
            base = uni64(base);
            if (alive) {
                const uint64_t at = base + rank_below(pass);
                if (at < cap) out[at] = x;
            }
        }
    }
    if (lane_id() == 0 && seen) atomicAdd(visits, seen);
}

namespace pms {

hipError_t launch_nbhd_verify(const uint32_t* cand, uint64_t count, const uint32_t* codes,
                              int32_t nw, int32_t s_begin, int32_t n, int32_t d, uint32_t* out,
                              uint64_t cap, unsigned long long* out_count,
                              unsigned long long* visits, uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL(pms_nbhd_verify_kernel, dim3(grid), dim3(256), 0, stream, cand, count,
                       codes, nw, s_begin, n, d, out, cap, out_count, visits);
    return hipGetLastError();
}

hipError_t launch_nbhd_codes(const uint8_t* seqs, int32_t t, int32_t l, int32_t rows,
                             uint32_t* codes, hipStream_t stream) {
    const int32_t nw = t - l + 1;
    const int64_t total = static_cast<int64_t>(rows) * nw;
    if (total <= 0) return hipSuccess;
    const uint32_t blocks = static_cast<uint32_t>((total + 255) / 256);
    hipLaunchKernelGGL(pms_nbhd_codes_kernel, dim3(blocks), dim3(256), 0, stream, seqs, t, l, nw,
                       rows, codes);
    return hipGetLastError();
}

hipError_t launch_nbhd_zero(uint32_t* p, uint64_t words, uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL(pms_nbhd_zero_kernel, dim3(grid), dim3(256), 0, stream,
                       reinterpret_cast<uint4*>(p), words / 4);
    return hipGetLastError();
}

hipError_t launch_nbhd_scatter(const uint32_t* codes, int32_t nw, const uint32_t* deltas,
                               int32_t nd, uint32_t* bitmap, unsigned long long* fresh,
                               uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL(pms_nbhd_scatter_kernel, dim3(grid), dim3(256), 0, stream, codes, nw,
                       deltas, nd, bitmap, fresh);
    return hipGetLastError();
}

hipError_t launch_nbhd_and(uint32_t* m, const uint32_t* b, uint64_t words,
                           unsigned long long* count, uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL(pms_nbhd_and_kernel, dim3(grid), dim3(256), 0, stream,
                       reinterpret_cast<uint4*>(m), reinterpret_cast<const uint4*>(b), words / 4,
                       count);
    return hipGetLastError();
}

hipError_t launch_nbhd_collect(const uint32_t* m, uint64_t words, uint32_t* out, uint64_t cap,
                               unsigned long long* count, uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL(pms_nbhd_collect_kernel, dim3(grid), dim3(256), 0, stream,
                       reinterpret_cast<const uint4*>(m), words / 4, out, cap, count);
    return hipGetLastError();
}

}  // namespace pms
