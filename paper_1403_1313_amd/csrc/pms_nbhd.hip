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
//   pms_nbhd_rec_*_kernel    (window, mask group) records by destination tile
//   pms_nbhd_tile_kernel     one sequence's pass: bit (w ^ delta) of B for every
//                            window w and mask delta, tile by tile in LDS, and
//                            M = B or M &= B for each tile, counting the bits
//   pms_nbhd_zero_kernel,    the same pass for few bits: zero B, set its bits
//   pms_nbhd_scatter_kernel, with global atomics (counting the fresh ones on
//   pms_nbhd_and_kernel      the first sequence), then M &= B
//   pms_nbhd_collect_kernel  motif codes of the set bits of M (one global
//                            atomicAdd per workgroup)
//   pms_nbhd_verify_kernel,  once few candidates are left, checks them against
//   pms_nbhd_verify_lds_     the remaining sequences directly (the rows' codes
//   kernel, ..._lds4_kernel  staged in LDS when they fit; one or four lanes
//                            per survivor)
//
// Bound: a tiled pass sets nw x |Ball| bits with LDS atomics and streams M
// once in and once out (16-byte vectors); a scatter pass issues nw x |Ball|
// global atomics and streams the maps three times; collection streams M once.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

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

// A bitmap pass takes one of two forms, whichever the host's cost model
// finds cheaper for the sequence: the tiled pass (every bit set in LDS, the
// map streamed once or twice) when there are many bits per tile, or the
// scatter pass (zero B, set its bits with global atomics, M &= B) when there
// are few.

// Counts of a pass are summed per workgroup (four wavefronts) into
// part[blockIdx.x] and then by pms_nbhd_sum_kernel: an atomic per wavefront
// on one counter serialises when there are tens of thousands of them.
__device__ __forceinline__ void block_count(uint32_t v, uint32_t* __restrict__ part) {
    __shared__ uint32_t wsum[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane_id() == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// *total = part[0] + ... + part[n-1] (one workgroup of 1024 threads).
extern "C" __global__ void __launch_bounds__(1024)
pms_nbhd_sum_kernel(const uint32_t* __restrict__ part, uint32_t n,
                    unsigned long long* __restrict__ total) {
    __shared__ unsigned long long wsum[16];
    unsigned long long v = 0;
    for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) v += part[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane_id() == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < 16; ++w) t += wsum[w];
        *total = t;
    }
}

// Zeroes `vecs` 16-byte vectors.
extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_zero_kernel(uint4* __restrict__ p, uint64_t vecs) {
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t k = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < vecs; k += step)
        p[k] = make_uint4(0u, 0u, 0u, 0u);
}

// Every (window, mask) pair of one row: a grid-stride loop over the pairs,
// mask index fastest, so a wavefront reads consecutive masks and one window.
// `fresh` (optional) receives per workgroup the bits this pass set that
// were clear, from the values the atomics return.
extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_scatter_kernel(const uint32_t* __restrict__ codes, int32_t nw,
                        const uint32_t* __restrict__ deltas, int32_t nd,
                        uint32_t* __restrict__ bitmap, uint32_t* __restrict__ fresh) {
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
    if (fresh) block_count(set, fresh);
}

// M &= B over `vecs` 16-byte vectors; `part` receives per workgroup the
// bits left.
extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_and_kernel(uint4* __restrict__ m, const uint4* __restrict__ b, uint64_t vecs,
                    uint32_t* __restrict__ part) {
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
    block_count(bits, part);
}

// A record: window index in the low 17 bits (t <= 2^17), mask group above.
constexpr uint32_t kRecGroupShift = 17;
constexpr uint32_t kRecWindowMask = (1u << kRecGroupShift) - 1u;

// Records of a tiled pass: every (window j, non-empty mask group h) pair
// belongs to tile (w_j >> T) ^ h.  With records a tile reads its own pairs
// instead of looking up every window's group, which pays when there are
// many more tiles than groups per window (l = 16: 16384 tiles, 585 windows,
// about a thousand non-empty groups).  Count per tile, exclusive scan, fill.
extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_rec_count_kernel(const uint32_t* __restrict__ codes, int32_t nw,
                          const uint32_t* __restrict__ ne, int32_t nne, int32_t T,
                          uint32_t* __restrict__ tcount) {
    const uint64_t total = static_cast<uint64_t>(nw) * static_cast<uint64_t>(nne);
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += step) {
        const uint32_t j = static_cast<uint32_t>(i / static_cast<uint64_t>(nne));
        const uint32_t k = static_cast<uint32_t>(i - static_cast<uint64_t>(j) * nne);
        atomicAdd(tcount + ((codes[j] >> T) ^ ne[k]), 1u);
    }
}

// Exclusive scan of tiles (<= 16384) counts into toff[0 .. tiles], one
// workgroup of 1024 threads; tcur (tiles words) is cleared for the fill.
extern "C" __global__ void __launch_bounds__(1024)
pms_nbhd_rec_scan_kernel(const uint32_t* __restrict__ tcount, uint32_t tiles,
                         uint32_t* __restrict__ toff, uint32_t* __restrict__ tcur) {
    __shared__ uint32_t wsum[16];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint32_t per = (tiles + 1023u) / 1024u;
    const uint32_t e0 = tid * per;
    uint32_t mine = 0;
    for (uint32_t e = e0; e < e0 + per && e < tiles; ++e) mine += tcount[e];
    uint32_t incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= static_cast<uint32_t>(off)) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (uint32_t w = 0; w < 16; ++w) {
        before += w < wave ? wsum[w] : 0u;
        total += wsum[w];
    }
    uint32_t run = before + incl - mine;
    for (uint32_t e = e0; e < e0 + per && e < tiles; ++e) {
        toff[e] = run;
        run += tcount[e];
        tcur[e] = 0u;
    }
    if (tid == 0) toff[tiles] = total;
}

extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_rec_fill_kernel(const uint32_t* __restrict__ codes, int32_t nw,
                         const uint32_t* __restrict__ ne, int32_t nne, int32_t T,
                         const uint32_t* __restrict__ toff, uint32_t* __restrict__ tcur,
                         uint32_t* __restrict__ rec) {
    const uint64_t total = static_cast<uint64_t>(nw) * static_cast<uint64_t>(nne);
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += step) {
        const uint32_t j = static_cast<uint32_t>(i / static_cast<uint64_t>(nne));
        const uint32_t k = static_cast<uint32_t>(i - static_cast<uint64_t>(j) * nne);
        const uint32_t h = ne[k];
        const uint32_t tile = (codes[j] >> T) ^ h;
        rec[toff[tile] + atomicAdd(tcur + tile, 1u)] = j | (h << kRecGroupShift);
    }
}

// One bitmap pass by tiles: workgroup g builds in LDS the bits
// [g 2^T, (g+1) 2^T) of B, the union of the sequence's window balls, then
// writes that tile of M as B (first sequence) or M & B, counting the bits it
// keeps into tile_bits[g].  Every bit is set with an LDS atomic; HBM
// sees one read and one write of M per pass.
//
// The ball's masks are sorted by their bits above T, group h holding
// deltas[group_off[h] .. group_off[h+1]), so the masks that take window w into
// tile g are group (w >> T) ^ g, at most 2^T of them.  Windows are taken
// kTileChunk at a time; an LDS prefix sum numbers their (window, mask) pairs
// (at most kTileChunk x 2^T < 2^32) and each thread takes an equal run.
// LDS: tile_words + 3 kTileChunk + 1 + kTileThreads words.
constexpr int kTileChunk = 1024;
#ifndef PMS_TILE_THREADS
#define PMS_TILE_THREADS 256
#endif
constexpr int kTileThreads = PMS_TILE_THREADS;
constexpr int kScanPer = kTileChunk / kTileThreads;   // prefix entries per thread
constexpr int kPartPer = kTileThreads / 64;           // thread sums per lane of the scan
constexpr int kPairUnroll = 4;                        // mask loads in flight per lane

extern "C" __global__ void __launch_bounds__(kTileThreads)
pms_nbhd_tile_kernel(const uint32_t* __restrict__ codes, int32_t nw,
                     const uint32_t* __restrict__ deltas, const uint32_t* __restrict__ group_off,
                     const uint32_t* __restrict__ rec, const uint32_t* __restrict__ rec_off,
                     int32_t T, uint32_t tile_words, uint4* __restrict__ m, int32_t first,
                     uint32_t* __restrict__ tile_bits) {
    extern __shared__ uint32_t lds[];
    uint32_t* const tile = lds;
    uint32_t* const pre = tile + tile_words;         // kTileChunk + 1: pairs before window j
    uint32_t* const beg = pre + kTileChunk + 1;      // kTileChunk: first mask of window j's group
    uint32_t* const win = beg + kTileChunk;          // kTileChunk: window codes
    uint32_t* const part = win + kTileChunk;         // kTileThreads: per-thread sums of the scan
    const uint32_t g = blockIdx.x;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t low = (1u << T) - 1u;
    // Items: the tile's records (window, group) when given, else every
    // window with its group (w >> T) ^ g.
    const uint32_t ibase = rec ? rec_off[g] : 0u;
    const int32_t nitems = rec ? static_cast<int32_t>(rec_off[g + 1] - ibase) : nw;
    for (uint32_t k = tid; k < tile_words; k += nt) tile[k] = 0u;
    for (int32_t c0 = 0; c0 < nitems; c0 += kTileChunk) {
        const uint32_t cn = static_cast<uint32_t>(min(kTileChunk, nitems - c0));
        __syncthreads();  // the tile is clear and the last chunk's pairs are done
        for (uint32_t j = tid; j < cn; j += nt) {
            uint32_t w, h;
            if (rec) {
                const uint32_t r = rec[ibase + c0 + j];
                w = codes[r & kRecWindowMask];
                h = r >> kRecGroupShift;
            } else {
                w = codes[c0 + j];
                h = (w >> T) ^ g;
            }
            const uint32_t lo = group_off[h];
            win[j] = w;
            beg[j] = lo;
            pre[j + 1] = group_off[h + 1] - lo;
        }
        __syncthreads();
        // Inclusive scan of pre[1 .. cn]: thread t sums its kScanPer entries,
        // the first wavefront scans the thread sums (kPartPer per lane), and
        // each thread adds its offset to its entries.
        const uint32_t e0 = kScanPer * tid + 1;
        uint32_t run = 0;
        for (uint32_t j = e0; j < e0 + kScanPer && j <= cn; ++j) run += pre[j];
        part[tid] = run;
        __syncthreads();
        if (tid < 64) {
            uint32_t v[kPartPer], sum = 0;
#pragma unroll
            for (int u = 0; u < kPartPer; ++u) {
                v[u] = part[kPartPer * tid + u];
                sum += v[u];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off, 64);
                if (static_cast<int>(tid) >= off) incl += y;
            }
            uint32_t base = incl - sum;
#pragma unroll
            for (int u = 0; u < kPartPer; ++u) {
                part[kPartPer * tid + u] = base;
                base += v[u];
            }
        }
        __syncthreads();
        {
            uint32_t acc = part[tid];
            for (uint32_t j = e0; j < e0 + kScanPer && j <= cn; ++j) {
                acc += pre[j];
                pre[j] = acc;
            }
        }
        if (tid == 0) pre[0] = 0u;
        __syncthreads();
        const uint32_t total = pre[cn];
        const uint32_t p0 = static_cast<uint32_t>(static_cast<uint64_t>(total) * tid / nt);
        const uint32_t p1 = static_cast<uint32_t>(static_cast<uint64_t>(total) * (tid + 1) / nt);
        if (p0 < p1) {
            // Each thread takes one run of pairs, so the lanes of a
            // wavefront work on different windows and their LDS atomics
            // rarely meet in one word; kPairUnroll mask loads are in flight.
            // j(q), the last j with pre[j] <= q, only grows along the run
            // (walking window by window instead, each lane with its own
            // segment lengths, diverged and was slower).
            uint32_t lo = 0, hi = cn;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (pre[mid] <= p0) lo = mid; else hi = mid;
            }
            uint32_t j = lo;
            for (uint32_t q0 = p0; q0 < p1; q0 += kPairUnroll) {
                uint32_t wv[kPairUnroll], dv[kPairUnroll];
#pragma unroll
                for (int u = 0; u < kPairUnroll; ++u) {
                    const uint32_t q = q0 + u;
                    if (q < p1) {
                        while (pre[j + 1] <= q) ++j;
                        wv[u] = win[j];
                        dv[u] = deltas[beg[j] + (q - pre[j])];
                    }
                }
#pragma unroll
                for (int u = 0; u < kPairUnroll; ++u) {
                    if (q0 + u < p1) {
                        const uint32_t x = (wv[u] ^ dv[u]) & low;
                        atomicOr(tile + (x >> 5), 1u << (x & 31u));
                    }
                }
            }
        }
    }
    __syncthreads();
    const uint32_t vecs = tile_words / 4;
    uint4* const out = m + static_cast<uint64_t>(g) * vecs;
    const uint4* const tv = reinterpret_cast<const uint4*>(tile);
    uint32_t bits = 0;
    for (uint32_t k = tid; k < vecs; k += nt) {
        uint4 v = tv[k];
        if (!first) {
            const uint4 o = out[k];
            v = make_uint4(v.x & o.x, v.y & o.y, v.z & o.z, v.w & o.w);
        }
        out[k] = v;
        bits += static_cast<uint32_t>(__builtin_popcount(v.x) + __builtin_popcount(v.y) +
                                      __builtin_popcount(v.z) + __builtin_popcount(v.w));
    }
    block_count(bits, tile_bits);
}

// Codes of the set bits of M (`vecs` 16-byte vectors), unsorted, at most
// `cap` written; *count receives the number of set bits.  Workgroup g takes
// one contiguous share of M and reads it twice: first it counts the share's
// bits and reserves room for all of them with a single atomic, then it
// writes them, each batch of kCollectBatch vectors per thread placed by a
// workgroup-wide scan of the threads' counts.  One atomic per workgroup
// (a counter shared by every wavefront of the grid serialised the earlier
// one-atomic-per-round form when the bits were many and sparse).
constexpr int kCollectBatch = 8;

__device__ __forceinline__ uint32_t popc4(const uint4& v) {
    return static_cast<uint32_t>(__builtin_popcount(v.x) + __builtin_popcount(v.y) +
                                 __builtin_popcount(v.z) + __builtin_popcount(v.w));
}

extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_collect_kernel(const uint4* __restrict__ m, uint64_t vecs, uint32_t* __restrict__ out,
                        uint64_t cap, unsigned long long* __restrict__ count) {
    __shared__ uint32_t wtot[4];
    __shared__ unsigned long long base_s;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    constexpr uint32_t kSpan = 256u * kCollectBatch;
    const uint64_t per = (vecs + gridDim.x - 1) / gridDim.x;
    const uint64_t lo = static_cast<uint64_t>(blockIdx.x) * per;
    const uint64_t hi = lo + per < vecs ? lo + per : vecs;
    // Count the share's bits, kCollectBatch loads in flight per thread.
    uint32_t bits = 0;
    for (uint64_t k0 = lo; k0 < hi; k0 += kSpan) {
        uint4 x[kCollectBatch];
#pragma unroll
        for (int u = 0; u < kCollectBatch; ++u) {
            const uint64_t k = k0 + u * 256u + tid;
            x[u] = k < hi ? m[k] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < kCollectBatch; ++u) bits += popc4(x[u]);
    }
    uint32_t wsum = bits;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off, 64);
    if (lane == 0) wtot[wave] = wsum;
    __syncthreads();
    if (tid == 0) {
        const unsigned long long total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
        base_s = total ? atomicAdd(count, total) : 0ull;
        wtot[0] = static_cast<uint32_t>(total != 0);
    }
    __syncthreads();
    if (!wtot[0]) return;
    uint64_t run = base_s;
    __syncthreads();
    // Write them: per batch, thread t's bits go after those of threads < t.
    for (uint64_t k0 = lo; k0 < hi; k0 += kSpan) {
        uint4 x[kCollectBatch];
#pragma unroll
        for (int u = 0; u < kCollectBatch; ++u) {
            const uint64_t k = k0 + u * 256u + tid;
            x[u] = k < hi ? m[k] : make_uint4(0u, 0u, 0u, 0u);
        }
        uint32_t mine = 0;
#pragma unroll
        for (int u = 0; u < kCollectBatch; ++u) mine += popc4(x[u]);
        uint32_t incl = mine;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t v = __shfl_up(incl, off, 64);
            if (lane >= static_cast<uint32_t>(off)) incl += v;
        }
        if (lane == 63) wtot[wave] = incl;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (uint32_t w = 0; w < 4; ++w) {
            const uint32_t t = wtot[w];
            before += w < wave ? t : 0u;
            total += t;
        }
        __syncthreads();   // wtot is rewritten by the next batch
        if (!total) continue;
        uint64_t at = run + before + (incl - mine);
#pragma unroll
        for (int u = 0; u < kCollectBatch; ++u) {
            const uint64_t k = k0 + u * 256u + tid;
            const uint32_t w4[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                for (uint32_t v = w4[e]; v; v &= v - 1, ++at)
                    if (at < cap) out[at] = static_cast<uint32_t>((4 * k + e) * 32 + __builtin_ctz(v));
            }
        }
        run += total;
    }
}

// Survivors of the bitmap passes checked against sequences s_begin .. n-1
// directly: lane k takes survivor k; the wavefront scans one sequence at a
// time (window codes wave-uniform), a lane whose smallest distance exceeds d
// drops out, and the wavefront stops at the first sequence no lane passes
// (the enhanced rule of Section III.A).  A wavefront with a lane that keeps
// passing scans every remaining sequence, so the kernel's time is that
// chain's: when the remaining rows' codes fit in kVerifyLdsBytes of LDS each
// workgroup stages them once (rows padded to a multiple of 4 windows with
// window 0, which cannot change a minimum) and the scan reads 4 codes per
// LDS load, 16 in flight, with four lanes per survivor (each a quarter of
// the windows) while survivors are few; otherwise the codes come through
// the scalar data cache, 16 per load.  Distance of codes x, w: the 2-bit
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

constexpr size_t kVerifyLdsBytes = 48 * 1024;
constexpr uint64_t kVerifyQuadMax = 3u << 16;   // survivors checked four lanes each

template <int kLanes>
__device__ __forceinline__ void verify_lds(const uint32_t* __restrict__ cand, uint64_t count,
                           const uint32_t* __restrict__ codes, int32_t nw, int32_t nw_pad,
                           int32_t s_begin, int32_t n, int32_t d, uint32_t* __restrict__ out,
                           uint64_t cap, unsigned long long* __restrict__ out_count,
                           unsigned long long* __restrict__ visits) {
    extern __shared__ uint4 rows4[];
    uint32_t* const rows = reinterpret_cast<uint32_t*>(rows4);
    const int32_t nrows = n - s_begin;
    for (int32_t k = threadIdx.x; k < nrows * nw_pad; k += blockDim.x) {
        const int32_t r = k / nw_pad, j = k - r * nw_pad;
        rows[k] = codes[static_cast<int64_t>(s_begin + r) * nw + (j < nw ? j : 0)];
    }
    __syncthreads();
    // kLanes lanes per survivor (1 or 4), each taking every kLanes-th group
    // of 4 windows, so one survivor's scan is 1/kLanes as long; the minima
    // meet by shuffles.  A wavefront holds 64 / kLanes survivors.
    const int32_t nq = nw_pad / 4;
    const uint32_t lane = lane_id(), part = lane & static_cast<uint32_t>(kLanes - 1);
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x / kLanes;
    const uint64_t first = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u)) / kLanes;
    // lane kLanes * i speaks for survivor i
    constexpr uint64_t kLeaders = kLanes == 4 ? 0x1111111111111111ull : ~0ull;
    unsigned long long seen = 0;
    for (uint64_t k0 = first; k0 < count; k0 += step) {
        const uint64_t k = k0 + lane / kLanes;
        bool alive = k < count;
        const uint32_t x = alive ? cand[k] : 0u;
        for (int32_t s = s_begin; s < n; ++s) {
            const uint64_t live = ballot(alive);
            if (!live) break;
            seen += static_cast<unsigned long long>(__builtin_popcountll(live & kLeaders));
            const uint4* w4 = rows4 + static_cast<int64_t>(s - s_begin) * nq;
            uint32_t best = 32u;
            int32_t q = static_cast<int32_t>(part);
            for (; q + 3 * kLanes < nq; q += 4 * kLanes) {
                uint4 c[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) c[u] = w4[q + kLanes * u];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    best = min(best, digit_mismatches(x, c[u].x));
                    best = min(best, digit_mismatches(x, c[u].y));
                    best = min(best, digit_mismatches(x, c[u].z));
                    best = min(best, digit_mismatches(x, c[u].w));
                }
            }
            for (; q < nq; q += kLanes) {
                const uint4 c = w4[q];
                best = min(best, digit_mismatches(x, c.x));
                best = min(best, digit_mismatches(x, c.y));
                best = min(best, digit_mismatches(x, c.z));
                best = min(best, digit_mismatches(x, c.w));
            }
            if constexpr (kLanes == 4) {
                best = min(best, static_cast<uint32_t>(__shfl_xor(static_cast<int>(best), 1, 64)));
                best = min(best, static_cast<uint32_t>(__shfl_xor(static_cast<int>(best), 2, 64)));
            }
            alive = alive && best <= static_cast<uint32_t>(d);
        }
        const bool lead = alive && part == 0u;
        const uint64_t pass = ballot(lead);
        if (pass) {
            unsigned long long base = 0;
            if (lane == 0)
                base = atomicAdd(out_count, static_cast<unsigned long long>(__builtin_popcountll(pass)));
            base = uni64(base);
            if (lead) {
                const uint64_t at = base + rank_below(pass);
                if (at < cap) out[at] = x;
            }
        }
    }
    if (lane == 0 && seen) atomicAdd(visits, seen);
}

extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_verify_lds_kernel(const uint32_t* __restrict__ cand, uint64_t count,
                           const uint32_t* __restrict__ codes, int32_t nw, int32_t nw_pad,
                           int32_t s_begin, int32_t n, int32_t d, uint32_t* __restrict__ out,
                           uint64_t cap, unsigned long long* __restrict__ out_count,
                           unsigned long long* __restrict__ visits) {
    verify_lds<1>(cand, count, codes, nw, nw_pad, s_begin, n, d, out, cap, out_count, visits);
}

extern "C" __global__ void __launch_bounds__(256)
pms_nbhd_verify_lds4_kernel(const uint32_t* __restrict__ cand, uint64_t count,
                            const uint32_t* __restrict__ codes, int32_t nw, int32_t nw_pad,
                            int32_t s_begin, int32_t n, int32_t d, uint32_t* __restrict__ out,
                            uint64_t cap, unsigned long long* __restrict__ out_count,
                            unsigned long long* __restrict__ visits) {
    verify_lds<4>(cand, count, codes, nw, nw_pad, s_begin, n, d, out, cap, out_count, visits);
}

namespace pms {

hipError_t launch_nbhd_verify(const uint32_t* cand, uint64_t count, const uint32_t* codes,
                              int32_t nw, int32_t s_begin, int32_t n, int32_t d, uint32_t* out,
                              uint64_t cap, unsigned long long* out_count,
                              unsigned long long* visits, uint32_t grid, hipStream_t stream) {
    // No more workgroups than survivors need (one lane each): idle ones
    // would only be launched and retired (and, below, stage rows for nothing).
    const uint64_t need_lds = (count * 4 + 255) / 256;   // four lanes per survivor
    const uint64_t need = (count + 255) / 256;
    const uint32_t blocks = static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(grid, need)));
    const int32_t nw_pad = (nw + 3) & ~3;
    const size_t lds = static_cast<size_t>(n - s_begin) * nw_pad * sizeof(uint32_t);
    // Four lanes per survivor while survivors are few enough that a lane
    // each would leave the device idle; beyond that every workgroup would
    // stage the rows for a quarter as many survivors.
    if (n > s_begin && lds <= kVerifyLdsBytes && count <= kVerifyQuadMax)
        hipLaunchKernelGGL(pms_nbhd_verify_lds4_kernel,
                           dim3(static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(grid, need_lds)))),
                           dim3(256), lds, stream, cand,
                           count, codes, nw, nw_pad, s_begin, n, d, out, cap, out_count, visits);
    else if (n > s_begin && lds <= kVerifyLdsBytes)
        hipLaunchKernelGGL(pms_nbhd_verify_lds_kernel, dim3(blocks), dim3(256), lds, stream, cand,
                           count, codes, nw, nw_pad, s_begin, n, d, out, cap, out_count, visits);
    else
        hipLaunchKernelGGL(pms_nbhd_verify_kernel, dim3(blocks), dim3(256), 0, stream, cand, count,
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
                               int32_t nd, uint32_t* bitmap, uint32_t* fresh,
                               uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL(pms_nbhd_scatter_kernel, dim3(grid), dim3(256), 0, stream, codes, nw,
                       deltas, nd, bitmap, fresh);
    return hipGetLastError();
}

hipError_t launch_nbhd_and(uint32_t* m, const uint32_t* b, uint64_t words,
                           uint32_t* part, uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL(pms_nbhd_and_kernel, dim3(grid), dim3(256), 0, stream,
                       reinterpret_cast<uint4*>(m), reinterpret_cast<const uint4*>(b), words / 4,
                       part);
    return hipGetLastError();
}

hipError_t launch_nbhd_sum(const uint32_t* part, uint32_t n, unsigned long long* total,
                           hipStream_t stream) {
    hipLaunchKernelGGL(pms_nbhd_sum_kernel, dim3(1), dim3(1024), 0, stream, part, n, total);
    return hipGetLastError();
}

size_t nbhd_tile_lds_bytes(uint32_t tile_words) {
    return (static_cast<size_t>(tile_words) + 3 * kTileChunk + 1 + kTileThreads) * sizeof(uint32_t);
}

hipError_t launch_nbhd_tile(const uint32_t* codes, int32_t nw, const uint32_t* deltas,
                            const uint32_t* group_off, const uint32_t* rec,
                            const uint32_t* rec_off, int32_t T, uint32_t tiles,
                            uint32_t tile_words, uint32_t* m, bool first,
                            uint32_t* part, hipStream_t stream) {
    hipLaunchKernelGGL(pms_nbhd_tile_kernel, dim3(tiles), dim3(kTileThreads),
                       nbhd_tile_lds_bytes(tile_words), stream, codes, nw, deltas, group_off, rec,
                       rec_off, T, tile_words, reinterpret_cast<uint4*>(m), first ? 1 : 0, part);
    return hipGetLastError();
}

hipError_t launch_nbhd_records(const uint32_t* codes, int32_t nw, const uint32_t* ne, int32_t nne,
                               int32_t T, uint32_t tiles, uint32_t* tcount, uint32_t* toff,
                               uint32_t* tcur, uint32_t* rec, uint32_t grid, hipStream_t stream) {
    hipError_t e = launch_fill(tcount, tiles, 0u, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pms_nbhd_rec_count_kernel, dim3(grid), dim3(256), 0, stream, codes, nw, ne,
                       nne, T, tcount);
    hipLaunchKernelGGL(pms_nbhd_rec_scan_kernel, dim3(1), dim3(1024), 0, stream, tcount, tiles, toff,
                       tcur);
    hipLaunchKernelGGL(pms_nbhd_rec_fill_kernel, dim3(grid), dim3(256), 0, stream, codes, nw, ne,
                       nne, T, toff, tcur, rec);
    return hipGetLastError();
}

hipError_t launch_nbhd_collect(const uint32_t* m, uint64_t words, uint32_t* out, uint64_t cap,
                               unsigned long long* count, uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL(pms_nbhd_collect_kernel, dim3(grid), dim3(256), 0, stream,
                       reinterpret_cast<const uint4*>(m), words / 4, out, cap, count);
    return hipGetLastError();
}

}  // namespace pms
