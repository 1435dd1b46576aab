// pms_noalloc.hip -- the fixed device scratch of pms_solve_dev_noalloc and
// the two small kernels that fill and read it.
//
// pms_solve_dev needs device memory beyond its inputs and outputs: the window
// table, the per-call records (instance, state, counters, window jobs, work
// items) and the stage-queue workspace of the search kernel.  It allocates
// them once and reuses them.  pms_solve_dev_noalloc takes all of it from one
// array of fixed size instead, so a caller that cannot allocate (graph
// capture, a serving loop) can still run a solve.  The host never writes the
// records: pms_noalloc_setup_kernel builds them on the device from the call's
// scalars, which also clears everything the search expects to start at zero.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pms.h"
#include "pms_internal.h"

// One array per device, held until the process ends.  Host code must not
// pass `scratch` itself to a kernel (it names a host-side stand-in): the
// device address comes from hipGetSymbolAddress in pms::noalloc_scratch.
static __device__ __align__(256) uint32_t scratch[PMS_NOALLOC_SCRATCH_BYTES / sizeof(uint32_t)];

// Writes the records of one instance at the offsets in `lay`: the instance
// record, its state (items_left = number of items), zeroed counters and
// bad-byte flag, one window job per row, and the work items.  Items are the
// ones the host planner would make for a launch of this one instance: `size`
// candidates each up to the first item that starts at or past head_end, then
// `small` candidates each; the last of either kind is cut at 4^l.
extern "C" __global__ void __launch_bounds__(256)
pms_noalloc_setup_kernel(uint8_t* __restrict__ base, pms::NoallocLayout lay, uint32_t* dev_out,
                         uint64_t capacity) {
    const uint64_t total = 1ull << (2 * lay.l);
    const uint64_t h = lay.n_head * lay.size < total ? lay.n_head * lay.size : total;
    const uint32_t rows = static_cast<uint32_t>(lay.n);
    const uint32_t span = rows > lay.n_items ? rows : lay.n_items;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid == 0) {
        pms_dev_instance* in = reinterpret_cast<pms_dev_instance*>(base + lay.off_inst);
        in->windows = reinterpret_cast<const uint32_t*>(base + lay.off_win);
        in->out = dev_out;
        in->out_cap = capacity;
        in->n = lay.n;
        in->nw_stride = lay.stride;
        in->l = lay.l;
        in->d = lay.d;
        pms_dev_state* st = reinterpret_cast<pms_dev_state*>(base + lay.off_state);
        st->count = 0;
        st->visits = 0;
        st->t_done = 0;
        st->items_left = lay.n_items;
        st->reserved = 0;
        pms_dev_counters* ctr = reinterpret_cast<pms_dev_counters*>(base + lay.off_ctr);
        ctr->next_item = 0;
        ctr->error = 0;
        ctr->batches = 0;
        ctr->t_start = 0;
        ctr->single_batches = 0;
        ctr->filtered_batches = 0;
        ctr->filtered_groups = 0;
        *reinterpret_cast<uint32_t*>(base + lay.off_bad) = 0;
    }
    for (uint32_t i = tid; i < span; i += gridDim.x * blockDim.x) {
        if (i < rows) {
            pms_win_job* job = reinterpret_cast<pms_win_job*>(base + lay.off_jobs) + i;
            job->src_off = static_cast<uint64_t>(i) * static_cast<uint64_t>(lay.t);
            job->dst_off = static_cast<uint64_t>(i) * static_cast<uint64_t>(lay.stride);
            job->t = lay.t;
            job->l = lay.l;
            job->stride = lay.stride;
            job->inst = 0;
            job->layout = lay.layout;
            job->flags = 0;
        }
        if (i < lay.n_items) {
            const uint64_t begin = i < lay.n_head ? static_cast<uint64_t>(i) * lay.size
                                                  : h + static_cast<uint64_t>(i - lay.n_head) * lay.small;
            const uint64_t step = i < lay.n_head ? lay.size : lay.small;
            const uint64_t len = total - begin < step ? total - begin : step;
            pms_work_item* w = reinterpret_cast<pms_work_item*>(base + lay.off_work) + i;
            w->begin = begin;
            w->len = static_cast<uint32_t>(len);
            w->inst = 0;
        }
    }
}

// *dev_count = the instance's motif count.
extern "C" __global__ void pms_noalloc_count_kernel(const pms_dev_state* __restrict__ st,
                                                    uint64_t* __restrict__ dev_count) {
    if (threadIdx.x == 0) *dev_count = st->count;
}

namespace pms {

hipError_t noalloc_scratch(void** ptr, size_t* bytes) {
    *ptr = nullptr;
    *bytes = 0;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    *ptr = p;
    *bytes = sizeof(scratch);
    return hipSuccess;
}

hipError_t launch_noalloc_setup(void* base, const NoallocLayout& lay, uint32_t* dev_out,
                                uint64_t capacity, hipStream_t stream) {
    const uint32_t span = static_cast<uint32_t>(lay.n) > lay.n_items ? static_cast<uint32_t>(lay.n)
                                                                     : lay.n_items;
    const uint32_t want = (span + 255u) / 256u + 1u;
    const uint32_t blocks = want < 1024u ? want : 1024u;
    hipLaunchKernelGGL(pms_noalloc_setup_kernel, dim3(blocks), dim3(256), 0, stream,
                       static_cast<uint8_t*>(base), lay, dev_out, capacity);
    return hipGetLastError();
}

hipError_t launch_noalloc_count(const pms_dev_state* st, uint64_t* dev_count, hipStream_t stream) {
    hipLaunchKernelGGL(pms_noalloc_count_kernel, dim3(1), dim3(64), 0, stream, st, dev_count);
    return hipGetLastError();
}

}  // namespace pms
