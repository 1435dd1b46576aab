// pms_probe.hip -- VALU issue-rate probe used to state the integer roofline.
//
// Every lane runs 16 independent dependency chains of one instruction kind
// for `iters` iterations; with enough resident waves the SIMDs never wait on
// a dependency, so lane-operations per second is the achievable issue rate
// of that instruction.  Each wave also reads the shader-clock counter
// (s_memtime) and the 100 MHz real-time counter (s_memrealtime) around its
// loop, which gives the engine clock during the run.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pms.h"
#include "pms_internal.h"

namespace {

#define CHAIN16(STMT) \
    STMT(x0) STMT(x1) STMT(x2) STMT(x3) STMT(x4) STMT(x5) STMT(x6) STMT(x7) \
    STMT(x8) STMT(x9) STMT(x10) STMT(x11) STMT(x12) STMT(x13) STMT(x14) STMT(x15)

#define OP_XOR(x) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(x) : "s"(c));
#define OP_BCNT(x) asm volatile("v_bcnt_u32_b32 %0, %0, %1" : "+v"(x) : "s"(c));
#define OP_MIN3(x) asm volatile("v_min3_u32 %0, %0, %1, %2" : "+v"(x) : "v"(y), "s"(c));
#define OP_SDWA(x) asm volatile( \
    "v_or_b32_sdwa %0, %0, %0 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:WORD_0" \
    : "+v"(x));
#define OP_ADD(x) asm volatile("v_add_u32 %0, %1, %0" : "+v"(x) : "s"(c));
#define OP_FMA(x) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x) : "v"(y), "s"(c));
#define OP_XORVV(x) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(x) : "v"(y));
// One window compare of the search loop on an independent chain: the
// candidate register is re-derived from the chain so nothing can be hoisted.
#define OP_CMP(x)                                                                          \
    {                                                                                      \
        uint32_t t_;                                                                       \
        asm volatile("v_xor_b32 %0, %1, %2" : "=v"(t_) : "s"(c), "v"(x));                 \
        asm volatile("v_or_b32_sdwa %0, %0, %0 dst_sel:DWORD dst_unused:UNUSED_PAD "        \
                     "src0_sel:WORD_1 src1_sel:WORD_0" : "+v"(t_));                        \
        asm volatile("v_bcnt_u32_b32 %0, %0, 0" : "+v"(t_));                               \
        asm volatile("v_min3_u32 %0, %0, %1, %2" : "+v"(x) : "v"(t_), "v"(y));             \
    }

// Moves from scalar registers (wave-uniform values copied into VGPRs): one
// 32-bit move, or one 64-bit move of an SGPR pair, into 16 destinations.
#define MOV16(D, INSN, CONS, SRC)                                                  \
    asm volatile(INSN " %0, %1" : "=v"(D##0) : CONS(SRC));                        \
    asm volatile(INSN " %0, %1" : "=v"(D##1) : CONS(SRC));                        \
    asm volatile(INSN " %0, %1" : "=v"(D##2) : CONS(SRC));                        \
    asm volatile(INSN " %0, %1" : "=v"(D##3) : CONS(SRC));                        \
    asm volatile(INSN " %0, %1" : "=v"(D##4) : CONS(SRC));                        \
    asm volatile(INSN " %0, %1" : "=v"(D##5) : CONS(SRC));                        \
    asm volatile(INSN " %0, %1" : "=v"(D##6) : CONS(SRC));                        \
    asm volatile(INSN " %0, %1" : "=v"(D##7) : CONS(SRC));                        \
    asm volatile(INSN " %0, %1" : "=v"(D##8) : CONS(SRC));                        \
    asm volatile(INSN " %0, %1" : "=v"(D##9) : CONS(SRC));                        \
    asm volatile(INSN " %0, %1" : "=v"(D##10) : CONS(SRC));                       \
    asm volatile(INSN " %0, %1" : "=v"(D##11) : CONS(SRC));                       \
    asm volatile(INSN " %0, %1" : "=v"(D##12) : CONS(SRC));                       \
    asm volatile(INSN " %0, %1" : "=v"(D##13) : CONS(SRC));                       \
    asm volatile(INSN " %0, %1" : "=v"(D##14) : CONS(SRC));                       \
    asm volatile(INSN " %0, %1" : "=v"(D##15) : CONS(SRC));
#define SCON(v) "s"(v)

template <int OP>
__global__ void __launch_bounds__(256) valu_probe_kernel(uint32_t* __restrict__ sink,
                                                         uint32_t iters, uint32_t c,
                                                         uint64_t* __restrict__ clocks) {
    uint32_t x0 = threadIdx.x, x1 = x0 + 1, x2 = x0 + 2, x3 = x0 + 3, x4 = x0 + 4, x5 = x0 + 5,
             x6 = x0 + 6, x7 = x0 + 7, x8 = x0 + 8, x9 = x0 + 9, x10 = x0 + 10, x11 = x0 + 11,
             x12 = x0 + 12, x13 = x0 + 13, x14 = x0 + 14, x15 = x0 + 15;
    const uint32_t y = blockIdx.x;
    uint64_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0, q5 = 0, q6 = 0, q7 = 0, q8 = 0, q9 = 0,
             q10 = 0, q11 = 0, q12 = 0, q13 = 0, q14 = 0, q15 = 0;
    const uint64_t c64 = (static_cast<uint64_t>(c) << 32) | (c ^ 0xffffu);
    const uint64_t c0 = __builtin_amdgcn_s_memtime();
    const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
    for (uint32_t i = 0; i < iters; ++i) {
        if (OP == 8) { MOV16(x, "v_mov_b32", SCON, c + i) }
        if (OP == 9) { MOV16(q, "v_mov_b64", SCON, c64 + i) }
        if (OP == 0) { CHAIN16(OP_XOR) }
        if (OP == 1) { CHAIN16(OP_BCNT) }
        if (OP == 2) { CHAIN16(OP_MIN3) }
        if (OP == 3) { CHAIN16(OP_SDWA) }
        if (OP == 4) { CHAIN16(OP_ADD) }
        if (OP == 5) { CHAIN16(OP_FMA) }
        if (OP == 6) { CHAIN16(OP_XORVV) }
        if (OP == 7) { CHAIN16(OP_CMP) }
    }
    const uint64_t c1 = __builtin_amdgcn_s_memtime();
    const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
    const uint64_t qa = q0 ^ q1 ^ q2 ^ q3 ^ q4 ^ q5 ^ q6 ^ q7 ^ q8 ^ q9 ^ q10 ^ q11 ^ q12 ^ q13 ^
                        q14 ^ q15;
    const uint32_t acc = x0 ^ x1 ^ x2 ^ x3 ^ x4 ^ x5 ^ x6 ^ x7 ^ x8 ^ x9 ^ x10 ^ x11 ^ x12 ^
                         x13 ^ x14 ^ x15 ^ static_cast<uint32_t>(qa) ^ static_cast<uint32_t>(qa >> 32);
    sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        clocks[0] = c1 - c0;
        clocks[1] = r1 - r0;
    }
}

template <int OP>
hipError_t launch_probe(uint32_t blocks, uint32_t iters, uint32_t* sink, uint64_t* clocks,
                        hipStream_t s) {
    hipLaunchKernelGGL(valu_probe_kernel<OP>, dim3(blocks), dim3(256), 0, s, sink, iters,
                       0x5bd1e995u, clocks);
    return hipGetLastError();
}

}  // namespace

namespace pms {

hipError_t valu_probe(int op, uint32_t blocks, uint32_t iters, uint32_t* sink, uint64_t* clocks,
                      hipStream_t s) {
    switch (op) {
        case PMS_PROBE_XOR: return launch_probe<0>(blocks, iters, sink, clocks, s);
        case PMS_PROBE_BCNT: return launch_probe<1>(blocks, iters, sink, clocks, s);
        case PMS_PROBE_MIN3: return launch_probe<2>(blocks, iters, sink, clocks, s);
        case PMS_PROBE_OR_SDWA: return launch_probe<3>(blocks, iters, sink, clocks, s);
        case PMS_PROBE_ADD: return launch_probe<4>(blocks, iters, sink, clocks, s);
        case PMS_PROBE_FMA_F32: return launch_probe<5>(blocks, iters, sink, clocks, s);
        case PMS_PROBE_XOR_VV: return launch_probe<6>(blocks, iters, sink, clocks, s);
        case PMS_PROBE_COMPARE: return launch_probe<7>(blocks, iters, sink, clocks, s);
        case PMS_PROBE_MOV_S: return launch_probe<8>(blocks, iters, sink, clocks, s);
        case PMS_PROBE_MOV64_S: return launch_probe<9>(blocks, iters, sink, clocks, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pms
