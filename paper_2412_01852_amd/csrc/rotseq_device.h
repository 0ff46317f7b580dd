// Device-side helpers shared by the sweep kernels of librotseq (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rotseq.h"
#include "rotseq_internal.h"

namespace rotseq {
namespace dev {

constexpr int kWave = 64;
// Dword 3 of a gfx9-family buffer descriptor: 32-bit data format, no swizzle.
constexpr int kRsrcWord3 = 0x00020000;
// Cache-policy bits of buffer accesses: SC0 makes a load miss in the CU's
// L1; SC1 (device scope) makes a load or store coherent across the CUs and
// XCDs of the device (stores are written through to memory).
constexpr int kPolicyL2 = 1;
constexpr int kPolicyDevice = 16;

template <typename T>
struct CoefPair {
    T a, b;
};

// Address space 4 (constant): wave-uniform loads through these pointers
// become scalar loads into SGPRs.
template <typename T>
using ConstPairs = const __attribute__((address_space(4))) CoefPair<T> *;
template <typename T>
using ConstScalars = const __attribute__((address_space(4))) T *;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(uint64_t base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, bytes, kRsrcWord3);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <int POLICY>
__device__ __forceinline__ double buf_load(double, __amdgpu_buffer_rsrc_t r, int voff)
{
    u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, POLICY);
    return __builtin_bit_cast(double, v);
}
template <int POLICY>
__device__ __forceinline__ float buf_load(float, __amdgpu_buffer_rsrc_t r, int voff)
{
    unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, POLICY);
    return __builtin_bit_cast(float, v);
}
template <int POLICY = 0>
__device__ __forceinline__ void buf_store(double x, __amdgpu_buffer_rsrc_t r, int voff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, voff, 0, POLICY);
}
template <int POLICY = 0>
__device__ __forceinline__ void buf_store(float x, __amdgpu_buffer_rsrc_t r, int voff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, voff, 0, POLICY);
}

// s_waitcnt immediate (gfx9 encoding) that waits until at most `n` vector
// memory operations of this wave are outstanding; LGKM and EXP not waited.
// Vector memory operations complete in issue order, so this guarantees
// that every operation except the last `n` has completed.
template <int N>
__device__ __forceinline__ void wait_vmem_at_most()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Keeps a running scalar value opaque to loop strength reduction, which
// would otherwise turn each unrolled step's address into its own 64-bit
// induction variable and exhaust the SGPR file.  Emits no instruction.
__device__ __forceinline__ void opaque(uint64_t &x) { asm volatile("" : "+s"(x)); }

// Compiler-only ordering point: memory operations are not moved across it.
// The lockstep barrier of the chain kernel puts one on each side of its
// LDS wait and s_barrier, so no LDS access of a group moves past them.
__device__ __forceinline__ void compiler_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Keeps a running scalar counter opaque to the optimiser (see opaque()).
__device__ __forceinline__ void opaque_i(int &x) { asm volatile("" : "+s"(x)); }

// Which wait gave up, recorded in bits 8.. of the status word beside
// ROTSEQ_E_TIMEOUT: the device-scope flag between workgroups.
constexpr int kWaitFlag = 1 << 10;

__device__ __forceinline__ void record_timeout(int *status, int kind)
{
    __hip_atomic_fetch_or(status, ROTSEQ_E_TIMEOUT | kind, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// End of a lockstep group: this wave's LDS accesses have completed (LGKM
// count 0; vector memory is not waited for), then all waves of the
// workgroup meet.  The compiler fences keep LDS accesses on their side.
__device__ __forceinline__ void group_barrier()
{
    compiler_fence();
    __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8));  // lgkmcnt(0) only
    __builtin_amdgcn_s_barrier();
    compiler_fence();
}

// `groups` lockstep groups without work.
__device__ __forceinline__ void idle_groups(int groups)
{
    for (int i = 0; i < groups; ++i)
        group_barrier();
}

// Bounded waits: after a timeout `limit` drops to 0, so the wave never waits
// again and the grid drains within one time-out per wave; the kind of wait
// that gave up is collected in `timed_out` and written to the status word
// once, when the wave ends (a memory write inside the step loop would make
// the compiler drain every outstanding vector memory operation at each wait
// site).
// Waits until the device-scope progress counter exceeds `need` (polls cost
// a memory round trip, so they get a sixteenth of the LDS budget).
__device__ __forceinline__ int wait_flag(int *p, int need, int &limit, int &timed_out)
{
    int v = uniform(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    for (int polls = 0; v <= need; ++polls) {
        if (polls >= (limit >> 4)) {
            timed_out |= kWaitFlag;
            limit = 0;
            return 0x7fffffff;
        }
        __builtin_amdgcn_s_sleep(2);
        v = uniform(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    return v;
}

__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// One rotation of the entries (x, y) of a row; (a, b) as prepared by the
// coefficient kernel: (c, s) for kExact/kFma, (s'/(1+c'), -s') for kLift.
template <int ARITH, typename T>
__device__ __forceinline__ void rotate(T &x, T &y, T a, T b)
{
    if constexpr (ARITH == kExact) {
        // Algorithm 1 as written: every product and sum rounded separately.
#pragma clang fp contract(off)
        T t = a * x + b * y;
        y = -b * x + a * y;
        x = t;
    } else if constexpr (ARITH == kFma) {
        T t = fmad(a, x, b * y);
        y = fmad(a, y, -(b * x));
        x = t;
    } else {
        x = fmad(a, y, x);
        y = fmad(b, x, y);
        x = fmad(a, y, x);
    }
}

}  // namespace dev
}  // namespace rotseq
