// Measured FP64 ceilings of the device (rotseq_fp64_ceiling): how fast the
// CUs issue FP64 fused multiply-adds in the forms the sweep kernels use, how
// fast they issue FP64 matrix instructions, whether the two overlap, and at
// which shader clock.  These figures decide between the vector sweep and a
// variant that accumulates rotations into small dense blocks and multiplies
// them with matrix instructions (the paper's GEMM-based alternative,
// Section 8).
//
// Each wave runs kChains independent dependency chains for `iters`
// iterations; every chain keeps its operands in registers, so nothing but
// the arithmetic is timed.  Wave 0 of every workgroup reads the shader-cycle
// counter (s_memtime) and the 100 MHz real-time counter (s_memrealtime) at
// its start and end; their ratio is the average shader clock.
#include <hip/hip_runtime.h>

#include <vector>

#include "rotseq.h"

namespace rotseq {
namespace {

constexpr int kChains = 8;

typedef double f64x4 __attribute__((ext_vector_type(4)));

enum CeilMode : int { kValu = 1, kValuDpp = 2, kMfma = 3, kMixed = 4, kMfmaLds = 5 };

constexpr int kLdsSlots = 8;  // doubles per lane of the LDS traffic in kMfmaLds

// 8 independent FMA chains: x_i += a * y_i, four iterations per trip.
__device__ __forceinline__ void valu_chains(double (&x)[kChains], double a, const double (&y)[kChains],
                                            int64_t iters)
{
    for (int64_t it = 0; it < iters; it += 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            asm volatile(
                "v_fmac_f64 %0, %8, %9\n v_fmac_f64 %1, %8, %10\n v_fmac_f64 %2, %8, %11\n"
                " v_fmac_f64 %3, %8, %12\n v_fmac_f64 %4, %8, %13\n v_fmac_f64 %5, %8, %14\n"
                " v_fmac_f64 %6, %8, %15\n v_fmac_f64 %7, %8, %16\n"
                : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]),
                  "+v"(x[7])
                : "v"(a), "v"(y[0]), "v"(y[1]), "v"(y[2]), "v"(y[3]), "v"(y[4]), "v"(y[5]), "v"(y[6]),
                  "v"(y[7]));
    }
}

// The same with the multiplier broadcast from lane 3 of each 16-lane row
// (DPP row_newbcast), as the rotation sweep reads its coefficients.  `a` is
// written once before the loop, so the DPP read never follows a VALU write.
__device__ __forceinline__ void valu_dpp_chains(double (&x)[kChains], double a, const double (&y)[kChains],
                                                int64_t iters)
{
#define ROTSEQ_DPPF(X, Y) "v_fmac_f64_dpp %" #X ", %8, %" #Y " row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
    for (int64_t it = 0; it < iters; it += 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            asm volatile(ROTSEQ_DPPF(0, 9) ROTSEQ_DPPF(1, 10) ROTSEQ_DPPF(2, 11) ROTSEQ_DPPF(3, 12)
                             ROTSEQ_DPPF(4, 13) ROTSEQ_DPPF(5, 14) ROTSEQ_DPPF(6, 15) ROTSEQ_DPPF(7, 16)
                         : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]),
                           "+v"(x[6]), "+v"(x[7])
                         : "v"(a), "v"(y[0]), "v"(y[1]), "v"(y[2]), "v"(y[3]), "v"(y[4]), "v"(y[5]),
                           "v"(y[6]), "v"(y[7]));
    }
#undef ROTSEQ_DPPF
}

// 8 independent accumulators of v_mfma_f64_16x16x4f64 (2048 flops each).
__device__ __forceinline__ double mfma_chains(double a, double b, int64_t iters)
{
    f64x4 acc[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i)
        acc[i] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int64_t it = 0; it < iters; it += 2) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int i = 0; i < kChains; ++i)
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kChains; ++i)
        s += acc[i].x + acc[i].y + acc[i].z + acc[i].w;
    return s;
}

// As mfma_chains, with the LDS traffic an MFMA sweep would add: every 8
// matrix instructions, 8 doubles per lane written to and read back from
// LDS, the values read feeding the next group's B operands.
__device__ __forceinline__ double mfma_lds_chains(double a, double b, int64_t iters, double *lds)
{
    const int lane = threadIdx.x & 63;
    // volatile: every write and read-back reaches LDS
    typedef __attribute__((address_space(3))) volatile double lds_f64;
    lds_f64 *mine = (lds_f64 *)(__attribute__((address_space(3))) double *)lds +
                    (threadIdx.x >> 6) * 64 * kLdsSlots + lane;
    f64x4 acc[kChains];
    double bb[kLdsSlots];
#pragma unroll
    for (int i = 0; i < kChains; ++i)
        acc[i] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < kLdsSlots; ++i)
        bb[i] = b + i;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i)
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb[i], acc[i], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < kLdsSlots; ++i)
            mine[i * 64] = acc[i].x;
#pragma unroll
        for (int i = 0; i < kLdsSlots; ++i)
            bb[i] = mine[((i + 1) % kLdsSlots) * 64];
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kChains; ++i)
        s += acc[i].x + acc[i].y + acc[i].z + acc[i].w;
    return s;
}

template <int MODE>
__global__ __launch_bounds__(1024) void fp64_ceiling(int64_t iters, double *sink,
                                                      unsigned long long *clk)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    unsigned long long c0 = 0, r0 = 0;
    if (wave == 0) {
        c0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
    }
    const double a = 1.0 + 1e-9 * lane;
    double x[kChains], y[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        x[i] = 1e-3 * (i + 1);
        y[i] = 1e-12 * (lane + i);
    }
    // Waves 4g..4g+3 land on the four SIMDs of the CU; in the mixed mode
    // every SIMD gets both kinds (groups alternate).
    const bool mfma = MODE == kMfma || MODE == kMfmaLds || (MODE == kMixed && ((wave >> 2) & 1));
    double s = 0.0;
    if (MODE == kMfmaLds) {
        extern __shared__ double ceil_lds[];
        s = mfma_lds_chains(a, y[1], iters, ceil_lds);
    } else if (mfma) {
        s = mfma_chains(a, y[1], iters);
    } else {
        // two wait states between the VALU write of `a` and its first DPP read
        asm volatile("s_nop 1");
        if (MODE == kValu)
            valu_chains(x, a, y, iters);
        else
            valu_dpp_chains(x, a, y, iters);
#pragma unroll
        for (int i = 0; i < kChains; ++i)
            s += x[i];
    }
    __syncthreads();
    if (wave == 0 && lane == 0) {
        clk[2 * blockIdx.x] = __builtin_amdgcn_s_memtime() - c0;
        clk[2 * blockIdx.x + 1] = __builtin_amdgcn_s_memrealtime() - r0;
    }
    if (s == 12345.678)  // never true; keeps the chains live
        sink[threadIdx.x] = s;
}

}  // namespace
}  // namespace rotseq

using namespace rotseq;

extern "C" int rotseq_fp64_ceiling(int32_t mode, int32_t waves, int64_t iters,
                                   rotseq_ceiling_result *out)
{
    if (mode < kValu || mode > kMfmaLds)
        return -1;
    if (waves < 1 || waves > 16 || (mode == kMixed && waves % 8 != 0))
        return -2;
    if (iters < 4 || iters % 4 != 0)
        return -3;
    if (out == nullptr)
        return -4;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return ROTSEQ_E_HIP;
    double *sink = nullptr;
    unsigned long long *clk = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ROTSEQ_SUCCESS;
    if (hipMalloc(&sink, 1024 * sizeof(double)) != hipSuccess ||
        hipMalloc(&clk, 2 * (size_t)cus * sizeof(unsigned long long)) != hipSuccess)
        rc = ROTSEQ_E_NOMEM;
    if (!rc && (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = ROTSEQ_E_HIP;
    if (!rc) {
        const dim3 grid((unsigned)cus), block((unsigned)(waves * 64));
        (void)hipEventRecord(e0, st);
        switch (mode) {
        case kValu: fp64_ceiling<kValu><<<grid, block, 0, st>>>(iters, sink, clk); break;
        case kValuDpp: fp64_ceiling<kValuDpp><<<grid, block, 0, st>>>(iters, sink, clk); break;
        case kMfma: fp64_ceiling<kMfma><<<grid, block, 0, st>>>(iters, sink, clk); break;
        case kMfmaLds:
            fp64_ceiling<kMfmaLds><<<grid, block, (size_t)waves * 64 * kLdsSlots * sizeof(double), st>>>(
                iters, sink, clk);
            break;
        default: fp64_ceiling<kMixed><<<grid, block, 0, st>>>(iters, sink, clk); break;
        }
        if (hipGetLastError() != hipSuccess)
            rc = ROTSEQ_E_HIP;
        (void)hipEventRecord(e1, st);
    }
    float ms = 0.f;
    std::vector<unsigned long long> h(2 * (size_t)cus, 0);
    if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
                hipMemcpy(h.data(), clk, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) !=
                    hipSuccess))
        rc = ROTSEQ_E_HIP;
    if (!rc) {
        double cyc = 0.0, real = 0.0;
        for (int i = 0; i < cus; ++i) {
            cyc += (double)h[2 * i];
            real += (double)h[2 * i + 1];
        }
        const double n_mfma_waves = mode == kMfma || mode == kMfmaLds ? waves : mode == kMixed ? waves / 2 : 0;
        const double n_valu_waves = waves - n_mfma_waves;
        *out = rotseq_ceiling_result{};
        out->ms = ms;
        out->valu_flops = (double)cus * n_valu_waves * 64.0 * kChains * (double)iters * 2.0;
        out->mfma_flops = (double)cus * n_mfma_waves * kChains * (double)iters * 2048.0;
        out->clock_mhz = real > 0.0 ? 100.0 * cyc / real : 0.0;
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (st)
        (void)hipStreamDestroy(st);
    if (sink)
        (void)hipFree(sink);
    if (clk)
        (void)hipFree(clk);
    return rc;
}
