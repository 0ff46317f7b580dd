// rotseq_noalloc_d: the plain FP64 call with its workspace in a fixed,
// file-scope device array instead of the library's allocated pool, for
// callers that cannot allocate device memory.  The C ABI is declared in
// include/rotseq.h.
//
// Layout of `scratch` on each device: bytes [0, 256) hold the sticky error
// word of this entry point's sweeps (int at offset 0), and bytes
// [256, 256 + workspace) the workspace of one call: coefficient records,
// lifting signs and negation masks (rewritten by the preparation kernels of
// every call) and the chain kernel's progress flags (zeroed by a kernel of
// every call).  Every call on a device shares that device's array, so calls
// that overlap on one device race.
#include "rotseq.h"

#include <hip/hip_runtime.h>

#include <mutex>

#include "rotseq_internal.h"

namespace rotseq {

// Status word, then one call's workspace; 128 MiB covers m = n = 10240
// with k up to about 360 (k = 192 needs 71 MB with the window matrices of
// the matrix-instruction sweep).
constexpr size_t kScratchHead = 256;
constexpr size_t kScratchBytes = (size_t)128 << 20;

namespace {

static __device__ __align__(256) char scratch[kScratchBytes];

__global__ void clear_words(int *p, int count)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < count)
        p[i] = 0;
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_scratch[kMaxDevices];  // device address of `scratch`, per device

// The current device's address of `scratch` (host code never uses the
// symbol itself, which is a host-side stand-in).  Taken once per device with
// that device current; the status word is cleared by a kernel on `stream`
// at the same time.
int scratch_of(int dev, hipStream_t stream, char **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return ROTSEQ_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return ROTSEQ_E_HIP;
        }
        clear_words<<<1, 64, 0, stream>>>((int *)p, (int)(kScratchHead / sizeof(int)));
        if (hipGetLastError() != hipSuccess)
            return ROTSEQ_E_HIP;
        g_scratch[dev] = (char *)p;
    }
    *out = g_scratch[dev];
    return ROTSEQ_SUCCESS;
}

}  // namespace

int noalloc_status(int reset, int *value)
{
    *value = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return ROTSEQ_E_HIP;
    char *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (dev >= 0 && dev < kMaxDevices)
            base = g_scratch[dev];
    }
    if (base == nullptr)  // the entry point never ran on this device
        return ROTSEQ_SUCCESS;
    if (hipMemcpy(value, base, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (reset && hipMemset(base, 0, sizeof(int)) != hipSuccess)
        return ROTSEQ_E_HIP;
    return ROTSEQ_SUCCESS;
}

}  // namespace rotseq

using namespace rotseq;

extern "C" int rotseq_noalloc_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda,
                                const double *C, int64_t ldc, const double *S, int64_t lds,
                                hipStream_t stream)
{
    const int bad = check_problem(m, n, k, A, lda, C, ldc, S, lds);
    if (bad)
        return bad;
    if (m == 0 || n <= 1 || k == 0)
        return ROTSEQ_SUCCESS;
    Plan p{};
    p.m = m;
    p.n = n;
    p.k = k;
    p.lda = lda;
    p.ldc = ldc;
    p.lds = lds;
    p.cstep = 1;
    p.arith = kLift;
    p.kind = kRotate;
    p.esize = (int)sizeof(double);
    // The same plan as rotseq_d: forward right application of rotations in
    // FP64 with automatic arithmetic, so the matrix sweep is eligible.
    const bool mfma_ok = (uint64_t)lda * 8u * 9u < ((uint64_t)1 << 30);
    if (!make_plan(p, 0, 0, mfma_ok) || p.n > INT32_MAX - 64 || (p.kernel != kMfma && p.steps <= 0))
        return ROTSEQ_E_UNSUPPORTED;
    if (p.total > kScratchBytes - kScratchHead)
        return ROTSEQ_E_TOO_LARGE;
    if (configure_launch(p, 0, 0) != hipSuccess)
        return ROTSEQ_E_HIP;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return ROTSEQ_E_HIP;
    char *base = nullptr;
    if (const int rc = scratch_of(dev, stream, &base))
        return rc;
    p.status = (int *)base;
    void *ws = base + kScratchHead;
    if (launch_prep(p, C, S, ws, stream) != hipSuccess || launch_sweep(p, A, ws, stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    return ROTSEQ_SUCCESS;
}
