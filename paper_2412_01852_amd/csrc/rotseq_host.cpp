// Host runtime of librotseq: argument checks, dispatch, the cached device
// workspace and the C ABI declared in include/rotseq.h.
#include "rotseq.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "rotseq_internal.h"

namespace rotseq {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool make_plan(Plan &p, int req_band)
{
    int band = req_band;
    if (band == 0) {
        band = 1;
        while (band < 16 && band < p.k)
            band *= 2;
    }
    if (band != 1 && band != 2 && band != 4 && band != 8 && band != 16)
        return false;
    p.band = band;
    p.npass = (int)((p.k + band - 1) / band);
    p.unroll = unroll_for_band(band);
    const int64_t real_steps = p.n + band - 1;  // t = 0 .. n+K-2
    p.steps = (int)(((real_steps + p.unroll - 1) / p.unroll) * p.unroll);
    const int64_t n1 = p.n - 1;
    size_t off = 0;
    p.off_coef = off;
    off = align256(off + (size_t)p.npass * p.steps * band * 2 * p.esize);
    p.off_negmask = off;
    off = align256(off + (size_t)p.npass * n1 * sizeof(uint64_t));
    p.off_parity = off;
    off = align256(off + (size_t)(p.npass + 1) * n1);
    p.off_sign = off;
    off = align256(off + (size_t)p.n * p.esize);
    p.total = off;
    return true;
}

namespace {

int check_args(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda, const void *C,
               int64_t ldc, const void *S, int64_t lds)
{
    if (m < 0)
        return -1;
    if (n < 0)
        return -2;
    if (k < 0)
        return -3;
    const bool work = m > 0 && n > 1 && k > 0;
    const int64_t n1 = n > 1 ? n - 1 : 1;
    if (work && A == nullptr)
        return -4;
    if (lda < (m > 1 ? m : 1))
        return -5;
    if (work && C == nullptr)
        return -6;
    if (ldc < n1)
        return -7;
    if (work && S == nullptr)
        return -8;
    if (lds < n1)
        return -9;
    return 0;
}

// One growable device buffer per (device, stream).  Growing waits for the
// stream so the old buffer is no longer in use when it is freed.
struct Pool {
    std::mutex mu;
    std::map<std::pair<int, hipStream_t>, std::pair<void *, size_t>> bufs;

    int get(hipStream_t stream, size_t bytes, void **out)
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess)
            return ROTSEQ_E_HIP;
        std::lock_guard<std::mutex> lock(mu);
        auto &slot = bufs[std::make_pair(dev, stream)];
        if (slot.second < bytes) {
            if (slot.first) {
                if (hipStreamSynchronize(stream) != hipSuccess)
                    return ROTSEQ_E_HIP;
                (void)hipFree(slot.first);
                slot.first = nullptr;
                slot.second = 0;
            }
            size_t want = bytes + bytes / 4;
            void *p = nullptr;
            if (hipMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                return ROTSEQ_E_NOMEM;
            }
            slot.first = p;
            slot.second = want;
        }
        *out = slot.first;
        return ROTSEQ_SUCCESS;
    }
};

Pool &pool()
{
    static Pool *p = new Pool();  // never destroyed: device memory is released at process exit
    return *p;
}

// Event-based kernel timing (rotseq_profile_*).
struct Profiler {
    std::atomic<bool> on{false};
    std::mutex mu;
    struct Rec {
        hipEvent_t e0, e1, e2;
    };
    std::vector<Rec> pending;
    rotseq_profile acc{};

    bool begin(Rec &r, hipStream_t st)
    {
        if (!on.load(std::memory_order_relaxed))
            return false;
        if (hipEventCreate(&r.e0) != hipSuccess)
            return false;
        (void)hipEventCreate(&r.e1);
        (void)hipEventCreate(&r.e2);
        (void)hipEventRecord(r.e0, st);
        return true;
    }
    void finish(const Rec &r)
    {
        std::lock_guard<std::mutex> lock(mu);
        pending.push_back(r);
    }
    int read(rotseq_profile *out, int reset)
    {
        std::lock_guard<std::mutex> lock(mu);
        int rc = ROTSEQ_SUCCESS;
        for (const Rec &r : pending) {
            float a = 0.f, b = 0.f;
            if (hipEventSynchronize(r.e2) != hipSuccess ||
                hipEventElapsedTime(&a, r.e0, r.e1) != hipSuccess ||
                hipEventElapsedTime(&b, r.e1, r.e2) != hipSuccess)
                rc = ROTSEQ_E_HIP;
            acc.prep_ms += a;
            acc.sweep_ms += b;
            acc.sweep_ms_min = acc.calls ? std::min(acc.sweep_ms_min, (double)b) : b;
            acc.sweep_ms_max = acc.calls ? std::max(acc.sweep_ms_max, (double)b) : b;
            acc.calls += 1;
            (void)hipEventDestroy(r.e0);
            (void)hipEventDestroy(r.e1);
            (void)hipEventDestroy(r.e2);
        }
        pending.clear();
        if (out)
            *out = acc;
        if (reset)
            acc = rotseq_profile{};
        return rc;
    }
};

Profiler &profiler()
{
    static Profiler *p = new Profiler();
    return *p;
}

bool resolve(const rotseq_opts *opts, int &arith, int &band)
{
    arith = opts ? opts->arith : 0;
    band = opts ? opts->band : 0;
    const int kernel = opts ? opts->kernel : 0;
    if (arith == ROTSEQ_ARITH_AUTO)
        arith = kLift;
    if (arith != kExact && arith != kFma && arith != kLift)
        return false;
    if (kernel != ROTSEQ_KERNEL_AUTO && kernel != ROTSEQ_KERNEL_MULTIPASS)
        return false;
    return true;
}

bool plan_for(Plan &p, int esize, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldc,
              int64_t lds, const rotseq_opts *opts)
{
    int arith = 0, band = 0;
    if (!resolve(opts, arith, band))
        return false;
    p = Plan{};
    p.m = m;
    p.n = n;
    p.k = k;
    p.lda = lda;
    p.ldc = ldc;
    p.lds = lds;
    p.arith = arith;
    p.esize = esize;
    return make_plan(p, band);
}

template <typename T>
int run(int64_t m, int64_t n, int64_t k, T *A, int64_t lda, const T *C, int64_t ldc, const T *S,
        int64_t lds, hipStream_t stream, const rotseq_opts *opts, void *ws, size_t ws_bytes)
{
    const int bad = check_args(m, n, k, A, lda, C, ldc, S, lds);
    if (bad)
        return bad;
    if (m == 0 || n <= 1 || k == 0)
        return ROTSEQ_SUCCESS;
    Plan p;
    if (!plan_for(p, (int)sizeof(T), m, n, k, lda, ldc, lds, opts))
        return ROTSEQ_E_UNSUPPORTED;
    if (n > INT32_MAX - 64 || p.steps <= 0)
        return ROTSEQ_E_UNSUPPORTED;
    if (ws) {
        if (ws_bytes < p.total || ((uintptr_t)ws & 255) != 0)
            return ROTSEQ_E_WORKSPACE;
    } else {
        const int rc = pool().get(stream, p.total, &ws);
        if (rc)
            return rc;
    }
    Profiler::Rec rec{};
    const bool timed = profiler().begin(rec, stream);
    if (launch_prep(p, C, S, ws, stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (timed)
        (void)hipEventRecord(rec.e1, stream);
    if (launch_sweep(p, A, ws, stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (timed) {
        (void)hipEventRecord(rec.e2, stream);
        profiler().finish(rec);
    }
    return ROTSEQ_SUCCESS;
}

}  // namespace
}  // namespace rotseq

using namespace rotseq;

extern "C" {

int rotseq_check_args(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda, const void *C,
                      int64_t ldc, const void *S, int64_t lds)
{
    return check_args(m, n, k, A, lda, C, ldc, S, lds);
}

size_t rotseq_workspace_bytes(char dtype, int64_t m, int64_t n, int64_t k, const rotseq_opts *opts)
{
    int esize = dtype == 'd' ? 8 : dtype == 's' ? 4 : 0;
    if (!esize || m <= 0 || n <= 1 || k <= 0)
        return 0;
    Plan p;
    const int64_t n1 = n - 1;
    if (!plan_for(p, esize, m, n, k, m, n1, n1, opts))
        return 0;
    return p.total;
}

int rotseq_ex_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda, const double *C,
                int64_t ldc, const double *S, int64_t lds, hipStream_t stream,
                const rotseq_opts *opts, void *workspace, size_t ws_bytes)
{
    return run<double>(m, n, k, A, lda, C, ldc, S, lds, stream, opts, workspace, ws_bytes);
}

int rotseq_ex_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda, const float *C,
                int64_t ldc, const float *S, int64_t lds, hipStream_t stream,
                const rotseq_opts *opts, void *workspace, size_t ws_bytes)
{
    return run<float>(m, n, k, A, lda, C, ldc, S, lds, stream, opts, workspace, ws_bytes);
}

int rotseq_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda, const double *C, int64_t ldc,
             const double *S, int64_t lds, hipStream_t stream)
{
    return run<double>(m, n, k, A, lda, C, ldc, S, lds, stream, nullptr, nullptr, 0);
}

int rotseq_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda, const float *C, int64_t ldc,
             const float *S, int64_t lds, hipStream_t stream)
{
    return run<float>(m, n, k, A, lda, C, ldc, S, lds, stream, nullptr, nullptr, 0);
}

const char *rotseq_strerror(int code)
{
    if (code < 0)
        return "invalid argument (the code is minus its 1-based position)";
    switch (code) {
    case ROTSEQ_SUCCESS: return "success";
    case ROTSEQ_E_HIP: return "HIP runtime call failed";
    case ROTSEQ_E_NOMEM: return "device workspace allocation failed";
    case ROTSEQ_E_WORKSPACE: return "caller workspace too small or not 256-byte aligned";
    case ROTSEQ_E_UNSUPPORTED: return "unsupported option combination";
    case ROTSEQ_E_TIMEOUT: return "device-side wait exceeded its spin limit";
    default: return "unknown error code";
    }
}

int rotseq_version(void) { return 100; }

int rotseq_profile_enable(int on)
{
    profiler().on.store(on != 0);
    return ROTSEQ_SUCCESS;
}

int rotseq_profile_read(rotseq_profile *out, int reset) { return profiler().read(out, reset); }

}  // extern "C"
