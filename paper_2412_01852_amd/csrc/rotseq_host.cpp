// Host runtime of librotseq: argument checks, dispatch, the cached device
// workspace and the C ABI declared in include/rotseq.h.
#include "rotseq.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "rotseq_internal.h"
#include "rotseq_refl3.h"

namespace rotseq {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

namespace {
constexpr int kDefaultSpinLimit = 1 << 22;
std::atomic<int> g_spin_limit{kDefaultSpinLimit};
std::atomic<int> g_wait_bias{0};
}  // namespace

int wait_spin_limit() { return g_spin_limit.load(std::memory_order_relaxed); }
int wait_bias() { return g_wait_bias.load(std::memory_order_relaxed); }

namespace {

// Windows per band of the matrix-instruction sweep: steps 0 .. n+6 in
// windows of 8 steps.
int64_t mfma_windows(int64_t n) { return (n + 7) / 8; }

// Workspace of the matrix-instruction sweep's window matrices, for any
// bands-per-wave choice (at most 2 padded bands), and of its flags.
size_t mfma_q_bytes(int64_t n, int64_t k) { return (size_t)((k + 7) / 8 + 2) * (mfma_windows(n) + 3) * 2048; }
// One progress flag per (tile, segment), each on its own 128-byte line
// (polled by one workgroup while another writes it through every
// super-step; neighbours on one line would share that traffic).  Tiles are
// at least 2 row blocks and segments at least 4 bands.
size_t mfma_flag_bytes(int64_t m, int64_t k)
{
    return (size_t)(((m + 15) / 16 + 1) / 2) * (size_t)(((k + 7) / 8 + 3) / 4) * (size_t)kMfmaFlagStride * sizeof(int);
}

}  // namespace

// SIMDs of an MI355X (256 CUs x 4): the band rule of the chain kernel is
// shape-only, so that a plan (and its workspace size) does not depend on
// the device it is queried on.
constexpr int64_t kChainSimds = 1024;

bool make_plan(Plan &p, int req_kernel, int req_band, bool mfma_ok)
{
    // The chain kernel addresses the n column signs with 32-bit byte
    // offsets; past 2^28 columns the multipass kernel takes over.
    constexpr int64_t kChainMaxN = (int64_t)1 << 28;
    p.deep = 0;
    if (req_kernel == kMfma) {
        // Window matrices for the forward right application of rotations
        // to a column-major FP64 matrix with 32-bit column offsets per block.
        if (!mfma_ok || req_band > 0 && req_band != 8)
            return false;
        p.kernel = kMfma;
        p.band = 8;
        p.pad = 0;
        p.unroll = 4;
        p.npass = (int)((p.k + 7) / 8);
        p.steps = 0;
        p.mfma_ok = 1;
        size_t off = 0;
        p.off_coef = off;
        off = align256(off + mfma_q_bytes(p.n, p.k));
        p.off_negmask = p.off_parity = p.off_sign = off;
        p.off_flags = off;
        off = align256(off + mfma_flag_bytes(p.m, p.k));
        p.total = off;
        return true;
    }
    p.kernel = req_kernel == 0 ? (p.n <= kChainMaxN ? kChain : kMultipass) : req_kernel;
    if (p.kernel == kChain && p.n > kChainMaxN)
        return false;
    // With the automatic choice the launch may still pick the matrix
    // sweep, so the workspace covers both.
    p.mfma_ok = req_kernel == 0 && mfma_ok && p.kernel == kChain ? 1 : 0;
    int band = req_band;
    if (p.kernel == kChain) {
        // K = 8 by default.  With k <= 8 a single band of 8 would leave one
        // wave per row tile, which reads, rotates and writes every column;
        // two or more chained bands (the last ones identity rotations when
        // k is small) split the A reads and writes over two waves, which is
        // what the memory-bound regime of small k needs (32768 x 4096,
        // k = 8: 0.68 -> 0.49 ms; k = 1: 0.56 -> 0.40 ms with the
        // streaming form).  Bands of 2 halve each wave's step, which pays
        // while their waves fit one per SIMD (1024 on MI355X; 8192^2,
        // k = 8: 0.52 -> 0.39 ms) and in FP32 (32768 x 4096, k = 8:
        // 0.38 -> 0.30 ms); FP64 at 2048 waves is slower (0.41 -> 0.49 ms).
        if (band == 0) {
            const int64_t tiles = (p.m + 63) / 64;
            const int64_t waves2 = tiles * std::max<int64_t>(2, (p.k + 1) / 2);
            // FP32 with 8 < k <= 16: four bands of 4 (32768 x 4096, k = 16:
            // 0.48 -> 0.39 ms; 8192^2: 0.90 -> 0.67 ms).
            band = p.k > 16 || (p.k > 8 && p.esize == 8) ? 8
                   : p.k > 8                                ? 4
                   : (p.esize == 4 || waves2 <= kChainSimds) ? 2
                                                             : 4;
        }
        if (band != 2 && band != 4 && band != 6 && band != 8)
            return false;
    } else if (p.kernel == kMultipass) {
        if (band == 0) {
            band = 1;
            while (band < 16 && band < p.k)
                band *= 2;
        }
        if (band != 1 && band != 2 && band != 4 && band != 8 && band != 16)
            return false;
        p.unroll = unroll_for_band(band);
    } else {
        return false;
    }
    p.band = band;
    p.pad = p.kernel == kChain ? kChainCoefPad : 1;
    p.npass = (int)((p.k + band - 1) / band);
    if (p.kernel == kChain) {
        if (req_band == 0 && p.npass < 2)
            p.npass = 2;  // bands past the k-th sequence are identity
        p.unroll = chain_unroll(band, p.npass <= kChainDeepBands);
    }
    const int64_t real_steps = p.n + band - 1;  // t = 0 .. n+K-2
    p.steps = (int)(((real_steps + p.unroll - 1) / p.unroll) * p.unroll);
    const int64_t n1 = p.n - 1;
    const int64_t tiles = (p.m + 63) / 64;
    size_t off = 0;
    p.off_coef = off;
    size_t coef = (size_t)p.npass * (p.steps + p.pad) * band * 2 * p.esize;
    if (p.mfma_ok)
        coef = std::max(coef, mfma_q_bytes(p.n, p.k));
    off = align256(off + coef);
    p.off_negmask = off;
    off = align256(off + (size_t)p.npass * n1 * sizeof(uint64_t));
    p.off_parity = off;
    off = align256(off + (size_t)(p.npass + 1) * n1);
    p.off_sign = off;
    off = align256(off + (size_t)p.n * p.esize);
    p.off_flags = off;
    size_t flags = (size_t)tiles * p.npass * sizeof(int);
    if (p.mfma_ok)
        flags = std::max(flags, mfma_flag_bytes(p.m, p.k));
    off = align256(off + flags);
    p.total = off;
    return true;
}

namespace {

struct DeviceInfo {
    int cus = 0;
    size_t max_lds = 0;
    size_t lds_per_cu = 0;
};

// Attributes of the current device (cached; queries only, no allocation).
int device_info(DeviceInfo &out)
{
    static std::mutex mu;
    static std::map<int, DeviceInfo> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return ROTSEQ_E_HIP;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(dev);
    if (it == cache.end()) {
        DeviceInfo d;
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return ROTSEQ_E_HIP;
        d.cus = v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            return ROTSEQ_E_HIP;
        d.max_lds = (size_t)v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess)
            return ROTSEQ_E_HIP;
        d.lds_per_cu = (size_t)v;
        it = cache.emplace(dev, d).first;
    }
    out = it->second;
    return ROTSEQ_SUCCESS;
}

// The current device's sticky error word of the plain calls, allocated
// and zeroed on first use.
int status_word(int **out)
{
    static std::mutex mu;
    static std::map<int, int *> words;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return ROTSEQ_E_HIP;
    std::lock_guard<std::mutex> lock(mu);
    auto it = words.find(dev);
    if (it == words.end()) {
        int *w = nullptr;
        if (hipMalloc(&w, sizeof(int)) != hipSuccess) {
            (void)hipGetLastError();
            return ROTSEQ_E_NOMEM;
        }
        if (hipMemset(w, 0, sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            return ROTSEQ_E_HIP;
        it = words.emplace(dev, w).first;
    }
    *out = it->second;
    return ROTSEQ_SUCCESS;
}

}  // namespace

namespace {

// Launch shape of the matrix-instruction sweep with the smallest modelled
// time; fills the mfma_* fields, waves, nwg, lds_bytes and remap of `p`
// and returns the modelled time in seconds (or a negative value if no
// shape fits).  Model, fitted to measured sweeps of 11 problem sizes and 7
// shapes (m x n from 512^2 to 32768 x 4096, k from 1 to 192): a workgroup
// runs T super-steps one after another; in each, a SIMD issues the 16x16x4
// FP64 products of its resident waves (64 cycles each; 15% slower with one
// wave per SIMD, whose other instructions then never overlap them) plus
// about 600 cycles of everything else, 150 more per extra wave; 2.4 GHz;
// rounds of workgroups follow one another; 15 us of preparation and launch.
double mfma_step_cycles(int64_t simd_waves, int nb, int rows)
{
    const double mfma = (double)simd_waves * nb * rows * 4 * 64 * (simd_waves == 1 ? 1.15 : 1.0);
    return mfma + 600.0 + 150.0 * (double)(simd_waves - 1);
}

double plan_mfma(Plan &p, int req_waves, int req_shape, const DeviceInfo &d)
{
    static const int kShapes[][2] = {{3, 5}, {3, 4}, {3, 2}, {2, 4}, {2, 2}, {1, 4}, {1, 2}};
    const int64_t rb = (p.m + 15) / 16;
    const int64_t nbands = (p.k + 7) / 8;
    const int nwin = (int)mfma_windows(p.n);
    double best = -1.0;
    Plan keep = p;
    for (const auto &sh : kShapes) {
        const int nb = sh[0], rows = sh[1];
        if (req_shape > 0 && req_shape != 10 * nb + rows)
            continue;
        {
            const int w = mfma_waves();
            if (req_waves > 0 && w != req_waves)
                continue;
            const int64_t tiles = (rb + rows - 1) / rows;
            const int64_t nchunks = (nbands + nb - 1) / nb;
            const int64_t nseg = (nchunks + w - 1) / w;
            const int64_t nwg = tiles * nseg;
            if (nwg > INT32_MAX || nchunks * nb > nbands + 2)  // reserved window matrices
                continue;
            if ((int64_t)nb * (nwin + 3) * 2048 >= ((int64_t)1 << 31))  // a wave's window matrices
                continue;
            const size_t lds = mfma_lds_bytes(rows);
            if (lds > d.max_lds)
                continue;
            int occ = 0;
            if (mfma_occupancy(nb, rows, lds, &occ) != hipSuccess || occ < 1)
                continue;
            const int64_t slots = (int64_t)occ * d.cus;
            const int64_t rounds = (nwg + slots - 1) / slots;
            const int64_t resident = std::min<int64_t>(nwg, slots);
            const int64_t simd_waves = (resident * w + 4 * (int64_t)d.cus - 1) / (4 * (int64_t)d.cus);
            const int delay = mfma_seg_delay(nb);
            const int64_t T = 4 + (nseg - 1) * delay + (w - 1) * mfma_wave_stride(nb) + 2 * nb + nwin;
            const double cycles = (double)rounds * (double)T * mfma_step_cycles(simd_waves, nb, rows);
            const double t = cycles / 2.4e9 + 15e-6;
            if (best < 0.0 || t < best * 0.999) {
                best = t;
                keep = p;
                keep.mfma_nb = nb;
                keep.mfma_rows = rows;
                keep.mfma_nwin = nwin;
                keep.mfma_nchunks = (int)nchunks;
                keep.mfma_nseg = (int)nseg;
                keep.mfma_tiles = (int)tiles;
                keep.mfma_seg_delay = delay;
                keep.waves = w;
                keep.nwg = (int)nwg;
                keep.lds_bytes = lds;
                keep.remap = (nwg % 8 == 0 && nwg <= slots) ? 1 : 0;
            }
        }
    }
    if (best >= 0.0)
        p = keep;
    return best;
}

// Modelled time of the vector chain sweep, fitted to the same measurements:
// the slower of its arithmetic (about 44 TFLOP/s counted) and its
// wavefront latency (a tile's waves step through n + k columns at about
// 0.11 us each), plus 30% of one read and write of A (about 4.5 TB/s;
// 3.2 TB/s with a single band, whose few waves keep fewer bytes in
// flight) that does not overlap them, plus 20 us.
double model_chain(const Plan &p, int cus)
{
    const double flops = 6.0 * (double)p.m * (double)(p.n - 1) * (double)p.k;
    const double bytes = 2.0 * (double)p.m * (double)p.n * (double)p.esize;
    if (p.npass <= kChainDeepBands) {
        // Streaming form: a lone wave's step costs about 55 ns with bands of
        // 2, 78 ns with bands of 4 and 120 ns with bands of 8 (one wave
        // issues at most one instruction per 4 cycles); each further wave
        // per SIMD adds 3/4 of that, unless HBM (about 5 TB/s for this mix
        // of reads and writes) takes longer.  Fitted to FP64 sweeps of m = 1024 .. 65536,
        // n = 1024 .. 16384, k = 1 .. 32.
        const double waves = (double)((p.m + 63) / 64) * (double)p.npass;
        const double per_simd = std::max(1.0, std::ceil(waves / (4.0 * (double)cus)));
        const double step = (p.band <= 2 ? 55e-9 : p.band <= 4 ? 78e-9 : 120e-9) *
                            (1.0 + 0.75 * (per_simd - 1.0));
        return std::max((double)p.steps * step, bytes / 5.0e12) + 15e-6;
    }
    const double lat = (double)(p.n + p.k) * 0.11e-6;
    return std::max(flops / 44e12, lat) + 0.3 * bytes / 4.5e12 + 20e-6;
}

}  // namespace

hipError_t configure_launch(Plan &p, int req_waves, int req_publish, int req_shape)
{
    if (p.kernel == kMfma || (p.kernel == kChain && p.mfma_ok)) {
        DeviceInfo d;
        if (device_info(d) != ROTSEQ_SUCCESS)
            return hipErrorInvalidDevice;
        Plan trial = p;
        const double t = p.kernel == kMfma ? plan_mfma(trial, req_waves, req_shape, d)
                                            : plan_mfma(trial, 0, 0, d);
        if (p.kernel == kMfma && t < 0.0)
            return hipErrorInvalidConfiguration;
        if (t >= 0.0 && (p.kernel == kMfma || t < model_chain(p, d.cus))) {
            p = trial;
            p.kernel = kMfma;
            p.spin_limit = wait_spin_limit();
            p.wait_bias = wait_bias();
            return hipSuccess;
        }
    }
    if (p.kernel != kChain)
        return hipSuccess;
    DeviceInfo d;
    if (device_info(d) != ROTSEQ_SUCCESS)
        return hipErrorInvalidDevice;
    const int64_t tiles = (p.m + 63) / 64;
    const int64_t total = tiles * p.npass;
    // Pick W (waves = bands per workgroup).  Each candidate is costed as
    // rounds x (waves per SIMD in a round): `occ` workgroups fit on a CU at
    // once (registers and LDS), so ceil(nwg / (occ * CUs)) rounds run one
    // after another, and within a round the busiest SIMD holds
    // ceil(W * wgs_per_cu / 4) waves.  Ties go to fewer workgroups (fewer
    // hand-offs through A).  A chain of at most kChainDeepBands bands runs
    // in the streaming form, whole in one workgroup: W a multiple of the
    // band count, at most kChainDeepWaves.
    const bool stream = p.npass <= kChainDeepBands && p.steps % chain_unroll(p.band, true) == 0;
    int waves = 0, per_cu = 1;
    size_t lds = 0;
    if (req_waves > 0) {
        waves = std::min(req_waves, 16);
        lds = chain_lds_bytes(p.band, waves, p.esize);
        while (waves > 1 && lds > d.max_lds)
            lds = chain_lds_bytes(p.band, --waves, p.esize);
        p.deep = stream && waves <= kChainDeepWaves && waves % p.npass == 0 ? 1 : 0;
        lds = chain_lds_bytes(p.band, waves, p.esize, p.deep != 0);
    } else {
        p.deep = stream ? 1 : 0;
        const int64_t wgs4 = (total + 3) / 4;  // workgroups at 4 waves
        const int deep_max = wgs4 >= (int64_t)(p.esize == 8 ? 2 : 4) * d.cus ? kChainDeepWaves : 4;
        double best = 1e300;
        for (int wv = 1; wv <= 16; ++wv) {
            // Streaming: 8 waves only where 4 would put several workgroups
            // on every CU (at least 2 in FP64, 4 in FP32), else at most 4.
            // Measured with 8: 65536 x 4096 FP64 k = 8 0.87 -> 0.81 ms, FP32
            // 0.52 -> 0.48 ms; but 32768 x 4096 FP32 k = 8 0.30 -> 0.34 ms;
            // the cost model below ties them.
            if (p.deep && (wv > deep_max || wv % p.npass != 0))
                continue;
            const size_t l = chain_lds_bytes(p.band, wv, p.esize, p.deep != 0);
            if (l > d.max_lds)
                break;
            int occ = 0;
            if (chain_occupancy(p.band, p.arith, p.esize, wv, l, &occ, false, p.deep != 0) !=
                    hipSuccess ||
                occ < 1)
                continue;
            const int64_t nwg = (total + wv - 1) / wv;
            const int64_t slots = (int64_t)occ * d.cus;
            const int64_t rounds = (nwg + slots - 1) / slots;
            const int64_t in_round = std::min<int64_t>(nwg, slots);
            const int64_t wg_per_cu = (in_round + d.cus - 1) / d.cus;
            const int64_t simd_waves = (wv * wg_per_cu + 3) / 4;
            const double cost = (double)rounds * (double)simd_waves + 1e-6 * (double)nwg;
            if (cost < best) {
                best = cost;
                waves = wv;
                per_cu = (int)wg_per_cu;
                lds = l;
            }
        }
        if (waves == 0) {
            waves = p.deep ? p.npass : 1;
            lds = chain_lds_bytes(p.band, waves, p.esize, p.deep != 0);
        }
    }
    (void)per_cu;
    p.waves = waves;
    p.lds_bytes = lds;
    p.nwg = (int)((total + waves - 1) / waves);
    int occ = 0;
    hipError_t e = chain_occupancy(p.band, p.arith, p.esize, waves, lds, &occ, false, p.deep != 0);
    if (e != hipSuccess)
        return e;
    // Consecutive workgroups share tiles; placing them on one XCD keeps the
    // hand-off in that XCD's L2.  Only safe when the whole grid is resident,
    // since the remapped order no longer follows the dispatch order.
    p.remap = (p.nwg % 8 == 0 && p.nwg >= 8 && (int64_t)p.nwg <= (int64_t)occ * d.cus) ? 1 : 0;
    // Publish once per unrolled ring period (R columns) unless asked otherwise.
    int publish = req_publish > 0 ? req_publish / p.unroll : 1;
    int pow2 = 1;
    while (pow2 < publish)
        pow2 *= 2;
    p.publish = pow2;
    p.spin_limit = wait_spin_limit();
    p.wait_bias = wait_bias();
    return hipSuccess;
}

namespace {


// Argument check of rotseq_d; `left`: the sequences mix rows, so C and S
// have m-1 rows and there is work only for n > 0, m > 1.
int check_args(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda, const void *C,
               int64_t ldc, const void *S, int64_t lds, bool left = false)
{
    if (m < 0)
        return -1;
    if (n < 0)
        return -2;
    if (k < 0)
        return -3;
    const int64_t r = left ? m : n;  // length of the dimension the sequences mix
    const bool work = (left ? n > 0 : m > 0) && r > 1 && k > 0;
    const int64_t n1 = r > 1 ? r - 1 : 1;
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
    // e0..e1: packing of A (left application) and coefficient preparation;
    // e1..e2: the sweep; e2..e3: unpacking.
    struct Rec {
        hipEvent_t e0, e1, e2, e3;
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
        (void)hipEventCreate(&r.e3);
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
            float a = 0.f, b = 0.f, c = 0.f;
            if (hipEventSynchronize(r.e3) != hipSuccess ||
                hipEventElapsedTime(&a, r.e0, r.e1) != hipSuccess ||
                hipEventElapsedTime(&b, r.e1, r.e2) != hipSuccess ||
                hipEventElapsedTime(&c, r.e2, r.e3) != hipSuccess)
                rc = ROTSEQ_E_HIP;
            acc.prep_ms += a + c;
            acc.sweep_ms += b;
            acc.sweep_ms_min = acc.calls ? std::min(acc.sweep_ms_min, (double)b) : b;
            acc.sweep_ms_max = acc.calls ? std::max(acc.sweep_ms_max, (double)b) : b;
            acc.calls += 1;
            (void)hipEventDestroy(r.e0);
            (void)hipEventDestroy(r.e1);
            (void)hipEventDestroy(r.e2);
            (void)hipEventDestroy(r.e3);
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

bool resolve(const rotseq_opts *opts, int &arith, int &band, int &kernel)
{
    arith = opts ? opts->arith : 0;
    band = opts ? opts->band : 0;
    kernel = opts ? opts->kernel : 0;
    if (arith == ROTSEQ_ARITH_AUTO)
        arith = kLift;
    if (arith != kExact && arith != kFma && arith != kLift)
        return false;
    if (kernel != ROTSEQ_KERNEL_AUTO && kernel != ROTSEQ_KERNEL_MULTIPASS &&
        kernel != ROTSEQ_KERNEL_CHAIN && kernel != ROTSEQ_KERNEL_MFMA)
        return false;
    if (opts && (opts->waves < 0 || opts->waves > 16 || opts->publish < 0 || opts->shape < 0))
        return false;
    return true;
}

// Plan of the sweep over the matrix whose columns the sequences mix: A
// itself (m x n), or for left application A^T (n x m) packed into the
// workspace after the plan's own buffers (off_pack, leading dimension n).
bool plan_for(Plan &p, int esize, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldc,
              int64_t lds, const rotseq_opts *opts, int kind, size_t &off_pack)
{
    int arith = 0, band = 0, kernel = 0;
    if (!resolve(opts, arith, band, kernel))
        return false;
    // Reflectors are applied as rotations plus tracked column negations,
    // which only the lifting form carries.
    if (kind != kRotate && arith != kLift)
        return false;
    const bool left = opts && opts->left;
    p = Plan{};
    p.m = left ? n : m;
    p.n = left ? m : n;
    p.k = k;
    p.lda = left ? p.m : lda;
    p.ldc = ldc;
    p.lds = lds;
    p.cstep = 1;
    p.arith = arith;
    p.kind = kind;
    p.esize = esize;
    // The matrix-instruction sweep: forward right application (or the
    // packed copy of a left application) of rotations, FP64, automatic
    // arithmetic, with every 8-column block of A within 32-bit offsets.
    // Automatic choice only when no chain-kernel tuning was asked for.
    const bool mfma_ok = kind == kRotate && esize == 8 && !(opts && opts->inverse) &&
                         (opts == nullptr || opts->arith == ROTSEQ_ARITH_AUTO) &&
                         (kernel == kMfma || opts == nullptr ||
                          (opts->waves == 0 && opts->publish == 0 && opts->band == 0)) &&
                         (uint64_t)(left ? p.m : lda) * 8u * 9u < ((uint64_t)1 << 30);
    if (!make_plan(p, kernel, band, mfma_ok))
        return false;
    off_pack = 0;
    if (left) {
        off_pack = p.total;
        p.total = align256(p.total + (size_t)p.m * (size_t)p.n * (size_t)esize);
    }
    return true;
}

template <typename T>
int run(int kind, int64_t m, int64_t n, int64_t k, T *A, int64_t lda, const T *C, int64_t ldc,
        const T *S, int64_t lds, hipStream_t stream, const rotseq_opts *opts, void *ws,
        size_t ws_bytes)
{
    const bool left = opts && opts->left;
    const int bad = check_args(m, n, k, A, lda, C, ldc, S, lds, left);
    if (bad)
        return bad;
    if ((left ? n == 0 || m <= 1 : m == 0 || n <= 1) || k == 0)
        return ROTSEQ_SUCCESS;
    Plan p;
    size_t off_pack = 0;
    if (!plan_for(p, (int)sizeof(T), m, n, k, lda, ldc, lds, opts, kind, off_pack))
        return ROTSEQ_E_UNSUPPORTED;
    if (p.n > INT32_MAX - 64 || (p.kernel != kMfma && p.steps <= 0))
        return ROTSEQ_E_UNSUPPORTED;
    if (const hipError_t e = configure_launch(p, opts ? opts->waves : 0, opts ? opts->publish : 0,
                                              opts ? opts->shape : 0))
        return e == hipErrorInvalidConfiguration ? ROTSEQ_E_UNSUPPORTED : ROTSEQ_E_HIP;
    if (const int rc = status_word(&p.status))
        return rc;
    if (ws) {
        if (ws_bytes < p.total || ((uintptr_t)ws & 255) != 0)
            return ROTSEQ_E_WORKSPACE;
    } else {
        const int rc = pool().get(stream, p.total, &ws);
        if (rc)
            return rc;
    }
    // X: the p.m x p.n matrix the sweep runs on (A, or the packed A^T).
    T *X = left ? (T *)((char *)ws + off_pack) : A;
    Profiler::Rec rec{};
    const bool timed = profiler().begin(rec, stream);
    if (left && launch_transpose(A, m, n, lda, X, p.lda, (int)sizeof(T), stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (opts && opts->inverse) {
        // The inverse applies, for p = k-1..0 and j = n-2..0, the rotation
        // (c, -s) to columns (j, j+1).  On the column-reversed matrix
        // A'(:, i) = A(:, n-1-i) that is the rotation (c, s) on columns
        // (n-2-j, n-1-j) in the forward order of Algorithm 2, with
        // C'(i, q) = C(n-2-i, k-1-q): a forward call on reversed views.
        // A reflector is its own inverse, so the inverse of a reflector
        // sequence is the same reflectors in reverse order; on the reversed
        // matrix each one reads as kReflectRev (see pair_rotation).
        const int64_t rn = p.n, ld = p.lda;
        X += (rn - 1) * ld;
        p.lda = -ld;
        C += (rn - 2) + (k - 1) * ldc;
        S += (rn - 2) + (k - 1) * lds;
        p.ldc = -ldc;
        p.lds = -lds;
        p.cstep = -1;
        if (p.kind == kReflect)
            p.kind = kReflectRev;
    }
    if (launch_prep(p, C, S, ws, stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (timed)
        (void)hipEventRecord(rec.e1, stream);
    if (launch_sweep(p, X, ws, stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (timed)
        (void)hipEventRecord(rec.e2, stream);
    if (left && launch_transpose((const char *)ws + off_pack, p.m, p.n, p.m, A, lda, (int)sizeof(T),
                                 stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (timed) {
        (void)hipEventRecord(rec.e3, stream);
        profiler().finish(rec);
    }
    return ROTSEQ_SUCCESS;
}

// Sequences of 3x3 reflectors: arguments checked in the order of
// rotseq_refl3_ex_d, then the records are prepared and the bands swept.
// The inverse order sweeps a column-reversed view of A (negative leading
// dimension) with the reflectors read backwards; left application sweeps a
// transposed copy of A packed after the records in the workspace.
bool refl3_opts_ok(const rotseq_opts *o)
{
    return o == nullptr || (o->arith == ROTSEQ_ARITH_AUTO && o->kernel == ROTSEQ_KERNEL_AUTO &&
                            o->band == 0 && o->waves == 0 && o->publish == 0 && o->shape == 0);
}

// Workspace of a 3x3 reflector call: the records, then (left application)
// the packed transposed copy.  False for shapes the sweep does not index.
bool refl3_layout(Refl3Plan &p, size_t &off_pack, size_t &total, int64_t m, int64_t n, int64_t k,
                  int64_t lda, int esize, bool left, int width = 3)
{
    if (!refl3_plan(p, left ? n : m, left ? m : n, k, left ? n : lda, esize, width))
        return false;
    off_pack = (p.total + 255) & ~(size_t)255;
    total = left ? off_pack + (((size_t)m * (size_t)n * (size_t)esize + 255) & ~(size_t)255) : p.total;
    return true;
}

// The sweep of a call whose arguments are checked: reflectors `width`
// columns wide (3; or 2 with NU2 == NULL), forward or inverse order, right
// or left side.
template <typename T>
int refl3_core(int64_t m, int64_t n, int64_t k, T *A, int64_t lda, const T *TAU, int64_t ldt,
               const T *NU1, int64_t ld1, const T *NU2, int64_t ld2, int width, bool inverse,
               bool left, hipStream_t stream, void *ws, size_t ws_bytes)
{
    const int64_t r = left ? m : n;
    Refl3Plan p;
    size_t off_pack = 0, total = 0;
    if (!refl3_layout(p, off_pack, total, m, n, k, lda, (int)sizeof(T), left, width))
        return ROTSEQ_E_UNSUPPORTED;
    if (ws) {
        if (ws_bytes < total || ((uintptr_t)ws & 255) != 0)
            return ROTSEQ_E_WORKSPACE;
    } else {
        const int rc = pool().get(stream, total, &ws);
        if (rc)
            return rc;
    }
    // The swept matrix: A itself, or its transpose packed in the workspace
    // (p.m x p.n, leading dimension p.lda).
    T *X = left ? (T *)((char *)ws + off_pack) : A;
    if (left && launch_transpose(A, m, n, lda, X, p.lda, (int)sizeof(T), stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    int64_t cj = 1;
    if (inverse) {
        // Reversed columns and reflectors: view column c is column p.n-1-c,
        // record (j, q) is reflector (p.n-3-j, k-1-q).
        X += (p.n - 1) * p.lda;
        p.lda = -p.lda;
        TAU += (r - 3) + (k - 1) * ldt;
        NU1 += (r - 3) + (k - 1) * ld1;
        NU2 += (r - 3) + (k - 1) * ld2;
        ldt = -ldt;
        ld1 = -ld1;
        ld2 = -ld2;
        cj = -1;
    }
    Profiler::Rec rec{};
    const bool timed = profiler().begin(rec, stream);
    if (launch_refl3_prep(p, TAU, ldt, NU1, ld1, NU2, ld2, cj, ws, stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (timed)
        (void)hipEventRecord(rec.e1, stream);
    if (launch_refl3_sweep(p, X, ws, inverse, stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (timed)
        (void)hipEventRecord(rec.e2, stream);
    if (left && launch_transpose((T *)((char *)ws + off_pack), n, m, n, A, lda, (int)sizeof(T),
                                 stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (timed) {
        (void)hipEventRecord(rec.e3, stream);
        profiler().finish(rec);
    }
    return ROTSEQ_SUCCESS;
}

template <typename T>
int run_refl3(int64_t m, int64_t n, int64_t k, T *A, int64_t lda, const T *TAU, int64_t ldt,
              const T *NU1, int64_t ld1, const T *NU2, int64_t ld2, hipStream_t stream,
              const rotseq_opts *opts, void *ws, size_t ws_bytes)
{
    const bool left = opts && opts->left, inverse = opts && opts->inverse;
    const int64_t r = left ? m : n;  // the dimension the reflectors mix
    if (m < 0)
        return -1;
    if (n < 0)
        return -2;
    if (k < 0)
        return -3;
    const bool work = (left ? n > 0 : m > 0) && r > 2 && k > 0;
    const int64_t r2 = r > 2 ? r - 2 : 1;
    if (work && A == nullptr)
        return -4;
    if (lda < (m > 1 ? m : 1))
        return -5;
    if (work && TAU == nullptr)
        return -6;
    if (ldt < r2)
        return -7;
    if (work && NU1 == nullptr)
        return -8;
    if (ld1 < r2)
        return -9;
    if (work && NU2 == nullptr)
        return -10;
    if (ld2 < r2)
        return -11;
    if (!refl3_opts_ok(opts))
        return ROTSEQ_E_UNSUPPORTED;
    if (!work)
        return ROTSEQ_SUCCESS;
    return refl3_core(m, n, k, A, lda, TAU, ldt, NU1, ld1, NU2, ld2, 3, inverse, left, stream, ws,
                      ws_bytes);
}

// 2x2 reflectors applied by the formula as written (ROTSEQ_ARITH_EXACT): any
// (tau, nu), as 3x3 reflectors with nu2 = 0 on the 3x3 sweep.  Forward order
// only (right, or left through the packed copy).
template <typename T>
int run_refl_exact(int64_t m, int64_t n, int64_t k, T *A, int64_t lda, const T *TAU, int64_t ldt,
                   const T *NU, int64_t ldn, hipStream_t stream, const rotseq_opts *opts, void *ws,
                   size_t ws_bytes)
{
    const bool left = opts->left != 0;
    const int bad = check_args(m, n, k, A, lda, TAU, ldt, NU, ldn, left);
    if (bad)
        return bad;
    if ((left ? n == 0 || m <= 1 : m == 0 || n <= 1) || k == 0)
        return ROTSEQ_SUCCESS;
    if (opts->inverse || opts->kernel != ROTSEQ_KERNEL_AUTO || opts->band || opts->waves ||
        opts->publish || opts->shape)
        return ROTSEQ_E_UNSUPPORTED;
    return refl3_core<T>(m, n, k, A, lda, TAU, ldt, NU, ldn, nullptr, 0, 2, false, left, stream, ws,
                         ws_bytes);
}

}  // namespace

int check_problem(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda, const void *C,
                  int64_t ldc, const void *S, int64_t lds)
{
    return check_args(m, n, k, A, lda, C, ldc, S, lds);
}

bool resolve_opts(const rotseq_opts *opts, int &arith, int &band, int &kernel)
{
    return resolve(opts, arith, band, kernel);
}

int device_query(int *cus, size_t *max_lds, int **status)
{
    DeviceInfo d;
    const int rc = device_info(d);
    if (rc)
        return rc;
    *cus = d.cus;
    *max_lds = d.max_lds;
    return status_word(status);
}

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
    if (!esize || k <= 0)
        return 0;
    const bool left = opts && opts->left;
    if (left ? n <= 0 || m <= 1 : m <= 0 || n <= 1)
        return 0;
    Plan p;
    size_t off_pack = 0;
    const int64_t n1 = (left ? m : n) - 1;
    if (!plan_for(p, esize, m, n, k, m, n1, n1, opts, kRotate, off_pack))
        return 0;
    return p.total;
}

int rotseq_ex_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda, const double *C,
                int64_t ldc, const double *S, int64_t lds, hipStream_t stream,
                const rotseq_opts *opts, void *workspace, size_t ws_bytes)
{
    return run<double>(kRotate, m, n, k, A, lda, C, ldc, S, lds, stream, opts, workspace, ws_bytes);
}

int rotseq_ex_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda, const float *C,
                int64_t ldc, const float *S, int64_t lds, hipStream_t stream,
                const rotseq_opts *opts, void *workspace, size_t ws_bytes)
{
    return run<float>(kRotate, m, n, k, A, lda, C, ldc, S, lds, stream, opts, workspace, ws_bytes);
}

int rotseq_refl_ex_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda, const double *TAU,
                     int64_t ldt, const double *NU, int64_t ldn, hipStream_t stream,
                     const rotseq_opts *opts, void *workspace, size_t ws_bytes)
{
    if (opts && opts->arith == ROTSEQ_ARITH_EXACT)
        return run_refl_exact<double>(m, n, k, A, lda, TAU, ldt, NU, ldn, stream, opts, workspace,
                                      ws_bytes);
    return run<double>(kReflect, m, n, k, A, lda, TAU, ldt, NU, ldn, stream, opts, workspace, ws_bytes);
}

int rotseq_refl_ex_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda, const float *TAU,
                     int64_t ldt, const float *NU, int64_t ldn, hipStream_t stream,
                     const rotseq_opts *opts, void *workspace, size_t ws_bytes)
{
    if (opts && opts->arith == ROTSEQ_ARITH_EXACT)
        return run_refl_exact<float>(m, n, k, A, lda, TAU, ldt, NU, ldn, stream, opts, workspace,
                                     ws_bytes);
    return run<float>(kReflect, m, n, k, A, lda, TAU, ldt, NU, ldn, stream, opts, workspace, ws_bytes);
}

int rotseq_refl3_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda, const double *TAU,
                   int64_t ldt, const double *NU1, int64_t ld1, const double *NU2, int64_t ld2,
                   hipStream_t stream, void *workspace, size_t ws_bytes)
{
    return run_refl3<double>(m, n, k, A, lda, TAU, ldt, NU1, ld1, NU2, ld2, stream, nullptr,
                             workspace, ws_bytes);
}

int rotseq_refl3_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda, const float *TAU,
                   int64_t ldt, const float *NU1, int64_t ld1, const float *NU2, int64_t ld2,
                   hipStream_t stream, void *workspace, size_t ws_bytes)
{
    return run_refl3<float>(m, n, k, A, lda, TAU, ldt, NU1, ld1, NU2, ld2, stream, nullptr,
                            workspace, ws_bytes);
}

int rotseq_refl3_ex_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda, const double *TAU,
                      int64_t ldt, const double *NU1, int64_t ld1, const double *NU2, int64_t ld2,
                      hipStream_t stream, const rotseq_opts *opts, void *workspace, size_t ws_bytes)
{
    return run_refl3<double>(m, n, k, A, lda, TAU, ldt, NU1, ld1, NU2, ld2, stream, opts,
                             workspace, ws_bytes);
}

int rotseq_refl3_ex_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda, const float *TAU,
                      int64_t ldt, const float *NU1, int64_t ld1, const float *NU2, int64_t ld2,
                      hipStream_t stream, const rotseq_opts *opts, void *workspace, size_t ws_bytes)
{
    return run_refl3<float>(m, n, k, A, lda, TAU, ldt, NU1, ld1, NU2, ld2, stream, opts,
                            workspace, ws_bytes);
}

size_t rotseq_refl3_workspace_bytes(char dtype, int64_t m, int64_t n, int64_t k)
{
    return rotseq_refl3_ex_workspace_bytes(dtype, m, n, k, nullptr);
}

size_t rotseq_refl3_ex_workspace_bytes(char dtype, int64_t m, int64_t n, int64_t k,
                                       const rotseq_opts *opts)
{
    const int esize = dtype == 'd' ? 8 : dtype == 's' ? 4 : 0;
    const bool left = opts && opts->left;
    const int64_t r = left ? m : n;
    if (!esize || k <= 0 || r <= 2 || (left ? n <= 0 : m <= 0) || !refl3_opts_ok(opts))
        return 0;
    Refl3Plan p;
    size_t off_pack = 0, total = 0;
    if (!refl3_layout(p, off_pack, total, m, n, k, m > 1 ? m : 1, esize, left))
        return 0;
    return total;
}

int rotseq_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda, const double *C, int64_t ldc,
             const double *S, int64_t lds, hipStream_t stream)
{
    return run<double>(kRotate, m, n, k, A, lda, C, ldc, S, lds, stream, nullptr, nullptr, 0);
}

int rotseq_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda, const float *C, int64_t ldc,
             const float *S, int64_t lds, hipStream_t stream)
{
    return run<float>(kRotate, m, n, k, A, lda, C, ldc, S, lds, stream, nullptr, nullptr, 0);
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
    case ROTSEQ_E_TIMEOUT: return "wait timed out (device-side spin limit or server wait)";
    case ROTSEQ_E_BUDGET: return "matrix exceeds the server's device memory budget";
    case ROTSEQ_E_INVAL: return "unknown matrix id or ticket";
    case ROTSEQ_E_CLOSED: return "matrix was closed";
    case ROTSEQ_E_FAILED: return "an earlier sweep of this matrix failed";
    case ROTSEQ_E_TOO_LARGE: return "workspace exceeds the fixed scratch of rotseq_noalloc_d";
    default: return "unknown error code";
    }
}

int rotseq_version(void) { return 100; }

int rotseq_launch_describe(char dtype, int64_t m, int64_t n, int64_t k, int64_t lda,
                           const rotseq_opts *opts, rotseq_launch_info *out)
{
    const int esize = dtype == 'd' ? 8 : dtype == 's' ? 4 : 0;
    if (!esize)
        return -1;
    if (m < 0)
        return -2;
    if (n < 0)
        return -3;
    if (k < 0)
        return -4;
    if (lda < (m > 1 ? m : 1))
        return -5;
    if (out == nullptr)
        return -7;
    *out = rotseq_launch_info{};
    const bool left = opts && opts->left;
    if ((left ? n == 0 || m <= 1 : m == 0 || n <= 1) || k == 0)
        return ROTSEQ_SUCCESS;
    Plan p;
    size_t off_pack = 0;
    const int64_t n1 = (left ? m : n) - 1;
    if (!plan_for(p, esize, m, n, k, lda, n1, n1, opts, kRotate, off_pack))
        return ROTSEQ_E_UNSUPPORTED;
    if (const hipError_t e = configure_launch(p, opts ? opts->waves : 0, opts ? opts->publish : 0,
                                              opts ? opts->shape : 0))
        return e == hipErrorInvalidConfiguration ? ROTSEQ_E_UNSUPPORTED : ROTSEQ_E_HIP;
    out->kernel = p.kernel;
    out->band = p.band;
    out->waves = p.waves;
    out->workgroups = p.nwg;
    if (p.kernel == kMfma) {
        out->bands_per_wave = p.mfma_nb;
        out->rows_per_wave = 16 * p.mfma_rows;
        out->segments = p.mfma_nseg;
    }
    out->workspace_bytes = p.total;
    return ROTSEQ_SUCCESS;
}

int rotseq_test_set_waits(int32_t spin_limit, int32_t unreachable)
{
    if (spin_limit < 0)
        return -1;
    g_spin_limit.store(spin_limit == 0 ? kDefaultSpinLimit : spin_limit, std::memory_order_relaxed);
    // Column counts are below 2^28 (larger n runs the multipass kernel,
    // which never waits), so a target 2^29 higher is never reached.
    g_wait_bias.store(unreachable ? (1 << 29) : 0, std::memory_order_relaxed);
    return ROTSEQ_SUCCESS;
}

int rotseq_device_status(int reset)
{
    int *word = nullptr;
    const int rc = status_word(&word);
    if (rc)
        return rc;
    if (hipDeviceSynchronize() != hipSuccess)
        return ROTSEQ_E_HIP;
    int v = 0;
    if (hipMemcpy(&v, word, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (reset && hipMemset(word, 0, sizeof(int)) != hipSuccess)
        return ROTSEQ_E_HIP;
    int na = 0;
    if (noalloc_status(reset, &na) != ROTSEQ_SUCCESS)
        return ROTSEQ_E_HIP;
    v |= na;
    if (reset && hipDeviceSynchronize() != hipSuccess)
        return ROTSEQ_E_HIP;
    return v;
}

int rotseq_profile_enable(int on)
{
    profiler().on.store(on != 0);
    return ROTSEQ_SUCCESS;
}

int rotseq_profile_read(rotseq_profile *out, int reset) { return profiler().read(out, reset); }

}  // extern "C"
