// HIP kernels of librotseq for gfx950 (CDNA4, wave64).
//
// Operation: A <- A * G(0,0) ... G(n-2,k-1) (Algorithms 1 and 2 of the
// paper).  Rows of A are independent, so one 64-lane wave owns a 64-row tile
// of A (one row per lane) and never talks to other waves.  Inside a tile the
// rotations are applied in the wavefront order of Section 1.1: step t of a
// band of K sequences (p0 .. p0+K-1) applies the rotations
//     (j = t - q, p = p0 + q)   for q = 0, 1, ..., K-1   (in that order),
// which respects the only ordering constraint of Algorithm 2 (rotation (j,p)
// after (j+1,p-1) and after (j-1,p)) and touches the K+1 columns t-K+1..t+1.
// Those columns live in a register ring; each step loads one new column
// (t+1+D, D steps ahead) and stores one finished column (t-K+1), so A is read
// and written once per band instead of once per sequence (Sections 1.1-3).
// The startup and shutdown triangles of every band (Section 2) are padded
// with identity rotations and virtual zero columns, so every step runs the
// same straight-line code.
//
// The coefficients of step t form one contiguous record of K pairs, prepared
// by prep_coef in the order the sweep consumes them (the paper's "packing of
// C and S", Section 4).  They are identical for all 64 lanes, so the sweep
// reads them through the scalar data cache into SGPRs (one SGPR-pair operand
// per FMA) instead of broadcasting through LDS or vector registers.
//
// Edges use buffer descriptors: a column descriptor covers exactly the valid
// rows of the tile (fewer than 64 in the last tile), and columns outside
// [0, n) get an empty descriptor, so out-of-range loads return 0 and
// out-of-range stores are dropped by the hardware without a branch.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rotseq.h"
#include "rotseq_device.h"
#include "rotseq_internal.h"

namespace rotseq {
namespace {

using namespace dev;

// Wavefront steps a column load is issued ahead of its first use.
constexpr int kPrefetch = 4;

// One band of K sequences over the whole tile: steps t = 0 .. steps-1.
// `tile` is the address of A(i0, 0), `ldab` the column stride in bytes.
template <typename T, int K, int ARITH, bool SIGN>
__device__ __forceinline__ void sweep_band(uint64_t tile, uint64_t ldab, uint32_t rowbytes, int voff,
                                           int n, ConstPairs<T> w, int steps, ConstScalars<T> sign)
{
    constexpr int D = kPrefetch;
    constexpr int R = K + 1 + D;  // ring: K+1 live columns + D in flight
    T ring[R];
#pragma unroll
    for (int s = 0; s < R; ++s)
        ring[s] = T(0);
    // Load stream: column lc at address lp.  Store stream: column sc at sp.
    uint64_t lp = tile;
    int lc = 0;
#pragma unroll
    for (int c = 0; c <= D; ++c) {
        ring[c] = buf_load<kPolicyL2>(T(), make_rsrc(lp, lc < n ? rowbytes : 0u), voff);
        lp += ldab;
        ++lc;
        opaque(lp);
    }
    uint64_t sp = tile - (uint64_t)(K - 1) * ldab;
    int sc = -(K - 1);
    uint64_t wp = (uint64_t)w;

    for (int t0 = 0; t0 < steps; t0 += R) {
#pragma unroll
        for (int u = 0; u < R; ++u) {
            // Column t+1+D goes into the slot of column t-K, stored last step.
            ring[(u + D + 1) % R] =
                buf_load<kPolicyL2>(T(), make_rsrc(lp, lc < n ? rowbytes : 0u), voff);
            lp += ldab;
            ++lc;
            opaque(lp);
            ConstPairs<T> wt = (ConstPairs<T>)wp;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const T a = wt[q].a, b = wt[q].b;
                rotate<ARITH>(ring[(u - q + R) % R], ring[(u - q + 1 + R) % R], a, b);
            }
            wp += K * sizeof(CoefPair<T>);
            opaque(wp);
            // Column t-K+1 has seen all K sequences of the band.
            T v = ring[(u - K + 1 + R) % R];
            const bool valid = (unsigned)sc < (unsigned)n;
            if constexpr (SIGN)
                v *= sign[valid ? sc : 0];
            buf_store(v, make_rsrc(sp, valid ? rowbytes : 0u), voff);
            sp += ldab;
            ++sc;
            opaque(sp);
            // Keep the scheduler from hoisting the scalar coefficient loads of
            // later steps: they would exhaust the SGPR file and spill.
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Multi-pass sweep: one wave per 64-row tile applies the bands one after the
// other; A round-trips through memory between bands.
template <typename T, int K, int ARITH>
__global__ __launch_bounds__(kWave) void sweep_multipass(T *__restrict__ A, int64_t lda, int64_t m,
                                                         int64_t n,
                                                         const CoefPair<T> *__restrict__ coef,
                                                         int steps, int npass,
                                                         const T *__restrict__ sign)
{
    const int64_t i0 = (int64_t)blockIdx.x * kWave;
    const int64_t rows = m - i0 < kWave ? m - i0 : kWave;
    const uint32_t rowbytes = (uint32_t)(rows * (int64_t)sizeof(T));
    const int voff = threadIdx.x * (int)sizeof(T);
    const uint64_t tile = (uint64_t)(A + i0);
    const uint64_t ldab = (uint64_t)lda * sizeof(T);
    for (int pass = 0; pass < npass; ++pass) {
        ConstPairs<T> w = (ConstPairs<T>)(coef + (int64_t)pass * (steps + 1) * K);  // pad = 1
        if (ARITH == kLift && pass == npass - 1)
            sweep_band<T, K, ARITH, true>(tile, ldab, rowbytes, voff, (int)n, w, steps,
                                          (ConstScalars<T>)sign);
        else
            sweep_band<T, K, ARITH, false>(tile, ldab, rowbytes, voff, (int)n, w, steps,
                                           (ConstScalars<T>)sign);
        // The next band re-reads the columns this band stored.
        __builtin_amdgcn_s_waitcnt(0);
    }
}

// ------------------------------------------------------------------ prep
//
// Column signs of the lifting form: a rotation with c < 0 is applied as
// (-c, -s) and leaves both of its columns negated.  A 2x2 reflector (kinds
// kReflect, kReflectRev) is a rotation followed by negating its right
// column, so it may negate either column alone.  Which columns pair (j,p)
// negates is known up front: bit q of the low half of negmask for the left
// column j, of the high half for the right column j+1.  The sign of a column
// just before rotation (j,p) in Algorithm 2's order is the parity of the
// negations by the rotations that touched it earlier:
//   column j:   (j-1, p') as its right column for p' <= p,
//               (j, p')   as its left column for p' < p;
//   column j+1: (j, p')   as its right column for p' < p,
//               (j+1, p') as its left column for p' < p.
// A rotation sees its columns' signs only through their product, which turns
// s into s' = s * sign(j) * sign(j+1).  For plain rotations both halves of
// negmask are equal and the terms of pair j cancel.

__device__ __forceinline__ uint64_t low_bits(int q) { return q >= 64 ? ~0ull : ((1ull << q) - 1); }

// Rotation part (c, s) of pair (j, p) of a sequence kind, and whether the
// pair also negates its right column.  Kind kReflect reads (C, S) as
// (tau, nu): H = I - tau v v^T with v = (1, nu) acts on (x, y) as
//   x' = (1-tau) x - tau nu y,   y' = -tau nu x + (1 - tau nu^2) y,
// and for an orthogonal H (tau (1 + nu^2) = 2) the second row is
// -(-s x + c y) with c = 1 - tau, s = -tau nu: the rotation (c, s), then the
// right column negated (none of this for tau = 0, where H = I).  Kind
// kReflectRev is the same reflector seen on the column-reversed matrix,
// where its left and right columns trade places: the rotation (-c, s),
// then the (new) right column negated (and still the identity for tau = 0).
template <typename T>
__device__ __forceinline__ void pair_rotation(int kind, T cv, T sv, double &c, double &s, bool &flip)
{
    if (kind == kRotate) {
        c = (double)cv;
        s = (double)sv;
        flip = false;
    } else {
        const double tau = (double)cv, nu = (double)sv;
        flip = tau != 0.0;
        c = 1.0 - tau;
        if (kind == kReflectRev && flip)
            c = -c;
        s = -(tau * nu);
    }
}

// negmask[pass*(n-1) + j]: bit q = pair (j, pass*K + q) negates column j,
// bit 32 + q = it negates column j+1 (K <= 32).
// `nonortho` is set when a reflector (tau, nu) with tau != 0 is not
// orthogonal, |tau (1 + nu^2) - 2| > 64 eps(T): the rotation-plus-negation
// form applies only to orthogonal reflectors (Section 6 counts the work of
// H = I - tau v v^T as a replacement for a rotation).
template <typename T>
__device__ __forceinline__ uint64_t negmask_elem(const T *__restrict__ C, int64_t cj, int64_t ldc,
                                                 const T *__restrict__ S, int64_t lds, int64_t n1,
                                                 int64_t k, int K, int kind, int64_t idx,
                                                 bool &nonortho)
{
    constexpr double kTol = 64.0 * (sizeof(T) == 8 ? 2.220446049250313e-16 : 1.1920928955078125e-07);
    const int64_t pass = idx / n1, j = idx - pass * n1;
    uint64_t mask = 0;
    for (int q = 0; q < K; ++q) {
        const int64_t p = pass * K + q;
        if (p >= k)
            continue;
        const T cv = C[j * cj + p * ldc];
        const T sv = kind == kRotate ? T(0) : S[j * cj + p * lds];
        double c, s;
        bool flip;
        pair_rotation(kind, cv, sv, c, s, flip);
        if (kind != kRotate && cv != T(0)) {
            const double nu = (double)sv;
            nonortho |= !(__builtin_fabs((double)cv * (1.0 + nu * nu) - 2.0) <= kTol);
        }
        const uint64_t neg = c < 0.0 ? 1u : 0u;
        mask |= (neg << q) | ((neg ^ (flip ? 1u : 0u)) << (32 + q));
    }
    return mask;
}

// parity[pass*(n-1) + j] = parities of the negations by pair j in bands
// < pass (bit 0: of its left column, bit 1: of its right column), for
// pass = 0 .. npass (the last row is the total).
// Parities of one band's negations of a pair (bit 0: its left column,
// bit 1: its right column).
__device__ __forceinline__ unsigned negmask_parities(uint64_t nm)
{
    return (__builtin_popcount((unsigned)nm) & 1u) | ((__builtin_popcount((unsigned)(nm >> 32)) & 1u) << 1);
}

__device__ __forceinline__ void parity_elem(const uint64_t *__restrict__ negmask, int64_t n1,
                                            int npass, uint8_t *__restrict__ parity, int64_t j)
{
    unsigned acc = 0;
    for (int pass = 0; pass < npass; ++pass) {
        parity[(int64_t)pass * n1 + j] = (uint8_t)acc;
        acc ^= negmask_parities(negmask[(int64_t)pass * n1 + j]);
    }
    parity[(int64_t)npass * n1 + j] = (uint8_t)acc;
}

// sign[c] = (-1)^(negations of column c: as the right column of pair c-1 and
// the left column of pair c, over all bands).
template <typename T>
__device__ __forceinline__ T sign_elem(const uint8_t *__restrict__ total, int64_t n, int64_t c)
{
    const unsigned f = ((c > 0 ? total[c - 1] >> 1 : 0u) ^ (c + 1 < n ? total[c] : 0u)) & 1u;
    return f ? T(-1) : T(1);
}

// coef[(pass*(steps+pad) + t)*K + q] = coefficients of rotation (t-q, pass*K+q),
// or the identity where that rotation does not exist (t >= steps is always
// identity padding).
template <typename T>
__device__ __forceinline__ CoefPair<T> coef_elem(const T *__restrict__ C, int64_t cj, int64_t ldc,
                                                 const T *__restrict__ S, int64_t lds, int64_t n1,
                                                 int64_t k, int K, int steps, int pad, int arith,
                                                 int kind, const uint64_t *__restrict__ negmask,
                                                 const uint8_t *__restrict__ parity, int64_t idx)
{
    const int q = (int)(idx % K);
    const int64_t t = (idx / K) % (steps + pad);
    const int64_t pass = idx / ((int64_t)K * (steps + pad));
    const int64_t j = t - q, p = pass * K + q;
    CoefPair<T> out;
    if (j >= 0 && j < n1 && p < k) {
        const T c = C[j * cj + p * ldc], s = S[j * cj + p * lds];
        if (arith == kLift) {
            const uint64_t *nm = negmask + pass * n1;
            const uint8_t *par = parity + pass * n1;
            const uint64_t lo = low_bits(q), lo1 = low_bits(q + 1);
            // sign(j) * sign(j+1) as a parity (see the comment above low_bits)
            unsigned tau = 0;
            if (j > 0)
                tau ^= (par[j - 1] >> 1) ^ (__builtin_popcountll((nm[j - 1] >> 32) & lo1) & 1u);
            tau ^= par[j] ^ (par[j] >> 1) ^ (__builtin_popcountll((nm[j] & lo) ^ ((nm[j] >> 32) & lo)) & 1u);
            if (j + 1 < n1)
                tau ^= par[j + 1] ^ (__builtin_popcountll(nm[j + 1] & lo) & 1u);
            tau &= 1u;
            double cd, sr;
            bool flip;
            pair_rotation(kind, c, s, cd, sr, flip);
            (void)flip;  // the negation is in negmask
            const double sd = tau ? -sr : sr;
            double a, b;
            if (!(cd < 0.0)) {
                a = sd / (1.0 + cd);
                b = -sd;
            } else {
                a = -sd / (1.0 - cd);
                b = sd;
            }
            out.a = (T)a;
            out.b = (T)b;
        } else {
            out.a = c;
            out.b = s;
        }
    } else {
        out.a = arith == kLift ? T(0) : T(1);
        out.b = T(0);
    }
    return out;
}

// Lifting form, first launch: thread j computes pair j's negation masks
// band by band and, as it goes, their parities over the bands before each
// one (the last row of `parity` is the total over all bands).
template <typename T>
__global__ void prep_masks(const T *__restrict__ C, int64_t cj, int64_t ldc, const T *__restrict__ S,
                           int64_t lds, int64_t n1, int64_t k, int K, int npass, int kind,
                           uint64_t *__restrict__ negmask, uint8_t *__restrict__ parity, int *status)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n1)
        return;
    bool nonortho = false;
    unsigned acc = 0;
    for (int pass = 0; pass < npass; ++pass) {
        const int64_t idx = (int64_t)pass * n1 + j;
        const uint64_t nm = negmask_elem(C, cj, ldc, S, lds, n1, k, K, kind, idx, nonortho);
        negmask[idx] = nm;
        parity[idx] = (uint8_t)acc;
        acc ^= negmask_parities(nm);
    }
    parity[(int64_t)npass * n1 + j] = (uint8_t)acc;
    if (nonortho)
        __hip_atomic_fetch_or(status, ROTSEQ_STATUS_NOT_ORTHOGONAL, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
}

// Second (or, without the lifting form, only) launch: the coefficient
// records; threads c < n also write column c's final sign (lifting form,
// from the total parities of the first launch), and threads i < flag_words
// zero the sweep's progress flags.
template <typename T>
__global__ void prep_coef(const T *__restrict__ C, int64_t cj, int64_t ldc, const T *__restrict__ S,
                          int64_t lds, int64_t n1, int64_t k, int K, int steps, int pad, int npass,
                          int arith, int kind, const uint64_t *__restrict__ negmask,
                          const uint8_t *__restrict__ parity, CoefPair<T> *__restrict__ coef,
                          T *__restrict__ sign, int *__restrict__ flags, int64_t flag_words)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < flag_words)
        flags[idx] = 0;
    if (arith == kLift && idx < n1 + 1)
        sign[idx] = sign_elem<T>(parity + (int64_t)npass * n1, n1 + 1, idx);
    const int64_t total = (int64_t)npass * (steps + pad) * K;
    if (idx >= total)
        return;
    coef[idx] = coef_elem(C, cj, ldc, S, lds, n1, k, K, steps, pad, arith, kind, negmask, parity, idx);
}


// ------------------------------------------------------------- packing
//
// Left application packs A transposed (Section 4.3: a packed copy laid out
// the way the sweep reads it), so the rows the rotations mix become the
// contiguous columns the sweep streams.  One 256-thread workgroup moves a
// 64 x 64 tile through LDS: it reads 64-element column segments of the
// source (512 B for FP64, one per wave and instruction) and writes 64-element
// column segments of the destination, so both sides are coalesced.  Each
// thread keeps all 16 of its loads in flight (about 128 KB per CU at four
// workgroups, enough to cover HBM latency at full bandwidth).  The tile
// has one padding column, which spreads a transposed read of LDS over all
// banks.

constexpr int kTile = 64;

template <typename T>
__global__ __launch_bounds__(256) void transpose_tiles(const T *__restrict__ src, int64_t rows,
                                                       int64_t cols, int64_t lds_src,
                                                       T *__restrict__ dst, int64_t ldd,
                                                       int64_t tiles_r, int64_t ntiles)
{
    __shared__ T tile[kTile][kTile + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t tid = blockIdx.x; tid < ntiles; tid += gridDim.x) {
        const int64_t r0 = (tid % tiles_r) * kTile, c0 = (tid / tiles_r) * kTile;
        const int64_t r = r0 + lane;
        // Constant trip counts, so that the loops unroll and all 16 loads
        // are issued before the first LDS write waits for one.
        T v[kTile / 4];
#pragma unroll
        for (int i = 0; i < kTile / 4; ++i) {
            const int64_t c = c0 + wave + 4 * i;
            v[i] = r < rows && c < cols ? src[r + c * lds_src] : T(0);
        }
#pragma unroll
        for (int i = 0; i < kTile / 4; ++i)
            tile[wave + 4 * i][lane] = v[i];
        __syncthreads();
        // dst(c, r) = src(r, c): destination column r holds source row r.
        const int64_t c = c0 + lane;
#pragma unroll
        for (int i = 0; i < kTile / 4; ++i) {
            const int rr = wave + 4 * i;
            const int64_t rw = r0 + rr;
            if (rw < rows && c < cols)
                dst[c + rw * ldd] = tile[lane][rr];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ batched prep
//
// One launch per stage covers every problem of a batch: the stage's index
// space is the concatenation of the problems' spaces, and each thread finds
// its problem by binary search over the items' first indices.  Two stages,
// as for a single call: the masks with their running parities (a thread
// per pair), then everything else (a thread per coefficient record, final
// sign or progress flag, whichever of the three is longest).

enum BatchStage : int { kStageMasks, kStageAll };

template <int STAGE>
__device__ __forceinline__ int64_t stage_off(const BatchItem &it)
{
    if constexpr (STAGE == kStageMasks)
        return it.off_parity;
    else
        return it.off_all;
}

// Last item whose first index is <= idx (items are in ascending offset order).
template <int STAGE>
__device__ __forceinline__ int find_item(const BatchItem *__restrict__ items, int count, int64_t idx)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (stage_off<STAGE>(items[mid]) <= idx)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// One search per workgroup: thread 0 finds the item of the workgroup's first
// index, and each thread steps forward from there past the (rarely more
// than one) item boundaries inside the workgroup's range.
template <typename T, int STAGE>
__global__ void prep_batch(const BatchItem *__restrict__ items, int count, int64_t total, int K,
                           int arith)
{
    __shared__ int first_item;
    const int64_t base = (int64_t)blockIdx.x * blockDim.x;
    if (threadIdx.x == 0)
        first_item = find_item<STAGE>(items, count, base < total ? base : total - 1);
    __syncthreads();
    const int64_t idx = base + threadIdx.x;
    if (idx >= total)
        return;
    int item = first_item;
    while (item + 1 < count && stage_off<STAGE>(items[item + 1]) <= idx)
        ++item;
    const BatchItem &it = items[item];
    const int64_t i = idx - stage_off<STAGE>(it);
    const int64_t n1 = it.n - 1;
    if constexpr (STAGE == kStageMasks) {
        bool unused = false;  // rotations only
        unsigned acc = 0;
        for (int pass = 0; pass < it.npass; ++pass) {
            const int64_t e = (int64_t)pass * n1 + i;
            const uint64_t nm = negmask_elem((const T *)it.C, 1, it.ldc, (const T *)it.S, it.lds, n1,
                                             it.k, K, kRotate, e, unused);
            it.negmask[e] = nm;
            it.parity[e] = (uint8_t)acc;
            acc ^= negmask_parities(nm);
        }
        it.parity[(int64_t)it.npass * n1 + i] = (uint8_t)acc;
    } else {
        if (i < (int64_t)it.tiles * it.npass)
            it.flags[i] = 0;
        if (arith == kLift && i < it.n)
            ((T *)it.sign)[i] = sign_elem<T>(it.parity + (int64_t)it.npass * n1, it.n, i);
        if (i < (int64_t)it.npass * (it.steps + it.pad) * K)
            ((CoefPair<T> *)it.coef)[i] = coef_elem((const T *)it.C, 1, it.ldc, (const T *)it.S, it.lds,
                                                    n1, it.k, K, it.steps, it.pad, arith, kRotate,
                                                    it.negmask, it.parity, i);
    }
}

inline unsigned blocks_for(int64_t count, int threads) { return (unsigned)((count + threads - 1) / threads); }

template <typename T>
hipError_t prep_t(const Plan &p, const T *C, const T *S, char *ws, hipStream_t st)
{
    const int64_t n1 = p.n - 1;
    uint64_t *negmask = (uint64_t *)(ws + p.off_negmask);
    uint8_t *parity = (uint8_t *)(ws + p.off_parity);
    T *sign = (T *)(ws + p.off_sign);
    CoefPair<T> *coef = (CoefPair<T> *)(ws + p.off_coef);
    constexpr int B = 256;
    if (p.arith == kLift)
        prep_masks<T><<<blocks_for(n1, B), B, 0, st>>>(C, p.cstep, p.ldc, S, p.lds, n1, p.k, p.band,
                                                      p.npass, p.kind, negmask, parity, p.status);
    const int64_t total = (int64_t)p.npass * (p.steps + p.pad) * p.band;
    const int64_t words = p.kernel == kChain ? ((p.m + 63) / 64) * (int64_t)p.npass : 0;
    const int64_t threads = std::max(std::max(total, words), p.arith == kLift ? (int64_t)p.n : 0);
    prep_coef<T><<<blocks_for(threads, B), B, 0, st>>>(C, p.cstep, p.ldc, S, p.lds, n1, p.k, p.band,
                                                      p.steps, p.pad, p.npass, p.arith, p.kind, negmask,
                                                      parity, coef, sign, (int *)(ws + p.off_flags),
                                                      words);
    return hipGetLastError();
}

template <typename T>
hipError_t prep_batch_t(const BatchLaunch &b, hipStream_t st)
{
    constexpr int B = 256;
    if (b.arith == kLift && b.total_parity > 0)
        prep_batch<T, kStageMasks><<<blocks_for(b.total_parity, B), B, 0, st>>>(
            b.items, b.count, b.total_parity, b.band, b.arith);
    if (b.total_all > 0)
        prep_batch<T, kStageAll><<<blocks_for(b.total_all, B), B, 0, st>>>(
            b.items, b.count, b.total_all, b.band, b.arith);
    return hipGetLastError();
}

template <typename T, int K, int ARITH>
hipError_t go_multipass(const Plan &p, T *A, const char *ws, hipStream_t st)
{
    const unsigned tiles = (unsigned)((p.m + kWave - 1) / kWave);
    sweep_multipass<T, K, ARITH><<<tiles, kWave, 0, st>>>(
        A, p.lda, p.m, p.n, (const CoefPair<T> *)(ws + p.off_coef), p.steps, p.npass,
        (const T *)(ws + p.off_sign));
    return hipGetLastError();
}

template <typename T, int ARITH>
hipError_t sweep_arith(const Plan &p, T *A, const char *ws, hipStream_t st)
{
    switch (p.band) {
    case 1: return go_multipass<T, 1, ARITH>(p, A, ws, st);
    case 2: return go_multipass<T, 2, ARITH>(p, A, ws, st);
    case 4: return go_multipass<T, 4, ARITH>(p, A, ws, st);
    case 8: return go_multipass<T, 8, ARITH>(p, A, ws, st);
    case 16: return go_multipass<T, 16, ARITH>(p, A, ws, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t sweep_t(const Plan &p, T *A, const char *ws, hipStream_t st)
{
    switch (p.arith) {
    case kExact: return sweep_arith<T, kExact>(p, A, ws, st);
    case kFma: return sweep_arith<T, kFma>(p, A, ws, st);
    case kLift: return sweep_arith<T, kLift>(p, A, ws, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int unroll_for_band(int band) { return band + 1 + kPrefetch; }

hipError_t launch_prep(const Plan &p, const void *C, const void *S, void *ws, hipStream_t stream)
{
    if (p.kernel == kMfma)
        return launch_mfma_prep(p, C, S, ws, stream);
    if (p.esize == 8)
        return prep_t<double>(p, (const double *)C, (const double *)S, (char *)ws, stream);
    return prep_t<float>(p, (const float *)C, (const float *)S, (char *)ws, stream);
}

hipError_t launch_transpose(const void *src, int64_t rows, int64_t cols, int64_t lds_src, void *dst,
                            int64_t ldd, int esize, hipStream_t stream)
{
    if (rows <= 0 || cols <= 0)
        return hipSuccess;
    const int64_t tiles_r = (rows + kTile - 1) / kTile;
    const int64_t ntiles = tiles_r * ((cols + kTile - 1) / kTile);
    const unsigned grid = (unsigned)std::min<int64_t>(ntiles, (int64_t)1 << 20);
    if (esize == 8)
        transpose_tiles<double><<<grid, 256, 0, stream>>>((const double *)src, rows, cols, lds_src,
                                                          (double *)dst, ldd, tiles_r, ntiles);
    else
        transpose_tiles<float><<<grid, 256, 0, stream>>>((const float *)src, rows, cols, lds_src,
                                                         (float *)dst, ldd, tiles_r, ntiles);
    return hipGetLastError();
}

hipError_t launch_prep_batch(const BatchLaunch &b, hipStream_t stream)
{
    if (b.count <= 0)
        return hipSuccess;
    if (b.esize == 8)
        return prep_batch_t<double>(b, stream);
    return prep_batch_t<float>(b, stream);
}

hipError_t launch_sweep(const Plan &p, void *A, const void *ws, hipStream_t stream)
{
    if (p.kernel == kChain)
        return launch_chain(p, A, ws, stream);
    if (p.kernel == kMfma)
        return launch_mfma(p, A, ws, stream);
    if (p.esize == 8)
        return sweep_t<double>(p, (double *)A, (const char *)ws, stream);
    return sweep_t<float>(p, (float *)A, (const char *)ws, stream);
}

}  // namespace rotseq
