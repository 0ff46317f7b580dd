// Pipelined sweep kernel of librotseq for gfx950: chains of band-waves.
//
// Work unit ("band-wave"): one 64-row tile of A (one row per lane) and one
// band of K consecutive sequences, swept over all columns in the wavefront
// order of Section 1.1 with the register ring of the multipass kernel.  The
// band-waves of a tile must run in band order, but only column by column:
// band b may consume column c as soon as band b-1 has finished it (the block
// dependency of Section 2).  Band-waves are numbered tile-major and
// consecutive ones are packed W to a workgroup (one wave each), so a
// workgroup holds a chain of bands of one tile, or the tail of one tile's
// chain and the head of the next.  Inside a workgroup, column hand-off
// between neighbours in a chain goes through an LDS ring of RB column slots
// with produced/consumed counters.  Where a chain crosses a workgroup
// boundary, the producer writes the columns to A in place with device-scope
// (write-through) stores and publishes how many leading columns are complete
// in a device-scope counter; the consumer polls that counter and reads A
// with device-scope loads.  The producer publishes a column only after
// `s_waitcnt` has seen its store complete (counting stores in issue order,
// kPublishLag columns behind the newest), so no cache write-back fence is
// needed on the producer's path.
// With W chosen so that the number of workgroups matches the number of CUs,
// every CU gets the same amount of work regardless of how m relates to 64.
//
// Every wait is bounded: after `spin_limit` polls a wave records
// ROTSEQ_E_TIMEOUT in the status word and carries on with whatever data it
// has, so the grid always drains.  All accesses stay in bounds whatever the
// data (buffer descriptors for A, ring indices modulo RB for LDS).
#include "rotseq.h"
#include "rotseq_device.h"
#include "rotseq_internal.h"

namespace rotseq {
using namespace dev;
namespace {

// Column prefetch distance of the chain kernel: R = K + 1 + D steps form
// one unrolled loop body and RB = R ring slots per LDS channel, so every
// slot index in the body is a compile-time constant.
template <int K>
struct ChainGeom {
    static constexpr int R = K <= 4 ? 8 : 16;
    static constexpr int D = R - K - 1;
};

struct ChainArgs {
    uint64_t A;      // address of A(0,0)
    uint64_t ldab;   // column stride of A in bytes
    int64_t m;
    int n;
    int steps;       // padded wavefront steps per band (multiple of R)
    int nbands;
    int tiles;
    int waves;       // band-waves (= waves) per workgroup
    int nwg;         // workgroups in the grid
    int remap;       // 1: consecutive workgroups on the same XCD
    int publish;     // columns (a power of 2) between cross-workgroup progress updates
    int spin_limit;  // polls before a wait gives up
    uint32_t lds_words;  // dynamic LDS size in 4-byte words
    uint64_t coef;   // [nbands][steps + 1][K] coefficient pairs
    uint64_t sign;   // [n] final column signs (lifting arithmetic)
    int *flags;      // [tiles][nbands] published progress (columns)
    int *status;     // error word
};

constexpr int kCounters = 32;  // produced[0..15], consumed[16..31]
// A producer publishes column c only once its store has completed; it waits
// for all but the newest kPublishLag stores, so it rarely waits at all.
constexpr int kPublishLag = 16;

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Keeps a running scalar counter opaque to the optimiser (see opaque()).
__device__ __forceinline__ void opaque_i(int &x) { asm volatile("" : "+s"(x)); }

__device__ __forceinline__ void record_timeout(int *status)
{
    __hip_atomic_fetch_or(status, ROTSEQ_E_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until the LDS counter exceeds `need`; returns its value.  After a
// timeout `limit` drops to 0, so the wave never waits again and the grid
// drains within one time-out per wave.
typedef __attribute__((address_space(3))) volatile int lds_counter;

__device__ __forceinline__ int wait_lds(lds_counter *p, int need, int &limit, int *status)
{
    int v = uniform(*p);
    for (int polls = 0; v <= need; ++polls) {
        if (polls >= limit) {
            record_timeout(status);
            limit = 0;
            return 0x7fffffff;
        }
        __builtin_amdgcn_s_sleep(1);
        v = uniform(*p);
    }
    return v;
}

// Waits until the device-scope progress counter exceeds `need` (polls cost
// a memory round trip, so they get a sixteenth of the LDS budget).
__device__ __forceinline__ int wait_flag(int *p, int need, int &limit, int *status)
{
    int v = uniform(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    for (int polls = 0; v <= need; ++polls) {
        if (polls >= (limit >> 4)) {
            record_timeout(status);
            limit = 0;
            return 0x7fffffff;
        }
        __builtin_amdgcn_s_sleep(2);
        v = uniform(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    return v;
}

template <typename T, int K>
__device__ __forceinline__ void load_coef(T (&ca)[K], T (&cb)[K], uint64_t wp)
{
    ConstPairs<T> w = (ConstPairs<T>)wp;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        ca[q] = w[q].a;
        cb[q] = w[q].b;
    }
}

// Where a band-wave's columns come from and go to.
enum In : int { kInLds = 0, kInFresh = 1, kInWait = 2 };       // LDS channel / A (band 0) / A after a flag
enum Out : int { kOutLds = 0, kOutPublish = 1, kOutFinal = 2 };  // LDS channel / A + flag / A (last band)

// One band-wave.  The step loop is unrolled over one ring period of R steps
// so every register-ring slot, LDS slot and coefficient offset is a
// compile-time constant.
//
// Flow control is per column.  A consumer (LDS input) may read column c
// once produced > c; a producer (LDS output) may overwrite the slot of
// column c - RB once consumed > c - RB.  Both counters are re-read
// asynchronously every kPollEvery steps (an LDS load whose value is folded
// in the next time), so a wave only stalls when its neighbour really is
// behind; when it must wait it waits for extra headroom (kInSlack columns,
// kOutSlack slots) so the next wait is far away.  kInSlack + kOutSlack <=
// RB - 1 keeps the two sides from ever waiting on each other.
//
// Channel reads and writes are unconditional: columns outside [0, n)
// travel as data too (zeros, or past n possibly an older finite column of
// the same row, which only ever meets identity rotations), and A is
// protected by empty buffer descriptors.
template <typename T, int K, int ARITH, int IN, int OUT>
__device__ __forceinline__ void bandwave(const ChainArgs &a, int tile, int b, int w, char *lds_generic)
{
    constexpr int D = ChainGeom<K>::D;
    constexpr int R = ChainGeom<K>::R;
    constexpr int RB = R;
    constexpr int SLOT = kWave;  // elements per ring slot
    constexpr int kPollEvery = 4;
    constexpr int kInSlack = RB / 2;
    constexpr int kOutSlack = RB - 1 - kInSlack;
    static_assert(R % kPollEvery == 0, "poll cadence must divide the unroll");
    typedef __attribute__((address_space(3))) T lds_T;
    const int n = a.n;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t i0 = (int64_t)tile * kWave;
    const int64_t rows = a.m - i0 < kWave ? a.m - i0 : kWave;
    const uint32_t rowbytes = (uint32_t)(rows * (int64_t)sizeof(T));
    const int voff = lane * (int)sizeof(T);
    const uint64_t tileaddr = a.A + (uint64_t)i0 * sizeof(T);
    const uint64_t ldab = a.ldab;
    int limit = a.spin_limit;
    int *status = a.status;

    __attribute__((address_space(3))) char *lds = (__attribute__((address_space(3))) char *)lds_generic;
    lds_counter *cnt = (lds_counter *)lds;
    lds_T *rings = (lds_T *)(lds + kCounters * sizeof(int));
    lds_counter *prod_in = cnt + (w - 1), *cons_in = cnt + 16 + (w - 1);
    lds_counter *prod_out = cnt + w, *cons_out = cnt + 16 + w;
    lds_T *ring_in = rings + (w - 1) * RB * SLOT + lane;
    lds_T *ring_out = rings + w * RB * SLOT + lane;
    int *flag_in = a.flags + (int64_t)tile * a.nbands + (b - 1);
    int *flag_out = a.flags + (int64_t)tile * a.nbands + b;
    const int pubmask = a.publish - 1;

    // Input columns < in_known exist; the LDS consumer has read columns
    // < out_known.  in_poll / out_poll: counter values read asynchronously.
    int in_known = IN == kInFresh ? 0x7fffffff : 0;
    int out_known = 0;
    int in_poll = 0, out_poll = 0;

    T ring[R];
#pragma unroll
    for (int s = 0; s < R; ++s)
        ring[s] = T(0);

    // Fetch stream: next input column lc (at address lp in A).
    int lc = 0;
    uint64_t lp = tileaddr;
    auto fetch = [&](T &dst, int slot) {
        if constexpr (IN != kInFresh) {
            if (lc >= in_known) {
                const int need = (lc + kInSlack < n ? lc + kInSlack : n) - 1;
                if (lc < n) {
                    if constexpr (IN == kInLds)
                        in_known = wait_lds(prod_in, need, limit, status);
                    else
                        in_known = wait_flag(flag_in, need, limit, status);
                }
            }
        }
        if constexpr (IN == kInLds) {
            dst = ring_in[slot * SLOT];
            compiler_fence();
            *cons_in = lc + 1;
        } else {
            dst = buf_load<kPolicyDevice>(T(), make_rsrc(lp, lc < n ? rowbytes : 0u), voff);
            lp += ldab;
            opaque(lp);
        }
        ++lc;
        opaque_i(lc);
    };

#pragma unroll
    for (int c = 0; c <= D; ++c)
        fetch(ring[c], c % RB);

    // Output stream: next output column sc (at address sp in A).
    int sc = -(K - 1);
    uint64_t sp = tileaddr - (uint64_t)(K - 1) * ldab;

    constexpr uint64_t kStepBytes = K * sizeof(CoefPair<T>);
    uint64_t wblk = a.coef + (uint64_t)b * (a.steps + 1) * kStepBytes;
    T ca[K], cb[K];
    load_coef<T, K>(ca, cb, wblk);
    ConstScalars<T> sign = (ConstScalars<T>)a.sign;
    constexpr bool kSign = OUT == kOutFinal && ARITH == kLift;
    T sg = T(1);
    if constexpr (kSign)
        sg = sign[0];
    int blk = 0;

    for (int t0 = 0; t0 < a.steps; t0 += R) {
#pragma unroll
        for (int u = 0; u < R; ++u) {
            // Fold in the counters read kPollEvery steps ago and read them again.
            if (u % kPollEvery == 0) {
                if constexpr (IN == kInLds || IN == kInWait) {
                    const int v = uniform(in_poll);
                    in_known = v > in_known ? v : in_known;
                    if constexpr (IN == kInLds)
                        in_poll = *prod_in;
                    else
                        in_poll = __hip_atomic_load(flag_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                if constexpr (OUT == kOutLds) {
                    const int v = uniform(out_poll);
                    out_known = v > out_known ? v : out_known;
                    out_poll = *cons_out;
                }
            }
            // Next step's coefficients (the record after the last step is padding).
            T na[K], nb[K];
            load_coef<T, K>(na, nb, wblk + (uint64_t)(u + 1) * kStepBytes);
            // Column t+1+D replaces column t-K, finished last step.
            fetch(ring[(u + D + 1) % R], (u + D + 1) % RB);
#pragma unroll
            for (int q = 0; q < K; ++q)
                rotate<ARITH>(ring[(u - q + R) % R], ring[(u - q + 1 + R) % R], ca[q], cb[q]);
            // Column sc = t-K+1 has seen the whole band.
            T val = ring[(u - K + 1 + R) % R];
            if constexpr (OUT == kOutLds) {
                if (sc >= out_known + RB) {
                    // Slot of column sc - RB must have been read.
                    out_known = wait_lds(cons_out, sc - RB + kOutSlack, limit, status);
                }
                ring_out[((u - K + 1 + RB) % RB) * SLOT] = val;
                compiler_fence();
                *prod_out = sc + 1;
            } else {
                const bool valid = (unsigned)sc < (unsigned)n;
                if constexpr (kSign) {
                    val *= sg;
                    const int cn = sc + 1;
                    sg = sign[(unsigned)cn < (unsigned)n ? cn : 0];
                }
                if constexpr (OUT == kOutPublish)
                    buf_store<kPolicyDevice>(val, make_rsrc(sp, valid ? rowbytes : 0u), voff);
                else
                    buf_store(val, make_rsrc(sp, valid ? rowbytes : 0u), voff);
                sp += ldab;
                opaque(sp);
            }
            ++sc;
            opaque_i(sc);
            if constexpr (OUT == kOutPublish) {
                // Columns < sc - kPublishLag are complete once at most
                // kPublishLag vector memory operations are outstanding.
                if (u == R - 1) {
                    ++blk;
                    if ((blk & pubmask) == 0 && sc > kPublishLag && sc - kPublishLag < n) {
                        wait_vmem_at_most<kPublishLag>();
                        __hip_atomic_store(flag_out, sc - kPublishLag, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < K; ++q) {
                ca[q] = na[q];
                cb[q] = nb[q];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        wblk += R * kStepBytes;
        opaque(wblk);
    }
    if constexpr (OUT == kOutPublish) {
        wait_vmem_at_most<0>();
        __hip_atomic_store(flag_out, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename T, int K, int ARITH, int IN>
__device__ __forceinline__ void bandwave_out(const ChainArgs &a, int tile, int b, int w, char *lds,
                                             int out)
{
    if (out == kOutLds)
        bandwave<T, K, ARITH, IN, kOutLds>(a, tile, b, w, lds);
    else if (out == kOutPublish)
        bandwave<T, K, ARITH, IN, kOutPublish>(a, tile, b, w, lds);
    else
        bandwave<T, K, ARITH, IN, kOutFinal>(a, tile, b, w, lds);
}

template <typename T, int K, int ARITH>
__global__ __launch_bounds__(1024) void sweep_chain(ChainArgs a)
{
    extern __shared__ __align__(16) char lds[];
    // Counters start at 0; rings start as zeros so that a column slot read
    // before its first write holds a finite value.
    for (uint32_t i = threadIdx.x; i < a.lds_words; i += blockDim.x)
        ((int *)lds)[i] = 0;
    __syncthreads();
    const int w = uniform((int)(threadIdx.x >> 6));
    const int p = (int)blockIdx.x;
    const int g = a.remap ? (p & 7) * (a.nwg >> 3) + (p >> 3) : p;
    const int64_t idx = (int64_t)g * a.waves + w;
    const int64_t total = (int64_t)a.tiles * a.nbands;
    if (idx >= total)
        return;
    const int tile = (int)(idx / a.nbands);
    const int b = (int)(idx - (int64_t)tile * a.nbands);
    // The previous wave of this workgroup holds band b-1 of the same tile
    // exactly when b > 0; likewise the next wave holds band b+1.
    const int in = (w > 0 && b > 0) ? kInLds : (b == 0 ? kInFresh : kInWait);
    const int out = (w + 1 < a.waves && b + 1 < a.nbands) ? kOutLds
                    : (b + 1 < a.nbands ? kOutPublish : kOutFinal);
    if (in == kInLds)
        bandwave_out<T, K, ARITH, kInLds>(a, tile, b, w, lds, out);
    else if (in == kInFresh)
        bandwave_out<T, K, ARITH, kInFresh>(a, tile, b, w, lds, out);
    else
        bandwave_out<T, K, ARITH, kInWait>(a, tile, b, w, lds, out);
}

template <typename T, int K, int ARITH>
hipError_t go_chain(const Plan &p, T *A, const char *ws, hipStream_t st)
{
    ChainArgs a;
    a.A = (uint64_t)A;
    a.ldab = (uint64_t)p.lda * sizeof(T);
    a.m = p.m;
    a.n = (int)p.n;
    a.steps = p.steps;
    a.nbands = p.npass;
    a.tiles = (int)((p.m + kWave - 1) / kWave);
    a.waves = p.waves;
    a.nwg = p.nwg;
    a.remap = p.remap;
    a.publish = p.publish;
    a.spin_limit = p.spin_limit;
    a.lds_words = (uint32_t)(p.lds_bytes / 4);
    a.coef = (uint64_t)(ws + p.off_coef);
    a.sign = (uint64_t)(ws + p.off_sign);
    a.flags = (int *)(ws + p.off_flags);
    a.status = p.status;
    sweep_chain<T, K, ARITH><<<p.nwg, p.waves * kWave, p.lds_bytes, st>>>(a);
    return hipGetLastError();
}

template <typename T, int ARITH>
hipError_t chain_arith(const Plan &p, T *A, const char *ws, hipStream_t st)
{
    switch (p.band) {
    case 4: return go_chain<T, 4, ARITH>(p, A, ws, st);
    case 6: return go_chain<T, 6, ARITH>(p, A, ws, st);
    case 8: return go_chain<T, 8, ARITH>(p, A, ws, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t chain_t(const Plan &p, T *A, const char *ws, hipStream_t st)
{
    switch (p.arith) {
    case kExact: return chain_arith<T, kExact>(p, A, ws, st);
    case kFma: return chain_arith<T, kFma>(p, A, ws, st);
    case kLift: return chain_arith<T, kLift>(p, A, ws, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
const void *chain_kernel_fn(int band, int arith)
{
#define ROTSEQ_CHAIN_FN(KK, AA) (const void *)&sweep_chain<T, KK, AA>
    if (band == 4)
        return arith == kExact ? ROTSEQ_CHAIN_FN(4, kExact)
               : arith == kFma ? ROTSEQ_CHAIN_FN(4, kFma)
                               : ROTSEQ_CHAIN_FN(4, kLift);
    if (band == 6)
        return arith == kExact ? ROTSEQ_CHAIN_FN(6, kExact)
               : arith == kFma ? ROTSEQ_CHAIN_FN(6, kFma)
                               : ROTSEQ_CHAIN_FN(6, kLift);
    return arith == kExact ? ROTSEQ_CHAIN_FN(8, kExact)
           : arith == kFma ? ROTSEQ_CHAIN_FN(8, kFma)
                           : ROTSEQ_CHAIN_FN(8, kLift);
#undef ROTSEQ_CHAIN_FN
}

}  // namespace

int chain_unroll(int band)
{
    return band == 4 ? ChainGeom<4>::R : band == 6 ? ChainGeom<6>::R : ChainGeom<8>::R;
}

size_t chain_lds_bytes(int band, int waves, int esize)
{
    const int R = chain_unroll(band);
    return kCounters * sizeof(int) + (size_t)(waves > 1 ? waves - 1 : 0) * R * kWave * esize;
}

hipError_t chain_occupancy(int band, int arith, int esize, int waves, size_t lds, int *blocks)
{
    const void *fn = esize == 8 ? chain_kernel_fn<double>(band, arith) : chain_kernel_fn<float>(band, arith);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, waves * kWave, lds);
}

hipError_t launch_chain(const Plan &p, void *A, const void *ws, hipStream_t stream)
{
    if (p.esize == 8)
        return chain_t<double>(p, (double *)A, (const char *)ws, stream);
    return chain_t<float>(p, (float *)A, (const char *)ws, stream);
}

}  // namespace rotseq
