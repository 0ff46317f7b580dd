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
// between neighbours in a chain goes through an LDS ring of RB column slots,
// and the waves advance in lockstep groups of steps separated by workgroup
// barriers, each wave a fixed number of groups behind the one it reads
// from, so a slot is never read before it is written nor overwritten before
// it is read.  Where a chain crosses a workgroup
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
// Every wait on another workgroup is bounded: after `spin_limit` polls a wave
// records ROTSEQ_E_TIMEOUT in the status word and carries on with whatever
// data it has, so the grid always drains; every wave of a workgroup passes
// the same number of barriers.  All accesses stay in bounds whatever the
// data (buffer descriptors for A, ring indices modulo RB for LDS).
#include <type_traits>

#include "rotseq.h"
#include "rotseq_device.h"
#include "rotseq_internal.h"

namespace rotseq {
using namespace dev;
namespace {

// Geometry of the chain kernel.  A wave's register ring holds R = K + 1 + D
// columns, D being how many steps ahead a column is fetched: as far as the
// ring allows, from A (HBM latency) and from an LDS channel alike.  Each LDS
// channel has RB = 16 column slots.  The step loop is unrolled U = 16 steps,
// a multiple of every R and of RB, so every ring, slot and coefficient index
// in the body is a compile-time constant.
template <int K>
struct ChainGeom {
    static constexpr int U = 16;
    static constexpr int RB = 16;
    static constexpr int R_lds = K <= 6 ? 8 : 16;     // ring of LDS-fed waves
    static constexpr int R_glob = 16;                 // ring of A-fed waves
    static constexpr int D_lds = R_lds - K - 1;
    static constexpr int D_glob = R_glob - K - 1;
    static constexpr int G = 4;                       // steps per lockstep group
    // Groups between the starts of neighbouring waves of a chain segment:
    // the smallest lag for which every LDS column slot is written, read and
    // overwritten in three different groups, in that order.
    static constexpr int LG = K == 8 ? 5 : 3;
    // Groups from the start of a workgroup's wave that publishes through A to
    // the start of the wave in the next workgroup that reads it, so that the
    // reader rarely waits (a wait inside a lockstep group holds up its whole
    // workgroup): publication is per 16-column block, 16 columns behind the
    // newest store, and a group needs G + D_glob columns ahead, so the reader
    // trails by about 14 groups; 2 more cover the flag's latency.
    static constexpr int DG = 16;
    // Streaming launches (every workgroup holds whole chains, so nothing is
    // handed on through A; small k, where HBM bounds the sweep): the step
    // loop runs over H_deep blocks of U steps, an A-fed wave's ring holds
    // R_deep columns, twice as many loads in flight, and lockstep groups are
    // G_deep steps long, half the barriers, with LDS channels of RB_deep
    // slots and a lag of LG_deep groups (the smallest safe one for those).
    // (The DPP broadcasts tie a block to 16 steps.)
    static constexpr int H_deep = 2;
    static constexpr int R_deep = 32;
    static constexpr int G_deep = 8;
    static constexpr int RB_deep = 32;
    static constexpr int LG_deep = K == 8 ? 3 : 2;
    static_assert(K == 2 || K == 4 || K == 6 || K == 8, "band widths of the chain kernel");
    static_assert(D_lds >= 1 && U % R_lds == 0 && U % R_glob == 0 && U % RB == 0 && U % G == 0,
                  "geometry");
    static_assert((U * H_deep) % R_deep == 0 && (U * H_deep) % RB_deep == 0 && U % G_deep == 0,
                  "streaming geometry");
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
    int wait_bias;   // added to every flag wait's target (0; a test hook)
    uint32_t lds_words;  // dynamic LDS size in 4-byte words
    uint64_t coef;   // [nbands][steps + 1 + 8][K] coefficient pairs
    uint64_t sign;   // [n] final column signs (lifting arithmetic)
    int *flags;      // [tiles][nbands] published progress (columns)
    int *status;     // error word
};

// A producer publishes column c only once its store has completed; it waits
// for all but the newest kPublishLag stores, so it rarely waits at all.
constexpr int kPublishLag = 16;


// ---------------------------------------------------------------- DPP
//
// Coefficients live in VGPRs: one vector load brings the records of
// 16/K consecutive steps, lane l of every 16-lane row holding pair l mod 16
// of them (rotation q of the j-th step in lane j*K + q), and an FMA reads a
// pair broadcast across the row with the DPP row_newbcast source modifier.
// This keeps them off the scalar path (whose loads complete out of order, so
// they can only be prefetched one step ahead) and out of the SGPR file.

template <int Q>
__device__ __forceinline__ void fmac_bcast(double &x, double a, double y)
{
    // x += a[lane Q of this row] * y
    asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(x) : "v"(a), "v"(y), "n"(Q));
}
template <int Q>
__device__ __forceinline__ double bcast(double a)
{
    double r;
    asm("v_mov_b64_dpp %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf" : "=v"(r) : "v"(a), "n"(Q));
    return r;
}
// Rotation q of a step with its coefficient pair held in lane q of each row.
// row_newbcast is a 64-bit DPP mode: FP64 lifting reads the coefficients
// straight into its FMAs; the other FP64 modes broadcast them first; FP32
// broadcasts its (a, b) pair as one 64-bit value.  A DPP source must not
// have been written by a VALU instruction in the two preceding instructions
// (the compiler cannot see the DPP inside the asm), so every DPP source here
// is a register written by the coefficient load itself; tests scan the ISA.
template <int ARITH, int Q>
__device__ __forceinline__ void rotate_bcast(double &x, double &y, double a, double b)
{
    if constexpr (ARITH == kLift) {
        fmac_bcast<Q>(x, a, y);
        fmac_bcast<Q>(y, b, x);
        fmac_bcast<Q>(x, a, y);
    } else {
        rotate<ARITH>(x, y, bcast<Q>(a), bcast<Q>(b));
    }
}
// FP32: `pair` holds the loaded (a, b) bits of lane q.
template <int ARITH, int Q>
__device__ __forceinline__ void rotate_bcast_pair(float &x, float &y, double pair)
{
    const unsigned long long p = __builtin_bit_cast(unsigned long long, bcast<Q>(pair));
    rotate<ARITH>(x, y, __builtin_bit_cast(float, (unsigned)p), __builtin_bit_cast(float, (unsigned)(p >> 32)));
}

// All K lifting rotations of one step, FP64, in one asm block: rotation q
// acts on (x, y) = (column t-q, column t-q+1) = (c[q+1], c[q]), with its
// coefficients in lane OFF+q of each row of `a` and `b`.  One block per step
// keeps the compiler from padding every FMA pair with wait states (it must
// assume any asm operand may be a DPP source); inside the block the only
// DPP sources are `a` and `b`, written by the coefficient load, and plain
// VALU dependencies are interlocked by the hardware.  Operands: %0..%K the
// columns c[0..K] (only these: a further operand would have to be
// materialised every step), %[a], %[b], and the broadcast lanes %[lq].
#define ROTSEQ_FMAC(X, A, Y, L) "v_fmac_f64_dpp %" #X ", %[" #A "], %" #Y " row_newbcast:%[" #L "] row_mask:0xf bank_mask:0xf\n"
#define ROTSEQ_ROT(L, X, Y) ROTSEQ_FMAC(X, a, Y, L) ROTSEQ_FMAC(Y, b, X, L) ROTSEQ_FMAC(X, a, Y, L)
#define ROTSEQ_COEF(OFF) [a] "v"(a), [b] "v"(b), [l0] "n"(OFF), [l1] "n"(OFF + 1), [l2] "n"(OFF + 2), [l3] "n"(OFF + 3)
template <int K, int OFF>
__device__ __forceinline__ void lift_step(double (&c)[K + 1], double a, double b)
{
    static_assert(OFF + K <= 16, "broadcast lanes lie in one 16-lane row");
    if constexpr (K == 8)
        asm(ROTSEQ_ROT(l0, 1, 0) ROTSEQ_ROT(l1, 2, 1) ROTSEQ_ROT(l2, 3, 2) ROTSEQ_ROT(l3, 4, 3)
            ROTSEQ_ROT(l4, 5, 4) ROTSEQ_ROT(l5, 6, 5) ROTSEQ_ROT(l6, 7, 6) ROTSEQ_ROT(l7, 8, 7)
            : "+v"(c[0]), "+v"(c[1]), "+v"(c[2]), "+v"(c[3]), "+v"(c[4]), "+v"(c[5]), "+v"(c[6]),
              "+v"(c[7]), "+v"(c[8])
            : ROTSEQ_COEF(OFF), [l4] "n"(OFF + 4), [l5] "n"(OFF + 5), [l6] "n"(OFF + 6),
              [l7] "n"(OFF + 7));
    else if constexpr (K == 6)
        asm(ROTSEQ_ROT(l0, 1, 0) ROTSEQ_ROT(l1, 2, 1) ROTSEQ_ROT(l2, 3, 2) ROTSEQ_ROT(l3, 4, 3)
            ROTSEQ_ROT(l4, 5, 4) ROTSEQ_ROT(l5, 6, 5)
            : "+v"(c[0]), "+v"(c[1]), "+v"(c[2]), "+v"(c[3]), "+v"(c[4]), "+v"(c[5]), "+v"(c[6])
            : ROTSEQ_COEF(OFF), [l4] "n"(OFF + 4), [l5] "n"(OFF + 5));
    else if constexpr (K == 4)
        asm(ROTSEQ_ROT(l0, 1, 0) ROTSEQ_ROT(l1, 2, 1) ROTSEQ_ROT(l2, 3, 2) ROTSEQ_ROT(l3, 4, 3)
            : "+v"(c[0]), "+v"(c[1]), "+v"(c[2]), "+v"(c[3]), "+v"(c[4])
            : ROTSEQ_COEF(OFF));
    else
        asm(ROTSEQ_ROT(l0, 1, 0) ROTSEQ_ROT(l1, 2, 1)
            : "+v"(c[0]), "+v"(c[1]), "+v"(c[2])
            : [a] "v"(a), [b] "v"(b), [l0] "n"(OFF), [l1] "n"(OFF + 1));
}
#undef ROTSEQ_COEF
#undef ROTSEQ_ROT
#undef ROTSEQ_FMAC

template <int Q, int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (Q < N) {
        f(std::integral_constant<int, Q>{});
        static_for<Q + 1, N>(f);
    }
}

// Calls f(std::integral_constant<int, J>) for the J == j in [0, N).  In the
// unrolled step loop j is a constant, so a single call remains.
template <int N, int J = 0, typename F>
__device__ __forceinline__ void select_const(int j, F &&f)
{
    if constexpr (J < N) {
        if (j == J)
            f(std::integral_constant<int, J>{});
        else
            select_const<N, J + 1>(j, f);
    }
}

// One coefficient record lane: the pair (a, b) as raw bits.
template <typename T>
struct CoefLane;
template <>
struct CoefLane<double> {
    typedef unsigned int bits __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ bits load(__amdgpu_buffer_rsrc_t r, int voff, int soff)
    {
        return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    }
    static __device__ __forceinline__ double a(bits v)
    {
        return __builtin_bit_cast(double, (unsigned long long)v.x | ((unsigned long long)v.y << 32));
    }
    static __device__ __forceinline__ double b(bits v)
    {
        return __builtin_bit_cast(double, (unsigned long long)v.z | ((unsigned long long)v.w << 32));
    }
};
template <>
struct CoefLane<float> {
    typedef unsigned int bits __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ bits load(__amdgpu_buffer_rsrc_t r, int voff, int soff)
    {
        return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    }
    static __device__ __forceinline__ double pair(bits v) { return __builtin_bit_cast(double, v); }
};

// Where a band-wave's columns come from and go to.
enum In : int { kInLds = 0, kInFresh = 1, kInWait = 2 };       // LDS channel / A (band 0) / A after a flag
enum Out : int { kOutLds = 0, kOutPublish = 1, kOutFinal = 2 };  // LDS channel / A + flag / A (last band)

// One band-wave, unrolled over U steps (H blocks of U steps for the A
// streams of a streaming launch, DEEP).
//
// Flow control inside a workgroup is lockstep: the step loop is cut into
// groups of G steps, and every wave of the workgroup ends every group at the
// same barrier (group_barrier), after its LDS writes of the group have
// completed.  A wave at position `pos` of its chain segment (pos = 0 reads
// A; pos > 0 reads the LDS channel of the wave before it) starts LG*pos
// groups after the segment's first wave: one group for the prologue's
// fetches, then its steps.  With that lag every column slot is written in a
// strictly earlier group than the one that reads it, and read in a strictly
// earlier group than the one that overwrites it (ChainGeom::LG; checked by
// tests/test_lockstep_schedule.py for every band width).  A segment fed
// through A by the previous workgroup starts later still (segment_offset).
// `pre` idle groups come before the wave's prologue and `post` after its
// steps, so that every wave of the workgroup (idle ones included) passes the
// same number of barriers: the workgroup's largest `pre` + 1 + steps/G.
//
// Channel reads and writes are unconditional: columns outside [0, n)
// travel as data too (zeros, or past n possibly an older finite column of
// the same row, which only ever meets identity rotations), and A is
// protected by empty buffer descriptors.
template <typename T, int K, int ARITH, int IN, int OUT, bool DEEP>
__device__ __forceinline__ void bandwave(const ChainArgs &a, int tile, int b, int w, int pre, int post,
                                         char *lds_generic)
{
    using Geo = ChainGeom<K>;
    constexpr int U = Geo::U;
    constexpr int RB = DEEP ? Geo::RB_deep : Geo::RB;
    constexpr int G = DEEP ? Geo::G_deep : Geo::G;
    constexpr int R = IN == kInLds ? Geo::R_lds : DEEP ? Geo::R_deep : Geo::R_glob;
    constexpr int D = R - K - 1;
    constexpr int H = DEEP ? Geo::H_deep : 1;
    constexpr int UH = U * H;  // steps per trip of the step loop
    constexpr int SLOT = kWave;  // elements per ring slot
    static_assert(U % G == 0, "groups must tile the unroll");
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
    int timed_out = 0;

    lds_T *rings = (lds_T *)(__attribute__((address_space(3))) char *)lds_generic;
    lds_T *ring_in = rings + (w - 1) * RB * SLOT + lane;
    lds_T *ring_out = rings + w * RB * SLOT + lane;
    int *flag_in = a.flags + (int64_t)tile * a.nbands + (b - 1);
    int *flag_out = a.flags + (int64_t)tile * a.nbands + b;
    const int pubmask = a.publish - 1;

    // Wait for the wave's place in the workgroup's schedule.
    idle_groups(pre);

    // Input columns < in_known exist (A-fed waves after a flag wait; LDS-fed
    // waves rely on the schedule).  in_poll: the flag read one group early.
    int in_known = IN == kInWait ? 0 : 0x7fffffff;
    int in_poll = 0;

    T ring[R];
#pragma unroll
    for (int s = 0; s < R; ++s)
        ring[s] = T(0);

    // Fetch stream: next input column lc (at address lp in A).
    int lc = 0;
    uint64_t lp = tileaddr;
    auto ensure_in = [&](int cols) {  // the next `cols` fetches must exist
        if constexpr (IN == kInWait) {
            if (lc + cols > in_known && lc < n) {
                const int want = lc + cols;
                in_known = wait_flag(flag_in, (want < n ? want : n) - 1 + a.wait_bias, limit,
                                     timed_out);
            }
        }
    };
    auto fetch = [&](T &dst, int slot) {
        if constexpr (IN == kInLds) {
            dst = ring_in[slot * SLOT];
        } else {
            dst = buf_load<kPolicyDevice>(T(), make_rsrc(lp, lc < n ? rowbytes : 0u), voff);
            lp += ldab;
            opaque(lp);
        }
        ++lc;
    };

    // Prologue group: the first D+1 columns.
    ensure_in(D + 1);
#pragma unroll
    for (int c = 0; c <= D; ++c)
        fetch(ring[c], c % RB);
    opaque_i(lc);
    if constexpr (IN == kInWait)
        in_poll = __hip_atomic_load(flag_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    group_barrier();

    // Output stream: next output column sc (at address sp in A).
    int sc = -(K - 1);
    uint64_t sp = tileaddr - (uint64_t)(K - 1) * ldab;

    // Coefficient pipeline: one load brings the records of SPL consecutive
    // steps (lane l of each row: pair l mod 16 from the first step's record
    // on; lanes past SPL*K repeat the last pair and are never read).  NL
    // loads are in flight, so a step's records arrive kAhead steps early.
    // (FP32 with K = 4 takes two steps per load: with four, the compiler
    // re-packs the loaded pairs with VALU moves right before their DPP reads.)
    constexpr int SPL = sizeof(T) == 4 && K == 4 ? 2 : 16 / K;
    constexpr int NL = K == 2 ? 2 : 4;
    constexpr int kAhead = NL * SPL;
    static_assert(U % kAhead == 0, "coefficient ring must tile the unroll");
    static_assert(kAhead < kChainCoefPad, "look-ahead must stay inside the identity padding");
    using CL = CoefLane<T>;
    constexpr int kStepBytes = K * (int)sizeof(CoefPair<T>);
    const int q16 = lane & 15;
    const int cvoff = (q16 < SPL * K ? q16 : SPL * K - 1) * (int)sizeof(CoefPair<T>);
    const uint64_t cbase = a.coef + (uint64_t)b * (a.steps + kChainCoefPad) * kStepBytes;
    const __amdgpu_buffer_rsrc_t crs =
        make_rsrc(cbase, (uint32_t)((a.steps + kChainCoefPad) * kStepBytes));
    int coff = 0;  // byte offset of the record of step t0 (block base)
    typename CL::bits cf[NL], cur;
#pragma unroll
    for (int i = 0; i < NL; ++i)
        cf[i] = CL::load(crs, cvoff, i * SPL * kStepBytes);
    ConstScalars<T> sign = (ConstScalars<T>)a.sign;
    constexpr bool kSign = OUT == kOutFinal && ARITH == kLift;
    // FP64: the final signs of a block's 16 output columns come in with one
    // vector load per block (lane l of each row: column sc + l mod 16 of the
    // block; 0 outside [0, n), where stores are dropped anyway), a block
    // ahead, and each step broadcasts its column's sign with DPP.  Scalar
    // loads in the step loop would force full LDS waits (scalar loads
    // complete out of order), every step, in the wave that ends each chain.
    constexpr bool kSignV = kSign && sizeof(T) == 8;
    T sg = T(1);
    if constexpr (kSign && !kSignV)
        sg = sign[0];
    // The range check of a buffer access covers the vector offset only, so
    // the column offset (negative, hence out of range, for the first block's
    // leading lanes) lives in a VGPR.
    __amdgpu_buffer_rsrc_t srs;
    u32x2 sgn_cur, sgn_next;
    int svoff = 0;  // byte offset of this lane's column in the next block
    if constexpr (kSignV) {
        srs = make_rsrc(a.sign, (uint32_t)((int64_t)n * (int64_t)sizeof(T)));
        svoff = (-(K - 1) + (lane & 15)) * (int)sizeof(T);
        sgn_cur = __builtin_amdgcn_raw_buffer_load_b64(srs, svoff, 0, 0);
        svoff += U * (int)sizeof(T);
        sgn_next = __builtin_amdgcn_raw_buffer_load_b64(srs, svoff, 0, 0);
        svoff += U * (int)sizeof(T);
    }
    int blk = 0;
    // Column t-K+1 (ring position hu, step uu of its block of U) has seen the whole band: to the
    // next band's LDS ring, or to A (with its final sign in the last band).
    auto emit = [&](int hu, int uu) {
        T val = ring[(hu - K + 1 + UH) % R];
        if constexpr (OUT == kOutLds) {
            ring_out[((hu - K + 1 + UH) % RB) * SLOT] = val;
        } else {
            const int c = sc + (uu % G);
            const bool valid = (unsigned)c < (unsigned)n;
            if constexpr (kSignV) {
                select_const<U>(uu % U, [&](auto qc) {
                    val *= bcast<decltype(qc)::value>(__builtin_bit_cast(double, sgn_cur));
                });
            } else if constexpr (kSign) {
                val *= sg;
                const int cn = c + 1;
                sg = sign[(unsigned)cn < (unsigned)n ? cn : 0];
            }
            if constexpr (OUT == kOutPublish)
                buf_store<kPolicyDevice>(val, make_rsrc(sp, valid ? rowbytes : 0u), voff);
            else
                buf_store(val, make_rsrc(sp, valid ? rowbytes : 0u), voff);
            sp += ldab;
            opaque(sp);
        }
    };
    // Drain the prologue's loads once: the compiler's wait-count analysis
    // merges the loop entry with the back edge, and a load still in flight
    // from the prologue would make it wait for nearly every load at the top
    // of each group instead of only for the one whose data is used.
    wait_vmem_at_most<0>();

    for (int t0 = 0; t0 < a.steps; t0 += UH) {
#pragma unroll
      for (int h = 0; h < H; ++h) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int hu = h * U + u;  // ring position; u: step within the block
            if constexpr (IN == kInWait) {
                if (u % G == 0) {
                    // Fold in the flag read a group ago, make sure this group's
                    // G fetches exist, and re-read the flag for the next group.
                    const int v = uniform(in_poll);
                    in_known = v > in_known ? v : in_known;
                    ensure_in(G);
                    in_poll = __hip_atomic_load(flag_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            // Coefficients of this step (lanes OFF..OFF+K-1 of each row of
            // `cur`); a new record group replaces the one just taken, kAhead
            // steps ahead (records past the last step are identity padding).
            if (u % SPL == 0) {
                cur = cf[(u / SPL) % NL];
                cf[(u / SPL) % NL] = CL::load(crs, cvoff, coff + (u + kAhead) * kStepBytes);
            }
            // Column t+1+D replaces column t-K, finished last step.
            fetch(ring[(hu + D + 1) % R], (hu + D + 1) % RB);
            select_const<SPL>(u % SPL, [&](auto jc) {
                constexpr int OFF = decltype(jc)::value * K;
                if constexpr (sizeof(T) == 8 && ARITH == kLift) {
                    // c[j] = column t+1-j, j = 0..K.
                    double c[K + 1];
#pragma unroll
                    for (int j = 0; j <= K; ++j)
                        c[j] = ring[(hu + 1 - j + UH) % R];
                    lift_step<K, OFF>(c, CL::a(cur), CL::b(cur));
#pragma unroll
                    for (int j = 0; j <= K; ++j)
                        ring[(hu + 1 - j + UH) % R] = c[j];
                } else {
                    static_for<0, K>([&](auto qc) {
                        constexpr int q = decltype(qc)::value;
                        if constexpr (sizeof(T) == 8)
                            rotate_bcast<ARITH, OFF + q>(ring[(hu - q + UH) % R], ring[(hu - q + 1 + UH) % R],
                                                         CL::a(cur), CL::b(cur));
                        else
                            rotate_bcast_pair<ARITH, OFF + q>(ring[(hu - q + UH) % R],
                                                              ring[(hu - q + 1 + UH) % R], CL::pair(cur));
                    });
                }
            });
            emit(hu, u);
            if (u % G == G - 1) {
                sc += G;
                opaque_i(lc);
                opaque_i(sc);
                group_barrier();
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (kSignV) {
            sgn_cur = sgn_next;
            sgn_next = __builtin_amdgcn_raw_buffer_load_b64(srs, svoff, 0, 0);
            svoff += U * (int)sizeof(T);
        }
        coff += U * kStepBytes;
        opaque_i(coff);
        if constexpr (OUT == kOutPublish) {
            // Columns < sc - kPublishLag are complete once at most
            // kPublishLag vector memory operations are outstanding.
            ++blk;
            if ((blk & pubmask) == 0 && sc > kPublishLag && sc - kPublishLag < n) {
                wait_vmem_at_most<kPublishLag>();
                __hip_atomic_store(flag_out, sc - kPublishLag, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }
      }
    }
    if constexpr (OUT == kOutPublish) {
        wait_vmem_at_most<0>();
        __hip_atomic_store(flag_out, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // Pad the schedule to the workgroup's common barrier count.
    idle_groups(post);
    if (timed_out)
        record_timeout(a.status, timed_out);
}

template <typename T, int K, int ARITH, int IN, bool DEEP>
__device__ __forceinline__ void bandwave_out(const ChainArgs &a, int tile, int b, int w, int pre,
                                             int post, char *lds, int out)
{
    if (out == kOutLds)
        bandwave<T, K, ARITH, IN, kOutLds, DEEP>(a, tile, b, w, pre, post, lds);
    else if (out == kOutPublish)
        bandwave<T, K, ARITH, IN, kOutPublish, DEEP>(a, tile, b, w, pre, post, lds);
    else
        bandwave<T, K, ARITH, IN, kOutFinal, DEEP>(a, tile, b, w, pre, post, lds);
}

// Groups by which a chain segment that starts at band b0 is held back in its
// workgroup's lockstep schedule.  A segment with b0 > 0 starts at wave 0 and
// reads band b0-1 through A from the last wave of the previous workgroup,
// which is at position r-1 = min(W, b0)-1 of a segment starting at band
// b0-r; that wave starts LG*(r-1) groups after its own segment, and its
// output trails it by DG groups.  Hence, with b0 = q*W + r (1 <= r <= W),
// the offset is q*(LG*(W-1) + DG) + LG*(r-1) + DG.
template <int K>
__device__ __forceinline__ int segment_offset(int b0, int W)
{
    if (b0 <= 0)
        return 0;
    constexpr int LG = ChainGeom<K>::LG, DG = ChainGeom<K>::DG;
    const int r = (b0 - 1) % W + 1;
    const int q = (b0 - r) / W;
    return q * (LG * (W - 1) + DG) + LG * (r - 1) + DG;
}

// Workgroup g of a problem's chain grid: its waves take the (tile, band)
// units g*W .. g*W+W-1 in tile-major order.  DEEP: a streaming launch, in
// which W is a multiple of the band count, so that no unit reads or writes
// a hand-off through A.
template <typename T, int K, int ARITH, bool DEEP>
__device__ __forceinline__ void chain_workgroup(const ChainArgs &a, int g, char *lds)
{
    constexpr int LG = DEEP ? ChainGeom<K>::LG_deep : ChainGeom<K>::LG;
    constexpr int G = DEEP ? ChainGeom<K>::G_deep : ChainGeom<K>::G;
    const int w = uniform((int)(threadIdx.x >> 6));
    const int64_t total = (int64_t)a.tiles * a.nbands;
    // Idle groups before each wave's prologue: its segment's offset plus LG
    // per position.  The previous wave of this workgroup holds band b-1 of
    // the same tile exactly when b > 0, so a wave's segment starts min(w, b)
    // waves back.  Every wave computes the workgroup's largest one the same
    // way, which fixes the common barrier count.
    int pre = 0, max_pre = 0;
    for (int v = 0; v < a.waves; ++v) {
        const int64_t iv = (int64_t)g * a.waves + v;
        if (iv >= total)
            break;
        const int bv = (int)(iv % a.nbands);
        const int pv = v < bv ? v : bv;
        const int pre_v = segment_offset<K>(bv - pv, a.waves) + LG * pv;
        max_pre = pre_v > max_pre ? pre_v : max_pre;
        if (v == w)
            pre = pre_v;
    }
    const int64_t idx = (int64_t)g * a.waves + w;
    if (idx >= total) {
        // No unit: keep the workgroup's barrier count.
        idle_groups(max_pre + 1 + a.steps / G);
        return;
    }
    const int tile = (int)(idx / a.nbands);
    const int b = (int)(idx - (int64_t)tile * a.nbands);
    const int in = (w > 0 && b > 0) ? kInLds : (b == 0 ? kInFresh : kInWait);
    const int out = (w + 1 < a.waves && b + 1 < a.nbands) ? kOutLds
                    : (b + 1 < a.nbands ? kOutPublish : kOutFinal);
    const int post = max_pre - pre;
    if constexpr (DEEP) {
        if (in == kInWait || out == kOutPublish) {
            // A hand-off through A in a streaming launch (the host never
            // makes one): report the call as a failed hand-off wait and keep
            // the workgroup's barrier count.
            if (threadIdx.x % kWave == 0)
                record_timeout(a.status, kWaitFlag);
            idle_groups(max_pre + 1 + a.steps / G);
            return;
        }
        if (in == kInLds)
            bandwave_out<T, K, ARITH, kInLds, true>(a, tile, b, w, pre, post, lds, out);
        else
            bandwave_out<T, K, ARITH, kInFresh, true>(a, tile, b, w, pre, post, lds, out);
    } else {
        if (in == kInLds)
            bandwave_out<T, K, ARITH, kInLds, false>(a, tile, b, w, pre, post, lds, out);
        else if (in == kInFresh)
            bandwave_out<T, K, ARITH, kInFresh, false>(a, tile, b, w, pre, post, lds, out);
        else
            bandwave_out<T, K, ARITH, kInWait, false>(a, tile, b, w, pre, post, lds, out);
    }
}

// Zeroes the workgroup's LDS rings, so that a column slot read before its
// first write (only columns past the band's last output) holds a finite value.
__device__ __forceinline__ void zero_lds(char *lds, uint32_t words)
{
    for (uint32_t i = threadIdx.x; i < words; i += blockDim.x)
        ((int *)lds)[i] = 0;
    __syncthreads();
}

// DEEP: a streaming launch of at most kChainDeepWaves waves per workgroup
// (the bound leaves the deeper rings their registers).
template <typename T, int K, int ARITH, bool DEEP>
__global__ __launch_bounds__(DEEP ? kChainDeepWaves * kWave : 1024) void sweep_chain(ChainArgs a)
{
    extern __shared__ __align__(16) char lds[];
    zero_lds(lds, a.lds_words);
    const int p = (int)blockIdx.x;
    const int g = a.remap ? (p & 7) * (a.nwg >> 3) + (p >> 3) : p;
    chain_workgroup<T, K, ARITH, DEEP>(a, g, lds);
}

// A batch in one launch: workgroup ranges of the items follow each other in
// item order (longest chains first, so the dispatcher starts them early);
// a workgroup finds its item by binary search and runs as in sweep_chain.
// Workgroups still only wait for lower-numbered ones of their own item.
struct BatchChainArgs {
    const BatchItem *items;
    int count, waves, publish, spin_limit, wait_bias;
    uint32_t lds_words;
};

template <typename T, int K, int ARITH>
__global__ __launch_bounds__(1024) void sweep_chain_batch(BatchChainArgs ba)
{
    extern __shared__ __align__(16) char lds[];
    zero_lds(lds, ba.lds_words);
    const int64_t g = blockIdx.x;
    int lo = 0, hi = ba.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ba.items[mid].off_wg <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BatchItem &it = ba.items[lo];
    ChainArgs a;
    a.A = (uint64_t)it.A;
    a.ldab = (uint64_t)it.lda * sizeof(T);
    a.m = it.m;
    a.n = (int)it.n;
    a.steps = it.steps;
    a.nbands = it.npass;
    a.tiles = it.tiles;
    a.waves = ba.waves;
    a.nwg = 0;
    a.remap = 0;
    a.publish = ba.publish;
    a.spin_limit = ba.spin_limit;
    a.wait_bias = ba.wait_bias;
    a.lds_words = ba.lds_words;
    a.coef = (uint64_t)it.coef;
    a.sign = (uint64_t)it.sign;
    a.flags = it.flags;
    a.status = it.status;
    chain_workgroup<T, K, ARITH, false>(a, (int)(g - it.off_wg), lds);
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
    a.wait_bias = p.wait_bias;
    a.lds_words = (uint32_t)(p.lds_bytes / 4);
    a.coef = (uint64_t)(ws + p.off_coef);
    a.sign = (uint64_t)(ws + p.off_sign);
    a.flags = (int *)(ws + p.off_flags);
    a.status = p.status;
    if (p.deep)
        sweep_chain<T, K, ARITH, true><<<p.nwg, p.waves * kWave, p.lds_bytes, st>>>(a);
    else
        sweep_chain<T, K, ARITH, false><<<p.nwg, p.waves * kWave, p.lds_bytes, st>>>(a);
    return hipGetLastError();
}

template <typename T, int K, int ARITH>
hipError_t go_chain_batch(const BatchLaunch &b, hipStream_t st)
{
    BatchChainArgs a;
    a.items = b.items;
    a.count = b.count;
    a.waves = b.waves;
    a.publish = b.publish;
    a.spin_limit = b.spin_limit;
    a.wait_bias = b.wait_bias;
    a.lds_words = (uint32_t)(b.lds_bytes / 4);
    sweep_chain_batch<T, K, ARITH><<<(unsigned)b.nwg, b.waves * kWave, b.lds_bytes, st>>>(a);
    return hipGetLastError();
}

template <typename T, int ARITH>
hipError_t chain_batch_arith(const BatchLaunch &b, hipStream_t st)
{
    switch (b.band) {
    case 4: return go_chain_batch<T, 4, ARITH>(b, st);
    case 6: return go_chain_batch<T, 6, ARITH>(b, st);
    case 8: return go_chain_batch<T, 8, ARITH>(b, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t chain_batch_t(const BatchLaunch &b, hipStream_t st)
{
    switch (b.arith) {
    case kExact: return chain_batch_arith<T, kExact>(b, st);
    case kFma: return chain_batch_arith<T, kFma>(b, st);
    case kLift: return chain_batch_arith<T, kLift>(b, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int ARITH>
hipError_t chain_arith(const Plan &p, T *A, const char *ws, hipStream_t st)
{
    switch (p.band) {
    case 2: return go_chain<T, 2, ARITH>(p, A, ws, st);
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
const void *chain_kernel_fn(int band, int arith, bool batch, bool deep)
{
#define ROTSEQ_CHAIN_FN(KK, AA)                                                                    \
    (batch  ? (const void *)&sweep_chain_batch<T, KK, AA>                                          \
     : deep ? (const void *)&sweep_chain<T, KK, AA, true>                                          \
            : (const void *)&sweep_chain<T, KK, AA, false>)
    if (band == 2) {  // single calls only (no batch kernel for bands of 2)
        if (batch)
            return nullptr;
        const bool e = arith == kExact, f = arith == kFma;
        return deep ? (e   ? (const void *)&sweep_chain<T, 2, kExact, true>
                       : f ? (const void *)&sweep_chain<T, 2, kFma, true>
                           : (const void *)&sweep_chain<T, 2, kLift, true>)
                    : (e   ? (const void *)&sweep_chain<T, 2, kExact, false>
                       : f ? (const void *)&sweep_chain<T, 2, kFma, false>
                           : (const void *)&sweep_chain<T, 2, kLift, false>);
    }
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

int chain_unroll(int band, bool deep)
{
    (void)band;
    return ChainGeom<8>::U * (deep ? ChainGeom<8>::H_deep : 1);
}

size_t chain_lds_bytes(int band, int waves, int esize, bool deep)
{
    (void)band;
    // at least one word, so that the zeroing loop has a valid extent
    const size_t slots = deep ? ChainGeom<8>::RB_deep : ChainGeom<8>::RB;
    const size_t rings = (size_t)(waves > 1 ? waves - 1 : 0) * slots * kWave * esize;
    return rings > 0 ? rings : 4;
}

hipError_t chain_occupancy(int band, int arith, int esize, int waves, size_t lds, int *blocks,
                           bool batch, bool deep)
{
    const void *fn = esize == 8 ? chain_kernel_fn<double>(band, arith, batch, deep)
                                : chain_kernel_fn<float>(band, arith, batch, deep);
    if (fn == nullptr)
        return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, waves * kWave, lds);
}

hipError_t launch_chain_batch(const BatchLaunch &b, hipStream_t stream)
{
    if (b.count <= 0 || b.nwg <= 0)
        return hipSuccess;
    if (b.esize == 8)
        return chain_batch_t<double>(b, stream);
    return chain_batch_t<float>(b, stream);
}

hipError_t launch_chain(const Plan &p, void *A, const void *ws, hipStream_t stream)
{
    if (p.esize == 8)
        return chain_t<double>(p, (double *)A, (const char *)ws, stream);
    return chain_t<float>(p, (float *)A, (const char *)ws, stream);
}

}  // namespace rotseq
