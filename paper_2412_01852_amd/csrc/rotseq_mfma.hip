// Sweep on FP64 matrix instructions (v_mfma_f64_16x16x4f64): a band of 8
// sequences is applied 8 wavefront steps at a time as dense 16 x 16 window
// matrices, the accumulate-then-multiply form of Section 8 of the paper
// (there done with a BLAS GEMM).
//
// Windows.  Band beta (sequences 8*beta .. 8*beta+7) applies at step t the
// rotations (t-q, 8*beta+q), q = 0..7 (Section 1.1).  Window w holds steps
// 8w+7 .. 8w+14, which touch only the 16 columns 8w .. 8w+15; their
// product is one orthogonal 16 x 16 matrix Q(beta, w), prepared once per
// call by `mfma_prep_q` for w = -1 .. nwin-1, nwin = ceil(n/8).  With X the
// 16 window columns of a row tile, the window is X <- X Q.  Afterwards
// columns 8w .. 8w+7 (block w) are final for the band, and columns 8w+8 ..
// 8w+15 stay "in flight" into window w+1, whose new columns are block w+1
// of the band's input.  Blocks never straddle column 0, so a lane's offset
// within a block is the same for every block.
// The windows do (16^2 / (3*8*8)) = 4/3 times the counted 6 flops per
// rotation and row.
//
// Matrix-instruction layout.  The product is taken transposed,
// D^T = Q^T X^T, with 16 rows of A as the N dimension.  The B operand
// (X^T, 4 window columns per instruction, "slab" s) holds column 4s + l/16
// of row l%16 in lane l; the result holds column 4e + l/16 of row l%16 in
// element e of lane l.  So result element e is exactly the B operand of
// slab e in the next product: the in-flight columns (elements 2, 3) are the
// next window's slabs 0, 1, and the finished block (elements 0, 1) is the
// next band's slabs 2, 3, with no data movement between lanes.  A wave
// therefore chains NB bands in registers, and hands its last band's blocks
// to the next wave through an LDS ring whose slots are lane-local.
//
// Schedule.  In wave-local super-step sp, band i runs window sp-1-2i: it
// takes band i-1's block finished one super-step earlier, so the bands of
// a super-step are independent.  The last band runs first, and its
// finished block is stored to A (or the ring) while the other bands'
// products execute; every memory operation of the super-step sits between
// two products (StepOps), so the matrix pipeline never waits for an issue.
//
// Work decomposition.  A wave owns R row blocks of 16 rows (a tile) and a
// chunk of NB consecutive bands; the 4 waves of a workgroup hold 4
// consecutive chunks of one tile's chain (a segment); a chain longer than
// 4 chunks continues in the next workgroup through A and a progress flag,
// as in the vector chain kernel.  The loads of A (the first wave's input)
// and the stores (the last wave's output) are shared by all four waves,
// row block by row block, through an LDS stage and the last wave's ring.
// Super-steps are separated by a workgroup barrier; wave j starts
// 4*ceil((2NB+3)/4) super-steps after wave j-1 and a later segment
// `seg_delay` super-steps after the previous one, so every block is
// produced at least one super-step before it is read (checked by
// tests/test_mfma_model.py).  All loop-carried register indices are
// compile-time: offsets are multiples of the unroll of 4.
//
// Edges.  Columns outside [0, n) are zeros (buffer-descriptor range
// checks) and only ever meet identity rotations; rows past m are computed
// on whatever the loads return (rows never mix: each is one N index of the
// products) and never stored.
#include "rotseq.h"
#include "rotseq_device.h"
#include "rotseq_internal.h"

namespace rotseq {
using namespace dev;
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kSeq = 8;    // sequences per band = steps per window
constexpr int kWin = 16;   // window width
constexpr int kUnroll = 4; // super-steps per loop body (ring depths)
constexpr int kQBytes = 64 * 4 * 8;  // one window matrix in operand layout

struct MfmaArgs {
    uint64_t A;      // address of A(0,0)
    uint64_t ldab;   // column stride of A in bytes
    int64_t m;
    int n;
    int nwin;        // windows -1 .. nwin-1 per band
    int nchunks;     // band chunks of one tile's chain
    int nseg;        // workgroups per tile chain
    int waves;       // waves (chunks) per workgroup
    int seg_delay;   // extra super-steps of each later segment
    int nwg;
    int remap;       // 1: consecutive workgroups on one XCD
    int spin_limit;
    int wait_bias;
    uint64_t q;      // [band][nwin+3][64 lanes][4 slabs] window matrices -2 .. nwin (ends zero)
    int *flags;      // [tile][seg][32] blocks published by the segment (first int of 128 bytes)
    int *status;
};

// Waves per workgroup (one per SIMD); a workgroup's waves also share the
// loads and stores of A.
constexpr int kWaves = 4;
// Super-steps between a flag poll and the use of its value (the poll of
// super-step u is read at u of the next trip round the unrolled loop).
constexpr int kPollLag = kUnroll;
// Super-steps between storing a block to A and the wait that covers those
// stores in every wave; the block is published one super-step later.
constexpr int kPubWait = 2;
// Super-steps between publishing a block and a poll sure to see it.
constexpr int kFlagMargin = 2;

template <int NB>
struct MfmaGeom {
    static_assert(NB >= 1 && NB <= 3, "bands per wave");
    // Super-steps between the starts of neighbouring waves: the last band
    // finishes block v at wave-local super-step v + 2NB - 1 and the next
    // wave's first band reads it at its super-step v.
    static constexpr int kStride = 4 * ((2 * NB + 3) / 4);
    // The four ring slots are rewritten four blocks later, after the read.
    static_assert(2 * NB - 1 + kUnroll > kStride, "ring slot reuse");
    // Super-steps from finishing block v (at v + 2NB - 1) to publishing it.
    static constexpr int kPubOff = 2 * NB + kPubWait + 1;
};

// One super-step of a wave: 4*NB*R products, the last band's first, with
// its memory operations between them (StepOps::kind of position k follows
// product k; positions past the last product follow it):
//   vector memory: the flag poll, 2*kSlots loads of input block sp+3 (this
//   wave's row blocks), 2*NB loads of window matrices, 2*kSlots stores of
//   the finished block of the super-step before (this wave's row blocks),
//   and after the products one flag store;
//   LDS: before the products, the first band's input (R reads), the block
//   to store (kSlots reads) and the input loaded two super-steps ago
//   (kSlots writes); among the products, the last band's finished block
//   into this wave's ring (R writes, two products after their row's last
//   product).
// Every wave issues the same vector memory operations in every super-step
// (a role it does not have gets an empty descriptor: loads return 0,
// stores are dropped), so no branch surrounds one and the compiler's wait
// counts are exact; the publication wait counts this sequence.
template <int NB, int R>
struct StepOps {
    static constexpr int kSlots = (R + kWaves - 1) / kWaves;  // row blocks per wave
    static constexpr int kProducts = 4 * NB * R;
    static constexpr int kPoll = 0;
    static constexpr int kLoad = 1;                     // 2*kSlots
    static constexpr int kQ = kLoad + 2 * kSlots;       // 2*NB
    static constexpr int kStore = kQ + 2 * NB;          // 2*kSlots
    static constexpr int kRing = (kStore + 2 * kSlots > 3 * R + 2) ? kStore + 2 * kSlots : 3 * R + 2;  // R
    static constexpr int kEnd = kRing + R;
    static constexpr int kPerStep = 1 + 2 * kSlots + 2 * NB + 2 * kSlots + 1;
    // vector memory operations issued after the stores of super-step s up
    // to the end of super-step s + kPubWait
    static constexpr int kAfterStores = 1 + kPubWait * kPerStep;
    static_assert(kAfterStores < 64, "publication count");
};

template <int NB, int R>
__global__ __launch_bounds__(kWaves * kWave, 1) void sweep_mfma(MfmaArgs a)
{
    using Ops = StepOps<NB, R>;
    using Geom = MfmaGeom<NB>;
    constexpr int kStride = Geom::kStride;
    constexpr int kS = Ops::kSlots;
    constexpr int kBlk = R * 64 * 2;  // doubles of one block (a ring or stage slot)
    extern __shared__ __align__(16) char lds_raw[];
    typedef __attribute__((address_space(3))) double lds_f64;
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) f64x2 lds_f64x2;
    // [kWaves rings + 1 stage][4 slots][R][64 lanes][2]
    lds_f64 *lds = (lds_f64 *)(__attribute__((address_space(3))) char *)lds_raw;

    const int lane = threadIdx.x & 63;
    const int g4 = lane >> 4;
    const int wv = uniform((int)(threadIdx.x >> 6));
    const int p = (int)blockIdx.x;
    const int g = a.remap ? (p & 7) * (a.nwg >> 3) + (p >> 3) : p;
    const int tile = g / a.nseg;
    const int seg = g - tile * a.nseg;
    const int chunk = seg * kWaves + wv;
    const int active = a.nchunks - seg * kWaves < kWaves ? a.nchunks - seg * kWaves : kWaves;
    const int nwin = a.nwin;
    const int pre = kUnroll + seg * a.seg_delay;
    const int off = pre + wv * kStride;
    const int off_out = pre + (active - 1) * kStride;
    const int T = (pre + (kWaves - 1) * kStride + 2 * NB + nwin + kUnroll - 1) & ~(kUnroll - 1);
    const bool in_wait = seg > 0;
    const bool publish = seg * kWaves + active < a.nchunks;

    // LDS starts zeroed: a wave reads ring and stage slots before they are
    // first written (the products there use zero window matrices, and 0 * x
    // is 0 only for finite x).
    for (int x = (int)threadIdx.x; x < (kWaves + 1) * kUnroll * kBlk; x += (int)blockDim.x)
        lds[x] = 0.0;
    __syncthreads();

    // This wave's row blocks for loads and stores: r = wv + kWaves*i.  Byte
    // offset of (row, column 8v + g4 + 4e) from column 8v; rows past m and
    // row blocks past R get an offset past every descriptor's range (the
    // planner keeps 8 columns of A below 2^30 bytes).
    const int64_t row0 = (int64_t)tile * R * 16 + (lane & 15);
    int voff[kS][2];
    int slot_r[kS];  // row block in a slot, clamped to R-1 for reads
#pragma unroll
    for (int i = 0; i < kS; ++i) {
        const int r = wv + kWaves * i;
        slot_r[i] = r < R ? r : R - 1;
        const bool ok = r < R && row0 + 16 * r < a.m;
        const uint32_t ro = ok ? (uint32_t)((row0 + 16 * r) * 8) : 0x80000000u;
#pragma unroll
        for (int e = 0; e < 2; ++e)
            voff[i][e] = (int)(ro + (uint32_t)((g4 + 4 * e) * a.ldab));
    }

    // Window matrices of this wave's bands (none for a wave past the last
    // chunk): [band][window -2 .. nwin][64 lanes][4 doubles], the first and
    // last zero; a band's window w is read at scalar offset
    // (band * (nwin+3) + clamp(w, -2, nwin) + 2) * kQBytes.
    const int qwin = nwin + 3;
    const __amdgpu_buffer_rsrc_t qrs = make_rsrc(
        a.q + (uint64_t)(chunk * NB) * (uint64_t)qwin * kQBytes,
        chunk < a.nchunks ? (uint32_t)(NB * qwin * kQBytes) : 0u);
    const int qvoff = lane * 32;

    int *flag_in = a.flags + ((int64_t)tile * a.nseg + (seg - 1)) * kMfmaFlagStride;
    int *flag_out = a.flags + ((int64_t)tile * a.nseg + seg) * kMfmaFlagStride;
    const __amdgpu_buffer_rsrc_t flag_in_rs = make_rsrc((uint64_t)flag_in, in_wait ? 4u : 0u);
    int limit = a.spin_limit, timed_out = 0, known = 0;
    int polled[kUnroll] = {0, 0, 0, 0};

    // First band's input: the stage (first wave) or the previous wave's ring.
    lds_f64 *const stage = lds + (int64_t)kWaves * kUnroll * kBlk;
    const lds_f64x2 *nin_src = (const lds_f64x2 *)(wv == 0 ? stage : lds + (int64_t)(wv - 1) * kUnroll * kBlk) + lane;
    lds_f64x2 *ring_out = (lds_f64x2 *)(lds + (int64_t)wv * kUnroll * kBlk) + lane;
    const lds_f64x2 *ring_last = (const lds_f64x2 *)(lds + (int64_t)(active - 1) * kUnroll * kBlk) + lane;
    lds_f64x2 *stage_w = (lds_f64x2 *)stage + lane;

    // Blocks loaded (tt + 3) and stored (t - off_out - 2NB) in the coming
    // super-step, with their first columns' addresses.
    const uint64_t blk_bytes = (uint64_t)kSeq * a.ldab;
    const uint32_t full_bytes = (uint32_t)blk_bytes;
    const uint32_t last_bytes = (uint32_t)((uint64_t)(a.n - kSeq * (nwin - 1)) * a.ldab);
    int in_v = 3 - pre, out_v = -off_out - 2 * NB;
    uint64_t in_base = a.A + (uint64_t)(int64_t)in_v * blk_bytes;
    uint64_t out_base = a.A + (uint64_t)(int64_t)out_v * blk_bytes;
    // Flag store of a super-step: real only in the first wave of a
    // publishing workgroup, for blocks 0 .. nwin-1.
    const __amdgpu_buffer_rsrc_t flag_on = make_rsrc((uint64_t)flag_out, publish && wv == 0 ? 4u : 0u);
    const __amdgpu_buffer_rsrc_t flag_off = make_rsrc((uint64_t)flag_out, 0u);
    int wp = -off_out - Geom::kPubOff;

    f64x4 D[2][NB][R];
#pragma unroll
    for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int r = 0; r < R; ++r)
                D[b2][i][r] = f64x4{0.0, 0.0, 0.0, 0.0};
    double IN[kUnroll][kS][2];  // this wave's part of input block v, slot v & 3
    double Qr[kUnroll][NB][4];  // window matrices, 3 ahead
#pragma unroll
    for (int x = 0; x < kUnroll; ++x) {
#pragma unroll
        for (int i = 0; i < kS; ++i)
            IN[x][i][0] = IN[x][i][1] = 0.0;
#pragma unroll
        for (int i = 0; i < NB; ++i)
            Qr[x][i][0] = Qr[x][i][1] = Qr[x][i][2] = Qr[x][i][3] = 0.0;
    }

    for (int t = 0; t < T; t += kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int tt = t + u - pre;  // workgroup-local super-step; tt % 4 == u % 4
            const int sp = t + u - off;  // wave-local super-step;      sp % 4 == u % 4
            const int cur = u & 1, prv = cur ^ 1;
            // 1. A later segment loads input block tt+3 once the previous
            // segment has published it: the poll of kPollLag super-steps
            // ago normally says so; otherwise wait here.
            if (in_wait) {
                const int v = tt + 3;
                const int need = (v + 1 < nwin ? v + 1 : nwin) + a.wait_bias;
                const int seen = uniform(polled[u]);
                known = known > seen ? known : seen;
                if (known < need)
                    known = wait_flag(flag_in, need - 1, limit, timed_out);
            }
            // 2. Descriptors of the super-step (blocks outside 0 .. nwin-1
            // are empty; block nwin-1 may be partial).
            const __amdgpu_buffer_rsrc_t in_rs = make_rsrc(in_base, (uint32_t)in_v < (uint32_t)(nwin - 1) ? full_bytes
                                                                    : in_v == nwin - 1 ? last_bytes : 0u);
            const __amdgpu_buffer_rsrc_t out_rs = make_rsrc(out_base, (uint32_t)out_v < (uint32_t)(nwin - 1) ? full_bytes
                                                                      : out_v == nwin - 1 ? last_bytes : 0u);
            in_v += 1;
            out_v += 1;
            in_base += blk_bytes;
            out_base += blk_bytes;
            int qsoff[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                int wq = sp + 2 - 2 * i;  // band i's window three super-steps on
                wq = wq < -2 ? -2 : (wq > nwin ? nwin : wq);
                qsoff[i] = uniform((i * qwin + wq + 2) * kQBytes);
            }
            // 3. LDS before the products: the first band's input block sp,
            // the block to store, and the stage of input block tt+1.
            f64x2 nin[R];
#pragma unroll
            for (int r = 0; r < R; ++r)
                nin[r] = nin_src[(u * R + r) * 64];
            f64x2 outv[kS];
#pragma unroll
            for (int i = 0; i < kS; ++i)
                outv[i] = ring_last[((((u - 2 * NB) & 3) * R) + slot_r[i]) * 64];
#pragma unroll
            for (int i = 0; i < kS; ++i)
                if (wv + kWaves * i < R)
                    stage_w[(((u + 1) & 3) * R + wv + kWaves * i) * 64] = f64x2{IN[(u + 1) & 3][i][0], IN[(u + 1) & 3][i][1]};
            compiler_fence();
            __builtin_amdgcn_sched_barrier(0);

            // Memory operation k of the super-step (compile-time k).
            auto memop = [&](const int k) {
                if (k == Ops::kPoll) {
                    polled[u] = (int)__builtin_amdgcn_raw_buffer_load_b32(flag_in_rs, 0, 0, kPolicyDevice);
                } else if (k >= Ops::kLoad && k < Ops::kQ) {
                    const int i = (k - Ops::kLoad) >> 1, e = (k - Ops::kLoad) & 1;
                    IN[(u + 3) & 3][i][e] = buf_load<kPolicyDevice>(double(), in_rs, voff[i][e]);
                } else if (k >= Ops::kQ && k < Ops::kStore) {
                    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
                    const int i = (k - Ops::kQ) >> 1, h = (k - Ops::kQ) & 1;
                    const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(qrs, qvoff + 16 * h, qsoff[i], kPolicyL2);
                    Qr[(u + 3) & 3][i][2 * h] = __builtin_bit_cast(double, (unsigned long long)q.x | ((unsigned long long)q.y << 32));
                    Qr[(u + 3) & 3][i][2 * h + 1] = __builtin_bit_cast(double, (unsigned long long)q.z | ((unsigned long long)q.w << 32));
                } else if (k >= Ops::kStore && k < Ops::kStore + 2 * kS) {
                    const int i = (k - Ops::kStore) >> 1, e = (k - Ops::kStore) & 1;
                    buf_store<kPolicyDevice>(e == 0 ? outv[i].x : outv[i].y, out_rs, voff[i][e]);
                } else if (k >= Ops::kRing && k < Ops::kEnd) {
                    const int r = k - Ops::kRing;
                    const f64x4 &d = D[cur][NB - 1][r];
                    ring_out[((((u - 2 * NB + 1) & 3) * R) + r) * 64] = f64x2{d.x, d.y};
                }
            };

            // 4. Products, last band first: band i runs window sp-1-2i on
            // its own in-flight columns and band i-1's block of the last
            // super-step.  Outside the band's windows the window matrix is
            // zero, so the band's state before its first window and what it
            // passes on after its last one are zero.
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) {
                const int i = NB - 1 - bi;
                const int ip = i > 0 ? i - 1 : 0;
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        double b;
                        if (s == 0)
                            b = D[prv][i][r].z;
                        else if (s == 1)
                            b = D[prv][i][r].w;
                        else if (i == 0)
                            b = s == 2 ? nin[r].x : nin[r].y;
                        else
                            b = s == 2 ? D[prv][ip][r].x : D[prv][ip][r].y;
                        D[cur][i][r] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            Qr[u][i][s], b, s == 0 ? f64x4{0.0, 0.0, 0.0, 0.0} : D[cur][i][r], 0, 0, 0);
                        memop((bi * 4 + s) * R + r);
                        __builtin_amdgcn_sched_barrier(0);
                    }
            }
#pragma unroll
            for (int k = Ops::kProducts; k < Ops::kEnd; ++k) {
                memop(k);
                __builtin_amdgcn_sched_barrier(0);
            }
            // 5. Publication: the first wave publishes the block whose
            // stores every wave covered with its wait of the last
            // super-step; every wave covers the stores of kPubWait
            // super-steps ago.
            compiler_fence();
            {
                __builtin_amdgcn_raw_buffer_store_b32((unsigned)(wp + 1), (uint32_t)wp < (uint32_t)nwin ? flag_on : flag_off,
                                                      0, 0, kPolicyDevice);
                ++wp;
                if (publish)
                    wait_vmem_at_most<Ops::kAfterStores>();
            }
            // 6. LDS writes of this super-step are complete; all waves meet.
            group_barrier();
        }
    }
    if (publish) {
        wait_vmem_at_most<0>();
        group_barrier();
        if (wv == 0)
            __hip_atomic_store(flag_out, nwin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (timed_out)
        record_timeout(a.status, timed_out);
}

// Window matrices: a block of 64 threads builds 4 consecutive windows of
// one band (thread 16*wl + r: row r of window wl).  The block first stages
// the 256 (c, s) pairs its windows use in LDS, loaded coalesced (sequence
// q, columns 8*w0+7-q .. 8*w0+38-q), identity pairs outside the problem;
// then every thread applies its window's rotations, in wavefront order, to
// e_r (reading the pairs as LDS broadcasts) and scatters the row to the
// operand layout: lane l, slab s holds Q[4s + l/16][l%16].  Windows -2 and
// nwin are zero.
constexpr int kPrepWins = 4;  // windows per block

// Also zeroes the sweep's progress flags (flag_words ints), spread over the
// launch's threads.
template <typename T>
__global__ __launch_bounds__(64) void mfma_prep_q(const T *__restrict__ C, int64_t ldc, const T *__restrict__ S, int64_t lds,
                            int n, int64_t k, int nbands, int nwin, double *__restrict__ q,
                            int *__restrict__ flags, int64_t flag_words)
{
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    __shared__ f64x2 cs[kSeq][kPrepWins * kSeq];  // [q][column - (8*w0 + 7 - q)]
    const int qwin = nwin + 3;
    const int per_band = (qwin + kPrepWins - 1) / kPrepWins;
    const int64_t band = blockIdx.x / per_band;
    const int wi0 = (int)(blockIdx.x - band * per_band) * kPrepWins;  // first window index (w = wi - 2)
    const int tid = (int)threadIdx.x;
    for (int64_t i = (int64_t)blockIdx.x * 64 + tid; i < flag_words; i += (int64_t)gridDim.x * 64)
        flags[i] = 0;
#pragma unroll
    for (int x = 0; x < kSeq * kPrepWins * kSeq / 64; ++x) {
        const int e = tid + 64 * x;
        const int qq = e / (kPrepWins * kSeq), jj = e % (kPrepWins * kSeq);
        const int64_t j = (int64_t)kSeq * (wi0 - 2) + kSeq - 1 - qq + jj;
        const int64_t pp = band * kSeq + qq;
        const bool ok = j >= 0 && j <= n - 2 && pp < k;
        const int64_t jc = ok ? j : 0, pc = ok ? pp : 0;
        const double cl = (double)C[jc + pc * ldc], sl = (double)S[jc + pc * lds];
        cs[qq][jj] = ok ? f64x2{cl, sl} : f64x2{1.0, 0.0};
    }
    __syncthreads();
    const int wl = tid >> 4, row = tid & 15;
    const int wi = wi0 + wl;
    if (wi >= qwin)
        return;
    const int w = wi - 2;
    const bool real = w >= -1 && w <= nwin - 1;
    double v[kWin];
#pragma unroll
    for (int c = 0; c < kWin; ++c)
        v[c] = c == row && real ? 1.0 : 0.0;
    if (real) {
#pragma unroll
        for (int tau = 0; tau < kSeq; ++tau) {
#pragma unroll
            for (int qq = 0; qq < kSeq; ++qq) {
                // rotation (j, 8*band + qq) with j = 8w + 7 + tau - qq, on
                // window columns uu = j - 8w and uu + 1
                const f64x2 p = cs[qq][kSeq * wl + tau];
                const int uu = kSeq - 1 + tau - qq;
                const double x = v[uu], y = v[uu + 1];
                v[uu] = __builtin_fma(p.x, x, p.y * y);
                v[uu + 1] = __builtin_fma(p.x, y, -(p.y * x));
            }
        }
    }
    const int s = row >> 2, gg = row & 3;
    double *dst = q + (((int64_t)band * qwin + wi) * 64 + 16 * gg) * 4 + s;
#pragma unroll
    for (int c = 0; c < kWin; ++c)
        dst[c * 4] = v[c];
}

template <int NB, int R>
hipError_t go_mfma(const Plan &p, double *A, const char *ws, hipStream_t st)
{
    MfmaArgs a;
    a.A = (uint64_t)A;
    a.ldab = (uint64_t)p.lda * sizeof(double);
    a.m = p.m;
    a.n = (int)p.n;
    a.nwin = p.mfma_nwin;
    a.nchunks = p.mfma_nchunks;
    a.nseg = p.mfma_nseg;
    a.waves = p.waves;
    a.seg_delay = p.mfma_seg_delay;
    a.nwg = p.nwg;
    a.remap = p.remap;
    a.spin_limit = p.spin_limit;
    a.wait_bias = p.wait_bias;
    a.q = (uint64_t)(ws + p.off_coef);
    a.flags = (int *)(ws + p.off_flags);
    a.status = p.status;
    sweep_mfma<NB, R><<<p.nwg, kWaves * kWave, p.lds_bytes, st>>>(a);
    return hipGetLastError();
}

}  // namespace

// Shapes (bands per wave, row blocks per wave) with a compiled kernel.
bool mfma_shape_supported(int nb_wave, int rows)
{
    return (nb_wave == 3 && (rows == 5 || rows == 4 || rows == 2)) ||
           (nb_wave == 2 && (rows == 4 || rows == 2)) || (nb_wave == 1 && (rows == 4 || rows == 2));
}

int mfma_wave_stride(int nb_wave) { return 4 * ((2 * nb_wave + 3) / 4); }

int mfma_waves() { return kWaves; }

int mfma_seg_delay(int nb_wave)
{
    // The waves of a later segment load block v at their super-step v-3
    // (from the segment's start) on the strength of a flag poll issued
    // kPollLag super-steps before; the previous segment finishes block v
    // in its last wave at (kWaves-1)*stride + v + 2NB-1, publishes it
    // 2 + kPubWait super-steps later, and a poll kFlagMargin super-steps
    // after that sees it.
    const int pub = 2 * nb_wave + kPubWait + 1;
    const int need = mfma_wave_stride(nb_wave) * (kWaves - 1) + pub + 3 + kPollLag + kFlagMargin;
    return 4 * ((need + 3) / 4);
}

size_t mfma_lds_bytes(int rows)
{
    // a ring per wave and the input stage: [5][4 slots][rows][64 lanes][2 doubles]
    return (size_t)(kWaves + 1) * kUnroll * rows * 64 * 2 * sizeof(double);
}

hipError_t mfma_occupancy(int nb_wave, int rows, size_t lds, int *blocks)
{
    const void *fn = nullptr;
#define ROTSEQ_MFMA_FN(NBV, RV) \
    if (nb_wave == NBV && rows == RV) fn = (const void *)&sweep_mfma<NBV, RV>;
    ROTSEQ_MFMA_FN(3, 5)
    ROTSEQ_MFMA_FN(3, 4)
    ROTSEQ_MFMA_FN(3, 2)
    ROTSEQ_MFMA_FN(2, 4)
    ROTSEQ_MFMA_FN(2, 2)
    ROTSEQ_MFMA_FN(1, 4)
    ROTSEQ_MFMA_FN(1, 2)
#undef ROTSEQ_MFMA_FN
    if (fn == nullptr)
        return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kWaves * kWave, lds);
}

hipError_t launch_mfma_prep(const Plan &p, const void *C, const void *S, void *ws, hipStream_t st)
{
    const int nbands = p.mfma_nchunks * p.mfma_nb;
    const int64_t blocks = (int64_t)nbands * ((p.mfma_nwin + 3 + kPrepWins - 1) / kPrepWins);
    if (blocks > INT32_MAX)
        return hipErrorInvalidConfiguration;
    double *q = (double *)((char *)ws + p.off_coef);
    int *flags = (int *)((char *)ws + p.off_flags);
    const int64_t words = (int64_t)p.mfma_tiles * p.mfma_nseg * kMfmaFlagStride;
    if (p.esize == 8)
        mfma_prep_q<double><<<(unsigned)blocks, 64, 0, st>>>((const double *)C, p.ldc, (const double *)S, p.lds,
                                                             (int)p.n, p.k, nbands, p.mfma_nwin, q, flags,
                                                             words);
    else
        mfma_prep_q<float><<<(unsigned)blocks, 64, 0, st>>>((const float *)C, p.ldc, (const float *)S, p.lds,
                                                            (int)p.n, p.k, nbands, p.mfma_nwin, q, flags,
                                                            words);
    return hipGetLastError();
}

hipError_t launch_mfma(const Plan &p, void *A, const void *ws, hipStream_t st)
{
    const char *w = (const char *)ws;
    double *X = (double *)A;
#define ROTSEQ_MFMA_GO(NBV, RV) \
    if (p.mfma_nb == NBV && p.mfma_rows == RV) return go_mfma<NBV, RV>(p, X, w, st);
    ROTSEQ_MFMA_GO(3, 5)
    ROTSEQ_MFMA_GO(3, 4)
    ROTSEQ_MFMA_GO(3, 2)
    ROTSEQ_MFMA_GO(2, 4)
    ROTSEQ_MFMA_GO(2, 2)
    ROTSEQ_MFMA_GO(1, 4)
    ROTSEQ_MFMA_GO(1, 2)
#undef ROTSEQ_MFMA_GO
    return hipErrorInvalidValue;
}

}  // namespace rotseq
