// Sweep on FP64 matrix instructions (v_mfma_f64_16x16x4f64): a band of 8
// sequences is applied 8 wavefront steps at a time as dense 16 x 16 window
// matrices, the accumulate-then-multiply form of Section 8 of the paper
// (there done with a BLAS GEMM).
//
// Windows.  Band beta (sequences 8*beta .. 8*beta+7) applies at step t the
// rotations (t-q, 8*beta+q), q = 0..7 (Section 1.1).  Window w holds steps
// 8w .. 8w+7, which touch only the 16 columns 8w-7 .. 8w+8; their product
// is one orthogonal 16 x 16 matrix Q(beta, w), prepared once per call by
// `mfma_prep_q` (with Q(beta, -1) = I).  With X the 16 window columns of a
// row tile, the window is X <- X Q.  Afterwards columns 8w-7 .. 8w (block
// w) are final for the band, and columns 8w+1 .. 8w+8 stay "in flight"
// into window w+1, whose new columns are block w+1 of the band's input.
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
// chunk of NB consecutive bands; the W waves of a workgroup hold W
// consecutive chunks of one tile's chain (a segment); a chain longer than
// W chunks continues in the next workgroup through A and a progress flag,
// as in the vector chain kernel.  Super-steps are separated by a workgroup
// barrier; wave j starts 4*ceil((2NB+3)/4) super-steps after wave j-1 and
// a later segment `seg_delay` super-steps after the previous one, so every
// block is produced at least one super-step before it is read (checked by
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
    uint64_t q;      // [band][nwin+1][64 lanes][4 slabs] window matrices
    int *flags;      // [tile][seg] blocks published by the segment's last wave
    int *status;
};

// A wave that hands its blocks to the next workgroup publishes block w one
// super-step after storing it, once the stores have completed.
constexpr int kPubLag = 1;
// Super-steps between a flag store and a poll that is sure to see it.
constexpr int kFlagMargin = 3;

template <int NB>
struct MfmaGeom {
    static_assert(NB >= 1 && NB <= 3, "bands per wave");
    // Super-steps between the starts of neighbouring waves: the last band
    // finishes block v at wave-local super-step v + 2NB - 1 and the next
    // wave's first band reads it at its super-step v.
    static constexpr int kStride = 4 * ((2 * NB + 3) / 4);
    // The four ring slots are rewritten four blocks later, after the read.
    static_assert(2 * NB - 1 + kUnroll > kStride, "ring slot reuse");
};

// Where one super-step's memory operations go in its stream of 4*NB*R
// products (the last band's first): after product k comes operation k, in
// the order
//   poll of the previous segment's flag (1), loads of input block sp+3
//   (2R), loads of window matrices (2NB), then per row block r the two
//   stores of the finished block and the ring write (3R, no earlier than
//   two products after that row's last product),
// and operations past the last product follow it.  The flag store that
// publishes the previous super-step's block ends the super-step.  Every
// working wave issues all of them (a role it does not have gets an empty
// descriptor: loads return 0, stores are dropped), so no branch surrounds
// a memory operation and the compiler's wait counts are exact.
template <int NB, int R>
struct StepOps {
    static constexpr int kProducts = 4 * NB * R;
    static constexpr int kPoll = 0;
    static constexpr int kIn = 1;                // 2R loads
    static constexpr int kQ = kIn + 2 * R;       // 2NB loads
    static constexpr int kOut0 = (kQ + 2 * NB > 3 * R + 2) ? kQ + 2 * NB : 3 * R + 2;
    static constexpr int kEnd = kOut0 + 3 * R;   // one past the last operation
    // vector memory operations after the last store of block w (stored in
    // super-step s) up to the flag store of super-step s+1
    static constexpr int kAfterStores = 1 + (1 + 2 * R + 2 * NB + 2 * R);
    static_assert(kAfterStores < 64, "publication count");
};

// Descriptor over the 8 columns of block v (8v-7 .. 8v) of A, clipped to
// [0, n), or an empty one if !on: lanes whose column lies outside get 0 on
// loads and are dropped on stores.  A lane's byte offset within it is its
// fixed part (column 8v-7 + g4 + 4e relative to 8v-7, and its row) plus
// `shift` = (8v-7 - first column of the descriptor) * column stride.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const MfmaArgs &a, int v, bool on, int &shift)
{
    // (readfirstlane: the clamp below is selected as a VALU instruction,
    // and a descriptor left in VGPRs costs a loop around every access)
    const int first = kSeq * v - (kSeq - 1);
    const int lo = uniform(first < 0 ? 0 : first);
    const int hi = kSeq * v + 1 < a.n ? kSeq * v + 1 : a.n;  // one past the last column
    shift = uniform((int)((int64_t)(first - lo) * (int64_t)a.ldab));
    const uint32_t bytes = (uint32_t)uniform(on && hi > lo ? (int)((uint64_t)(hi - lo) * a.ldab) : 0);
    return make_rsrc(a.A + (uint64_t)lo * a.ldab, bytes);
}

template <int NB, int R>
__global__ __launch_bounds__(256, 1) void sweep_mfma(MfmaArgs a)
{
    using Ops = StepOps<NB, R>;
    constexpr int kStride = MfmaGeom<NB>::kStride;
    static_assert(kPubLag == 1, "publication count");
    extern __shared__ __align__(16) char lds_raw[];
    typedef __attribute__((address_space(3))) double lds_f64;
    lds_f64 *ring = (lds_f64 *)(__attribute__((address_space(3))) char *)lds_raw;

    const int lane = threadIdx.x & 63;
    const int g4 = lane >> 4;
    const int wv = uniform((int)(threadIdx.x >> 6));
    const int p = (int)blockIdx.x;
    const int g = a.remap ? (p & 7) * (a.nwg >> 3) + (p >> 3) : p;
    const int tile = g / a.nseg;
    const int seg = g - tile * a.nseg;
    const int chunk = seg * a.waves + wv;
    const int active_waves = a.nchunks - seg * a.waves < a.waves ? a.nchunks - seg * a.waves : a.waves;
    const int nwin = a.nwin;
    const int pre = kUnroll + seg * a.seg_delay;
    const int off = pre + wv * kStride;
    const int T = (pre + (a.waves - 1) * kStride + 2 * NB - 1 + nwin + 1 + kUnroll - 1) & ~(kUnroll - 1);
    // The ring starts zeroed: a wave reads its slots before the previous
    // wave first writes them (the products there use zero window matrices,
    // and 0 * x is 0 only for finite x).
    for (int x = (int)threadIdx.x; x < a.waves * kUnroll * R * 2 * 64; x += (int)blockDim.x)
        ring[x] = 0.0;
    __syncthreads();

    if (wv >= active_waves) {  // no chunk: only the barriers
        idle_groups(T);
        return;
    }
    const bool in_global = wv == 0;
    const bool in_wait = in_global && seg > 0;
    const bool out_global = wv == active_waves - 1;
    const bool publish = out_global && chunk + 1 < a.nchunks;

    // Fixed part of this lane's byte offsets within a block, per row block
    // and column group e (columns g4 + 4e of the block); rows past m get an
    // offset past every descriptor's range (the planner keeps 9 columns of
    // A below 2^30 bytes), so their stores are dropped.
    const int64_t row0 = (int64_t)tile * R * 16 + (lane & 15);
    int voff[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t ro = row0 + 16 * r < a.m ? (uint32_t)((row0 + 16 * r) * 8) : 0x80000000u;
#pragma unroll
        for (int e = 0; e < 2; ++e)
            voff[r][e] = (int)(ro + (uint32_t)((g4 + 4 * e) * a.ldab));
    }

    // Window matrices of this wave's bands: one descriptor per band.
    __amdgpu_buffer_rsrc_t qrs[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
        qrs[i] = make_rsrc(a.q + ((uint64_t)(chunk * NB + i) * (nwin + 1)) * kQBytes,
                           (uint32_t)((nwin + 1) * kQBytes));
    const int qvoff = lane * 32;

    int *flag_in = a.flags + (int64_t)tile * a.nseg + (seg - 1);
    int *flag_out = a.flags + (int64_t)tile * a.nseg + seg;
    const __amdgpu_buffer_rsrc_t flag_in_rs = make_rsrc((uint64_t)flag_in, in_wait ? 4u : 0u);
    int limit = a.spin_limit, timed_out = 0, known = 0, polled = 0;

    // Ring of wave j -> j+1: [4 slots][R][2 elements][64 lanes] per wave
    // (the first wave reads its own ring, and ignores what it reads).
    lds_f64 *ring_in = ring + (int64_t)(wv > 0 ? wv - 1 : 0) * (kUnroll * R * 2 * 64) + lane;
    lds_f64 *ring_out = ring + (int64_t)wv * (kUnroll * R * 2 * 64) + lane;

    f64x4 D[2][NB][R];
#pragma unroll
    for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int r = 0; r < R; ++r)
                D[b2][i][r] = f64x4{0.0, 0.0, 0.0, 0.0};
    double IN[kUnroll][R][2];  // input blocks of the first wave, 3 ahead
    double Qr[kUnroll][NB][4]; // window matrices, 3 ahead
#pragma unroll
    for (int x = 0; x < kUnroll; ++x) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            IN[x][r][0] = IN[x][r][1] = 0.0;
#pragma unroll
        for (int i = 0; i < NB; ++i)
            Qr[x][i][0] = Qr[x][i][1] = Qr[x][i][2] = Qr[x][i][3] = 0.0;
    }

    for (int t = 0; t < T; t += kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int sp = t + u - off;  // wave-local super-step; sp % 4 == u % 4
            const int cur = u & 1, prv = cur ^ 1;
            // 1. A later segment's first wave loads input block sp + 3 once
            // the previous segment has published it: the poll issued last
            // super-step normally says so; otherwise wait here.
            if (in_wait) {
                const int v = sp + 3;
                const int need = (v + 1 < nwin ? v + 1 : nwin) + a.wait_bias;
                const int seen = uniform(polled);
                known = known > seen ? known : seen;
                if (known < need)
                    known = wait_flag(flag_in, need - 1, limit, timed_out);
            }
            // 2. Descriptors of the super-step: input block sp+3 (first
            // wave), finished block sp-2NB+1 of the last band (last wave).
            int in_shift, out_shift;
            const __amdgpu_buffer_rsrc_t in_rs = block_rsrc(a, sp + 3, in_global, in_shift);
            const int wo = sp - 2 * NB + 1;
            const __amdgpu_buffer_rsrc_t out_rs = block_rsrc(a, wo, out_global && wo >= 0 && wo <= nwin - 1, out_shift);
            // New columns for band 0, block sp: from A (first wave, loaded
            // three super-steps ago) or the previous wave's ring slot, read
            // here and selected where band 0 uses them (the reads are
            // volatile, so they are issued in every wave and the choice is
            // a select, not a branch).
            double ringv[R][2];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int e = 0; e < 2; ++e)
                    ringv[r][e] = ((volatile lds_f64 *)ring_in)[((u * R + r) * 2 + e) * 64];
            compiler_fence();
            __builtin_amdgcn_sched_barrier(0);

            // Memory operation k of the super-step (compile-time k).
            auto memop = [&](const int k) {
                if (k == Ops::kPoll) {
                    polled = (int)__builtin_amdgcn_raw_buffer_load_b32(flag_in_rs, 0, 0, kPolicyDevice);
                } else if (k >= Ops::kIn && k < Ops::kQ) {
                    const int r = (k - Ops::kIn) >> 1, e = (k - Ops::kIn) & 1;
                    IN[(u + 3) & 3][r][e] = buf_load<kPolicyDevice>(double(), in_rs, voff[r][e] + in_shift);
                } else if (k >= Ops::kQ && k < Ops::kQ + 2 * NB) {
                    // band i's window sp+2-2i, used three super-steps later
                    // (outside -1 .. nwin-1: zeros)
                    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
                    const int i = (k - Ops::kQ) >> 1, h = (k - Ops::kQ) & 1;
                    const int vo = (sp + 2 - 2 * i + 1) * kQBytes + qvoff + 16 * h;
                    const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(qrs[i], vo, 0, kPolicyL2);
                    Qr[(u + 3) & 3][i][2 * h] = __builtin_bit_cast(double, (unsigned long long)q.x | ((unsigned long long)q.y << 32));
                    Qr[(u + 3) & 3][i][2 * h + 1] = __builtin_bit_cast(double, (unsigned long long)q.z | ((unsigned long long)q.w << 32));
                } else if (k >= Ops::kOut0 && k < Ops::kEnd) {
                    const int r = (k - Ops::kOut0) / 3, o = (k - Ops::kOut0) % 3;
                    const f64x4 &d = D[cur][NB - 1][r];
                    if (o < 2) {
                        buf_store<kPolicyDevice>(o == 0 ? d.x : d.y, out_rs, voff[r][o] + out_shift);
                    } else {
                        ring_out[((((u - 2 * NB + 1) & 3) * R + r) * 2 + 0) * 64] = d.x;
                        ring_out[((((u - 2 * NB + 1) & 3) * R + r) * 2 + 1) * 64] = d.y;
                    }
                }
            };

            // 3. Products, last band first: band i runs window sp-1-2i on
            // its own in-flight columns and band i-1's block of the last
            // super-step.  Outside the band's windows the window matrix is
            // zero, so the band's state before its first window and what it
            // passes on after its last one are zero (every operand is
            // finite: loads outside A return 0 and the ring starts zeroed).
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
                            b = in_global ? IN[u][r][s - 2] : ringv[r][s - 2];
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
            // 4. Publish the block stored last super-step, once every
            // vector memory operation but the kAfterStores issued since its
            // stores has completed.
            compiler_fence();
            {
                const int wp = sp - 2 * NB;
                const bool pub = publish && wp >= 0 && wp <= nwin - 1;
                if (publish)
                    wait_vmem_at_most<Ops::kAfterStores>();
                compiler_fence();
                __builtin_amdgcn_raw_buffer_store_b32((unsigned)(wp + 1), make_rsrc((uint64_t)flag_out, pub ? 4u : 0u),
                                                      0, 0, kPolicyDevice);
            }
            // 5. Ring writes of this super-step are complete; all waves meet.
            group_barrier();
        }
    }
    if (publish) {
        wait_vmem_at_most<0>();
        __hip_atomic_store(flag_out, nwin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (timed_out)
        record_timeout(a.status, timed_out);
}

// Window matrices: thread (band, window w, row r) builds row r of Q(band, w)
// by applying the window's rotations, in wavefront order, to e_r, then
// scatters it to the operand layout: lane l, slab s holds Q[4s + l/16][l%16].
template <typename T>
__global__ __launch_bounds__(64) void mfma_prep_q(const T *__restrict__ C, int64_t ldc, const T *__restrict__ S, int64_t lds,
                            int n, int64_t k, int nbands, int nwin, double *__restrict__ q)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)nbands * (nwin + 1) * kWin;
    if (idx >= total)
        return;
    const int row = (int)(idx % kWin);
    const int64_t bw = idx / kWin;
    const int wi = (int)(bw % (nwin + 1));
    const int64_t band = bw / (nwin + 1);
    const int w = wi - 1;
    double v[kWin];
#pragma unroll
    for (int c = 0; c < kWin; ++c)
        v[c] = c == row ? 1.0 : 0.0;
    if (w >= 0) {
#pragma unroll
        for (int tau = 0; tau < kSeq; ++tau) {
#pragma unroll
            for (int qq = 0; qq < kSeq; ++qq) {
                const int64_t j = (int64_t)kSeq * w + tau - qq;
                const int64_t pp = band * kSeq + qq;
                double c = 1.0, s = 0.0;
                if (j >= 0 && j <= n - 2 && pp < k) {
                    c = (double)C[j + pp * ldc];
                    s = (double)S[j + pp * lds];
                }
                const int uu = tau - qq + kSeq - 1;
                const double x = v[uu], y = v[uu + 1];
                v[uu] = __builtin_fma(c, x, s * y);
                v[uu + 1] = __builtin_fma(c, y, -(s * x));
            }
        }
    }
    const int s = row >> 2, gg = row & 3;
    double *dst = q + (bw * 64 + 16 * gg) * 4 + s;
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
    sweep_mfma<NB, R><<<p.nwg, p.waves * kWave, p.lds_bytes, st>>>(a);
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

int mfma_seg_delay(int waves, int nb_wave)
{
    // The first wave of a later segment loads block v+3 at its super-step
    // v, on the strength of the flag poll it issued one super-step before;
    // the previous segment's last wave stored that block at
    // (waves-1)*stride + 2NB-1 + v+3 and publishes it kPubLag super-steps
    // later, and a poll kFlagMargin super-steps after that sees it.
    const int need = mfma_wave_stride(nb_wave) * (waves - 1) + 2 * nb_wave + 3 + kPubLag + kFlagMargin;
    return 4 * ((need + 3) / 4);
}

size_t mfma_lds_bytes(int waves, int rows)
{
    // one ring per wave (the last wave's is written and never read)
    return (size_t)waves * kUnroll * rows * 2 * 64 * sizeof(double);
}

hipError_t mfma_occupancy(int nb_wave, int rows, int waves, size_t lds, int *blocks)
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
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, waves * kWave, lds);
}

hipError_t launch_mfma_prep(const Plan &p, const void *C, const void *S, void *ws, hipStream_t st)
{
    const int nbands = p.mfma_nchunks * p.mfma_nb;
    const int64_t total = (int64_t)nbands * (p.mfma_nwin + 1) * kWin;
    constexpr int B = 64;
    const unsigned blocks = (unsigned)((total + B - 1) / B);
    double *q = (double *)((char *)ws + p.off_coef);
    if (p.esize == 8)
        mfma_prep_q<double><<<blocks, B, 0, st>>>((const double *)C, p.ldc, (const double *)S, p.lds,
                                                  (int)p.n, p.k, nbands, p.mfma_nwin, q);
    else
        mfma_prep_q<float><<<blocks, B, 0, st>>>((const float *)C, p.ldc, (const float *)S, p.lds,
                                                 (int)p.n, p.k, nbands, p.mfma_nwin, q);
    const int64_t words = (int64_t)p.mfma_tiles * p.mfma_nseg;
    return launch_zero((int *)((char *)ws + p.off_flags), words, st);
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
