// Sequences of 3x3 reflectors (the double-shift QR case named among the
// paper's future work, Section 9) on gfx950.
//
// Reflector (j, p) is I - tau v v^T with v = e_j + nu1 e_{j+1} + nu2 e_{j+2};
// A <- A H(0,0) H(1,0) ... H(n-3,k-1).  Per row, with (x, y, z) the entries
// in columns j, j+1, j+2:
//     w = x + nu1 y + nu2 z,   x -= tau w,   y -= tau nu1 w,   z -= tau nu2 w.
//
// Schedule: the wavefront of Section 1.1 with a band of K sequences per
// wave.  Reflector (j, p+1) reads the columns that (j+2, p) writes, so within
// a band sequence q runs two columns behind sequence q-1: at local step t the
// wave applies (t - 2q, q) for q = 0..K-1 in ascending q.  Column c is final
// for the band after step c + 2K - 2 and leaves the wave then.
//
// One workgroup owns a 64-row tile (one row per lane, rows stay in
// registers) and runs one wave per band; wave w takes the columns that wave
// w-1 has finished through an LDS ring, and the last wave writes A.  The
// waves advance in lockstep: every G steps they end a group with an LDS wait
// and a workgroup barrier, and wave w starts L steps (L/G groups) after wave
// w-1, which is enough for every column it reads to have been written in an
// earlier group and for every ring slot to have been read before it is
// reused (the conditions are stated beside R3Geom and checked on the CPU by
// the schedule tests).  No wave ever spins, so there is nothing to time out.
//
// Coefficients are reordered by a preparation kernel into wavefront order:
// the records (nu1, nu2, -tau, -tau nu1, -tau nu2) of the K reflectors of one
// step side by side.  With the products formed once, a reflector is
//     w = x + nu1 y + nu2 z;  x += (-tau) w;  y += (-tau nu1) w;  z += (-tau nu2) w,
// five FMAs per row.  A wave takes the records of a group of steps with
// vector loads, one group ahead, lane l of every 16-lane row holding records
// 2l and 2l+1 of a 32-record block, and reads them in the FMAs through the
// DPP row_newbcast operand modifier (a copy of x into w makes it six
// instructions).  Scalar loads would be simpler, but they complete out of
// order, so a wave can only wait for all of them: every step would wait for
// its own records.  FP32 does the same with 32-bit DPP (quad_perm broadcast
// within each quad of lanes).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rotseq_device.h"
#include "rotseq_internal.h"
#include "rotseq_refl3.h"

namespace rotseq {
namespace {

using namespace dev;

// K: sequences per band (per wave).
// G: steps per lockstep group.  D: columns fetched ahead of their first use.
// R: register ring (columns held per lane): at step t the columns
//    t-2K+2 .. t+2+D are live, 2K+1+D of them; a multiple of 2G so that the
//    unrolled chunk of R steps ends on a group boundary and the records of
//    its groups alternate between two register sets.
// L: lag between neighbouring waves in steps, a multiple of G.  Wave w reads
//    column c at its step c-2-D, which is wave w-1's step c-2-D+L >=
//    c+2K+G-2; wave w-1 wrote the column at its step c+2K-2, at least G
//    steps and so at least one group earlier (L >= 2K+D+G).
// RB: LDS ring slots (column c in slot c mod RB).  Wave w-1 overwrites the
//    slot of column c with column c+RB at its step c+RB+2K-2.  Wave w reads
//    column c >= D+2 at wave w-1's step c+2K+G-2 (L = 2K+D+G), a group
//    earlier when RB >= 2G-1; it reads columns 0..D+1 together in its first
//    group, wave w-1's steps L..L+G-1, which ends before step RB+2K-2 when
//    RB >= L+G-2K+2.  Wave w-1 wrote column D+1, the last of those, at its
//    step 2K+D-1 < L - G + 1, in an earlier group.
template <int K>
struct R3Geom {
    static constexpr int G = 4;
    static constexpr int D = 4;
    static constexpr int R = (2 * K + 1 + D + 2 * G - 1) / (2 * G) * (2 * G);
    static constexpr int L = (2 * K + D + G + G - 1) / G * G;
    static constexpr int RB = L + G - 2 * K + 2;
    static_assert(R >= 2 * K + 1 + D && R % (2 * G) == 0, "register ring");
    static_assert(L >= 2 * K + D + G && L % G == 0, "wave lag");
    static_assert(RB >= 2 * G - 1, "LDS ring");
};

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int Q, int N, typename F>
__device__ __forceinline__ void unroll(F &&f)
{
    if constexpr (Q < N) {
        f(std::integral_constant<int, Q>{});
        unroll<Q + 1, N>(f);
    }
}

// End of a lockstep group: this wave's LDS accesses have completed, then all
// waves of the workgroup meet.  The compiler fences keep every memory access
// of a group on its side of the barrier.
__device__ __forceinline__ void r3_barrier()
{
    compiler_fence();
    __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8));  // lgkmcnt(0) only
    __builtin_amdgcn_s_barrier();
    compiler_fence();
}

// Record fields of one reflector.
constexpr int kRec = 5;  // nu1, nu2, -tau, -tau*nu1, -tau*nu2

// One 3x3 reflector on the entries (x, y, z) of a row, with the record
// fields broadcast from lanes L0..L4 of each 16-lane row of a0..a4 (DPP
// row_newbcast): w = x + nu1 y + nu2 z, then x, y, z += (field) * w.  A DPP
// source must not have been written by a VALU instruction in the two
// preceding instructions, which the compiler cannot see inside the asm;
// a0..a4 are written by the record loads only (tests scan the ISA).
#define R3_FMAC(X, A, Y, L) \
    "v_fmac_f64_dpp %" #X ", %" #A ", %" #Y " row_newbcast:%" #L " row_mask:0xf bank_mask:0xf\n"
template <int L0, int L1, int L2, int L3, int L4>
__device__ __forceinline__ void reflect3_dpp(double &x, double &y, double &z, double a0, double a1,
                                             double a2, double a3, double a4)
{
    double w;
    asm("v_mov_b64 %3, %0\n" R3_FMAC(3, 4, 1, 9) R3_FMAC(3, 5, 2, 10) R3_FMAC(0, 6, 3, 11)
            R3_FMAC(1, 7, 3, 12) R3_FMAC(2, 8, 3, 13)
        : "+v"(x), "+v"(y), "+v"(z), "=&v"(w)
        : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(a4), "n"(L0), "n"(L1), "n"(L2), "n"(L3), "n"(L4));
}
#undef R3_FMAC

// FP32: the same with record fields broadcast from lane S0..S4 of each quad
// of a0..a4 (DPP quad_perm); 32-bit DPP has no row_newbcast.
#define R3_FMAC32(X, A, Y, S) \
    "v_fmac_f32_dpp %" #X ", %" #A ", %" #Y " quad_perm:[%" #S ",%" #S ",%" #S ",%" #S "] row_mask:0xf bank_mask:0xf\n"
template <int S0, int S1, int S2, int S3, int S4>
__device__ __forceinline__ void reflect3_dpp32(float &x, float &y, float &z, float a0, float a1,
                                               float a2, float a3, float a4)
{
    float w;
    asm("v_mov_b32 %3, %0\n" R3_FMAC32(3, 4, 1, 9) R3_FMAC32(3, 5, 2, 10) R3_FMAC32(0, 6, 3, 11)
            R3_FMAC32(1, 7, 3, 12) R3_FMAC32(2, 8, 3, 13)
        : "+v"(x), "+v"(y), "+v"(z), "=&v"(w)
        : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(a4), "n"(S0), "n"(S1), "n"(S2), "n"(S3), "n"(S4));
}
#undef R3_FMAC32

// Records in wavefront order: for band g (sequences gK .. gK+K-1), local step
// t and member q, rec[((g * steps + t) * K + q) * 5 + {0..4}] holds
// (nu1, nu2, -tau, -tau nu1, -tau nu2) of reflector (t - 2q, gK + q), or
// zeros where that reflector does not exist (the sweep never applies those).
// Reflector (j, p) is read at TAU[j*cj + p*ldt] (likewise NU1, NU2): cj = -1
// with negative leading dimensions reads the reflectors in the inverse order.
// Reflectors j < nrefl exist (n-2; n-1 for 2x2 reflectors, which run as 3x3
// ones with NU2 == NULL, i.e. nu2 = 0: the third column of the last one
// lies past A and is neither read into nor written by it).
template <typename T>
__global__ void refl3_prep(const T *__restrict__ TAU, int64_t ldt, const T *__restrict__ NU1,
                           int64_t ld1, const T *__restrict__ NU2, int64_t ld2, int64_t cj,
                           int64_t nrefl, int64_t k, int K, int steps, int64_t total,
                           T *__restrict__ rec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total)
        return;
    const int q = (int)(i % K);
    const int64_t r = i / K;
    const int64_t t = r % steps, g = r / steps;
    const int64_t j = t - 2 * q, p = g * K + q;
    T tau = T(0), nu1 = T(0), nu2 = T(0);
    if (j >= 0 && j < nrefl && p < k) {
        tau = TAU[j * cj + p * ldt];
        nu1 = NU1[j * cj + p * ld1];
        nu2 = NU2 != nullptr ? NU2[j * cj + p * ld2] : T(0);
    }
    T *out = rec + kRec * i;
    out[0] = nu1;
    out[1] = nu2;
    out[2] = -tau;
    out[3] = -(tau * nu1);
    out[4] = -(tau * nu2);
}

struct Refl3Args {
    uint64_t A;            // T*, column-major, lda (negative: a column-reversed view)
    int64_t lda;
    uint64_t rec;          // records of this launch's first band
    int64_t band_stride;   // elements between the records of neighbouring bands
    int m, n;
    int chunks;            // R-step chunks per band
};

// At most 12 waves (bands) per workgroup: 3 waves per SIMD leave each wave
// up to 168 VGPRs.
constexpr int kRefl3MaxWaves = 12;
// Sequences per band (per wave): FP32 keeps its records of a group in half
// the registers with bands of 4.
constexpr int refl3_band(int esize) { return esize == 8 ? 8 : 4; }

// REV: the reflectors of a column-reversed view (the inverse order): the
// reflector at view columns c, c+1, c+2 has its unit component on c+2, so
// the formula runs with the roles of the first and third column swapped.
template <typename T, int K, bool REV>
__global__ __launch_bounds__(kRefl3MaxWaves * 64) void refl3_sweep(Refl3Args a)
{
    using Gm = R3Geom<K>;
    constexpr int G = Gm::G, D = Gm::D, R = Gm::R, L = Gm::L, RB = Gm::RB;
    extern __shared__ char lds_raw[];
    T *ring = reinterpret_cast<T *>(lds_raw);

    const int W = (int)(blockDim.x / kWave);
    const int w = uniform_i((int)(threadIdx.x / kWave));
    const int lane = (int)(threadIdx.x % kWave);
    const int64_t row0 = (int64_t)blockIdx.x * kWave;
    const int rows = (int)(a.m - row0 < kWave ? a.m - row0 : kWave);
    // Lanes past the last row of a ragged tile repeat that row (finite
    // values, same work) and store nothing.
    const int lrow = lane < rows ? lane : rows - 1;
    const bool from_a = w == 0, to_a = w == W - 1;
    const int n = a.n;
    const int64_t lda = a.lda;
    // A through the global address space: flat accesses would also count
    // against the LDS/scalar counter, so every wait for a coefficient or a
    // ring entry would drain the column prefetch as well.
    using GT = __attribute__((address_space(1))) T;
    GT *A = (GT *)(uintptr_t)a.A + row0;
    const T *in_ring = ring + (w > 0 ? w - 1 : 0) * RB * kWave + lane;
    T *out_ring = ring + w * RB * kWave + lane;
    const T *rec_v = reinterpret_cast<const T *>(a.rec) + w * a.band_stride;

    // Column sources and sinks.  ROLE bit 0: this wave reads A (else the
    // previous wave's ring); bit 1: it writes A (else its own ring).  Lanes
    // past the last row of a ragged tile hold a bitwise copy of that row and
    // store the same value to it, so stores need no lane mask.
    auto fetch = [&](int c, auto role) -> T {
        constexpr int ROLE = decltype(role)::value;
        if (c >= n)
            return T(0);
        if (ROLE & 1)
            return A[(int64_t)c * lda + lrow];
        return in_ring[(c % RB) * kWave];
    };
    auto put = [&](int c, T v, auto role) {
        constexpr int ROLE = decltype(role)::value;
        if (c < 0 || c >= n)
            return;
        if (ROLE & 2)
            A[(int64_t)c * lda + lrow] = v;
        else
            out_ring[(c % RB) * kWave] = v;
    };
    // Calls f with this wave's role as a compile-time constant.
    auto with_role = [&](auto &&f) {
        if (from_a && to_a)
            f(std::integral_constant<int, 3>{});
        else if (from_a)
            f(std::integral_constant<int, 1>{});
        else if (to_a)
            f(std::integral_constant<int, 2>{});
        else
            f(std::integral_constant<int, 0>{});
    };

    T x[R];
    unroll<0, R>([&](auto ic) { x[decltype(ic)::value] = T(0); });

    for (int i = 0; i < w * (L / G); ++i)
        r3_barrier();
    with_role([&](auto role) {
        unroll<0, D + 2>([&](auto ic) { x[decltype(ic)::value] = fetch(decltype(ic)::value, role); });
    });

    // Records through DPP: a group's G*K records are NB blocks of BLK, 16
    // bytes per lane, in register set (group index) mod 2.  FP64: blocks of
    // 32, lane l of each 16-lane row holding records 2l and 2l+1 (read with
    // row_newbcast).  FP32: blocks of 16, lane s of each quad holding records
    // 4s..4s+3 (read with quad_perm).
    constexpr int PER = 16 / sizeof(T);              // records per lane and load
    constexpr int BLK = sizeof(T) == 8 ? 32 : 16;    // records per block
    static_assert((G * K * kRec) % BLK == 0, "a group's records fill whole blocks");
    constexpr int NB = G * K * kRec / BLK;
    typedef T tx4 __attribute__((ext_vector_type(PER)));
    using GV = __attribute__((address_space(1))) const tx4;
    tx4 rd[2][NB];
    const uint64_t rec_b = (uint64_t)rec_v + (sizeof(T) == 8 ? (lane & 15) : (lane & 3)) * 16;
    auto load_group = [&](auto setc, int step0) {
        constexpr int SET = decltype(setc)::value;
        const uint64_t base = rec_b + (uint64_t)step0 * K * kRec * sizeof(T);
        unroll<0, NB>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            rd[SET][b] = *(GV *)(base + b * BLK * sizeof(T));
        });
    };
    bool have_first = false;  // records of the chunk's first group are in set 0
    const int steps = a.chunks * R;

    // One chunk of R steps.  Edge chunks (GUARD) check the columns they
    // fetch and store against A; interior chunks are straight-line code
    // between barriers.  Reflectors that do not exist (before column 0, past
    // column n-3, past sequence k-1) have zero records: an exact identity on
    // finite entries.
    const uint64_t ldab = (uint64_t)lda * sizeof(T);
    auto chunk = [&](int t0, auto guarded, auto role) {
        constexpr bool GUARD = decltype(guarded)::value;
        // Running column addresses (fetch: column t+2+D; store: column
        // t-2K+2), kept opaque so that the unrolled steps share one SGPR pair
        // each instead of one 64-bit offset per step.
        uint64_t fa = (uint64_t)(A + (int64_t)(t0 + 2 + D) * lda);
        uint64_t sa = (uint64_t)(A + (int64_t)(t0 - 2 * K + 2) * lda);
        if (!have_first)
            load_group(std::integral_constant<int, 0>{}, t0);
        unroll<0, R>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            const int t = t0 + u;
            if constexpr (u % G == 0) {
                // records of the next group (after the last group, the next
                // chunk's first; interior chunks are never the last chunk)
                if (!GUARD || u + G < R || t + G < steps)
                    load_group(std::integral_constant<int, (u / G + 1) & 1>{}, t + G);
            }
            if constexpr (GUARD) {
                x[(u + 2 + D) % R] = fetch(t + 2 + D, role);
            } else if constexpr (decltype(role)::value & 1) {
                x[(u + 2 + D) % R] = ((GT *)fa)[lrow];
                fa += ldab;
                opaque(fa);
            } else {
                x[(u + 2 + D) % R] = in_ring[((t + 2 + D) % RB) * kWave];
            }
            unroll<0, K>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int s = (u - 2 * q + 2 * R) % R;  // slot of column t - 2q
                // record field f is element e+f: block (e+f)/BLK, lane
                // ((e+f) % BLK)/PER of the row or quad, component (e+f) % PER
                constexpr int set = (u / G) & 1, e = ((u % G) * K + q) * kRec;
                constexpr int L0 = (e % BLK) / PER, L1 = ((e + 1) % BLK) / PER,
                              L2 = ((e + 2) % BLK) / PER, L3 = ((e + 3) % BLK) / PER,
                              L4 = ((e + 4) % BLK) / PER;
                const T a0 = rd[set][e / BLK][e % PER], a1 = rd[set][(e + 1) / BLK][(e + 1) % PER],
                        a2 = rd[set][(e + 2) / BLK][(e + 2) % PER],
                        a3 = rd[set][(e + 3) / BLK][(e + 3) % PER],
                        a4 = rd[set][(e + 4) / BLK][(e + 4) % PER];
                T &c0 = x[REV ? (s + 2) % R : s], &c2 = x[REV ? s : (s + 2) % R];
                if constexpr (sizeof(T) == 8)
                    reflect3_dpp<L0, L1, L2, L3, L4>(c0, x[(s + 1) % R], c2, a0, a1, a2, a3, a4);
                else
                    reflect3_dpp32<L0, L1, L2, L3, L4>(c0, x[(s + 1) % R], c2, a0, a1, a2, a3, a4);
            });
            const int c = t - 2 * K + 2;
            const T v = x[(u - 2 * K + 2 + 2 * R) % R];
            if constexpr (GUARD) {
                put(c, v, role);
            } else if constexpr (decltype(role)::value & 2) {
                ((GT *)sa)[lrow] = v;
                sa += ldab;
                opaque(sa);
            } else {
                out_ring[(c % RB) * kWave] = v;
            }
            if constexpr ((u + 1) % G == 0)
                r3_barrier();
        });
        have_first = t0 + R < steps;
    };

    for (int ch = 0; ch < a.chunks; ++ch) {
        const int t0 = ch * R;
        // Interior chunks: every column fetched or stored is inside A.
        const bool interior = t0 >= 2 * K - 2 && t0 + R + D + 1 < n;
        if (interior)
            with_role([&](auto role) { chunk(t0, std::false_type{}, role); });
        else
            with_role([&](auto role) { chunk(t0, std::true_type{}, role); });
    }

    for (int i = 0; i < (W - 1 - w) * (L / G); ++i)
        r3_barrier();
}

template <typename T, int K, bool REV>
hipError_t sweep_launches(const Refl3Plan &p, T *A, const T *rec, hipStream_t st)
{
    using Gm = R3Geom<K>;
    const int tiles = (int)((p.m + kWave - 1) / kWave);
    const int64_t band_stride = (int64_t)p.steps * K * kRec;
    for (int b0 = 0; b0 < p.nbands; b0 += p.waves) {
        const int W = p.nbands - b0 < p.waves ? p.nbands - b0 : p.waves;
        Refl3Args a;
        a.A = (uint64_t)A;
        a.lda = p.lda;
        a.rec = (uint64_t)(rec + b0 * band_stride);
        a.band_stride = band_stride;
        a.m = (int)p.m;
        a.n = (int)p.n;
        a.chunks = p.steps / Gm::R;
        const size_t lds = W > 1 ? (size_t)(W - 1) * Gm::RB * kWave * sizeof(T) : 4;
        refl3_sweep<T, K, REV><<<tiles, W * kWave, lds, st>>>(a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace

bool refl3_plan(Refl3Plan &p, int64_t m, int64_t n, int64_t k, int64_t lda, int esize, int width)
{
    if (m <= 0 || n < width || k <= 0 || m > INT32_MAX - kWave || n > INT32_MAX / 2)
        return false;
    p.m = m;
    p.n = n;
    p.k = k;
    p.lda = lda;
    p.esize = esize;
    p.band = refl3_band(esize);
    const int R = esize == 8 ? R3Geom<refl3_band(8)>::R : R3Geom<refl3_band(4)>::R;
    p.nbands = (int)((k + p.band - 1) / p.band);
    // Local steps per band: column n-1 leaves after step n+2K-3.
    const int64_t steps = n + 2 * p.band - 2;
    p.steps = (int)((steps + R - 1) / R * R);
    // Launches of at most kRefl3MaxWaves waves, balanced.
    const int launches = (p.nbands + kRefl3MaxWaves - 1) / kRefl3MaxWaves;
    p.waves = (p.nbands + launches - 1) / launches;
    p.rec_elems = (int64_t)p.nbands * p.steps * p.band * kRec;
    p.nrefl = n - width + 1;
    p.total = ((size_t)p.rec_elems * esize + 255) & ~(size_t)255;
    return true;
}

hipError_t launch_refl3_prep(const Refl3Plan &p, const void *TAU, int64_t ldt, const void *NU1,
                             int64_t ld1, const void *NU2, int64_t ld2, int64_t cj, void *ws,
                             hipStream_t st)
{
    const int B = 256;
    const int64_t total = p.rec_elems / kRec;
    const unsigned blocks = (unsigned)((total + B - 1) / B);
    if (p.esize == 8)
        refl3_prep<double><<<blocks, B, 0, st>>>((const double *)TAU, ldt, (const double *)NU1, ld1,
                                                 (const double *)NU2, ld2, cj, p.nrefl, p.k, p.band,
                                                 p.steps, total, (double *)ws);
    else
        refl3_prep<float><<<blocks, B, 0, st>>>((const float *)TAU, ldt, (const float *)NU1, ld1,
                                               (const float *)NU2, ld2, cj, p.nrefl, p.k, p.band,
                                               p.steps, total, (float *)ws);
    return hipGetLastError();
}

hipError_t launch_refl3_sweep(const Refl3Plan &p, void *A, const void *ws, bool rev, hipStream_t st)
{
    if (p.esize == 8 && p.band == refl3_band(8))
        return rev ? sweep_launches<double, refl3_band(8), true>(p, (double *)A, (const double *)ws, st)
                   : sweep_launches<double, refl3_band(8), false>(p, (double *)A, (const double *)ws, st);
    if (p.esize == 4 && p.band == refl3_band(4))
        return rev ? sweep_launches<float, refl3_band(4), true>(p, (float *)A, (const float *)ws, st)
                   : sweep_launches<float, refl3_band(4), false>(p, (float *)A, (const float *)ws, st);
    return hipErrorInvalidValue;
}

}  // namespace rotseq
