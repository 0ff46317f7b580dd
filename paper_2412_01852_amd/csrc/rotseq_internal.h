// Internal interfaces between the host runtime and the HIP kernels of
// librotseq.  Not installed; the public interface is include/rotseq.h.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace rotseq {

// Per-rotation arithmetic (values of rotseq_opts.arith after resolving AUTO).
enum Arith : int { kExact = 1, kFma = 2, kLift = 3 };

// What the (C, S) arrays of a call hold: rotations (c, s); 2x2 reflectors
// (tau, nu); or reflectors read on the column-reversed matrix (the inverse
// order of a reflector sequence).
enum Kind : int { kRotate = 0, kReflect = 1, kReflectRev = 2 };

// Sweep kernel families (values of rotseq_opts.kernel after resolving AUTO).
enum Kernel : int { kMultipass = 1, kChain = 2, kMfma = 3 };

// Identity records after the last step of each band for the chain kernel;
// covers its deepest coefficient look-ahead (16 steps) plus one.
constexpr int kChainCoefPad = 17;

// Shape of one call after dispatch decisions: A is m x n (column-major, lda),
// the k sequences are cut into `npass` bands of `band` sequences (the last
// band is padded with identity rotations), and every sweep over the columns
// takes `steps` wavefront steps (n + band - 1 rounded up to the kernel's
// unroll length; steps past the last real one are identity).
// The coefficient buffer holds steps + pad records per band (pad = 1 for the
// multipass kernel, kChainCoefPad for the chain kernel): sweeps prefetch
// records past their last step, which are identity padding.
struct Plan {
    // lda, ldc, lds may be negative and cstep is 1 or -1: the inverse call
    // runs the forward sweep on a column-reversed view of A with C and S
    // read backwards (see run() in rotseq_host.cpp).
    int64_t m, n, k, lda, ldc, lds;
    int64_t cstep;  // step between C(j,p) and C(j+1,p) (and likewise S)
    int kernel;  // Kernel
    int band;    // sequences per band (K)
    int npass;   // number of bands
    int steps;   // padded wavefront steps per band
    int pad;     // identity records after the last step of each band
    int unroll;  // kernel unroll length (register ring size)
    int arith;
    int kind;    // Kind
    int esize;   // sizeof element: 8 (double) or 4 (float)
    // Launch shape of the chain kernel (configure_launch).
    int waves, nwg, remap, publish, spin_limit, wait_bias;
    int deep;  // streaming form: whole chains per workgroup (chain_unroll(band, true))
    size_t lds_bytes;
    int *status;  // sticky device error word (ROTSEQ_E_* bits)
    // Matrix-instruction sweep (kMfma): bands per wave, 16-row blocks per
    // wave, windows per band, band chunks and workgroups per tile chain,
    // row tiles, extra super-steps per later segment.  Its window matrices
    // live at off_coef.
    int mfma_ok;  // the workspace covers the matrix-instruction sweep
    int mfma_nb, mfma_rows, mfma_nwin, mfma_nchunks, mfma_nseg, mfma_tiles, mfma_seg_delay;
    // Workspace layout (byte offsets from the workspace base, 256-aligned).
    size_t off_coef, off_negmask, off_parity, off_sign, off_flags, total;
};

// One problem of a batch, as the batched kernels read it from device memory.
// The batched launches concatenate the problems' index spaces; the off_*
// fields are each problem's first index in the concatenation (ascending in
// item order), so a thread finds its problem by binary search.
struct BatchItem {
    void *A;
    const void *C, *S;
    int64_t lda, ldc, lds, m, n, k;
    int npass, steps, tiles, pad;
    uint64_t *negmask;
    uint8_t *parity;
    void *sign;  // T[n]
    void *coef;  // CoefPair<T>[npass * (steps + pad) * band]
    int *flags;  // int[tiles * npass]
    int *status; // this item's error word (ROTSEQ_E_* bits of its waits)
    int64_t off_negmask, off_parity, off_sign, off_coef, off_flags, off_wg;
    int64_t off_all;  // first index of the item in the coefficient/sign/flag stage
};

// Launch parameters shared by all items of a batch.
struct BatchLaunch {
    int count;         // items
    int esize, arith, band, waves, publish, spin_limit, wait_bias;
    size_t lds_bytes;
    int64_t total_negmask, total_parity, total_sign, total_coef, total_flags, nwg;
    int64_t total_all;  // index space of the coefficient/sign/flag stage
    const BatchItem *items;  // device copy, `count` entries
    size_t status_off;       // byte offset of the items' error words in the block
};

// One problem of a batch before layout (all fields as in rotseq_d).
struct BatchEntry {
    void *A;
    const void *C, *S;
    int64_t m, n, k, lda, ldc, lds;
};
// Lays out a batch in the given order: fills `items` and the totals of `L`
// (count, band, esize, total_*, status_off); every device pointer of an item
// is an offset from the start of one device block whose first bytes hold the
// item table, followed by one error word per item (status_off; the owner
// zeroes them).  Returns the block's size.  Host-only.
size_t batch_layout(const BatchEntry *entries, int count, int band, int esize,
                    std::vector<BatchItem> &items, BatchLaunch &L);
// Turns the offsets of batch_layout into addresses inside the block at `base`.
void batch_rebase(std::vector<BatchItem> &items, uintptr_t base);
// Workgroup ranges for `waves` waves per workgroup; returns their total.
int64_t batch_assign_workgroups(std::vector<BatchItem> &items, int waves);

hipError_t launch_prep_batch(const BatchLaunch &b, hipStream_t stream);
// Host helpers of rotseq_host.cpp shared with the batch runtime.
int check_problem(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda, const void *C,
                  int64_t ldc, const void *S, int64_t lds);
int device_query(int *cus, size_t *max_lds, int **status);
hipError_t launch_chain_batch(const BatchLaunch &b, hipStream_t stream);

// Fills the shape-only fields of `p` (kernel, band, npass, steps, unroll,
// workspace offsets) from its shape and the requested kernel and band
// (0 = auto).  Returns false for unsupported requests.  Host-only.
// `mfma_ok`: the problem may run on the matrix-instruction sweep (forward
// right application of rotations, FP64, automatic arithmetic); with the
// automatic kernel choice the workspace then covers it as well.
bool make_plan(Plan &p, int req_kernel, int req_band, bool mfma_ok = false);

// Polls before a wait between workgroups gives up, and the amount added to
// every such wait's target (0, or past any column count, so that every wait
// gives up: a test hook for the error path); set by rotseq_test_set_waits.
int wait_spin_limit();
int wait_bias();

// Error word of rotseq_noalloc_d on the current device (0 if it never ran
// there); `reset` clears it.  Host-only, synchronous.
int noalloc_status(int reset, int *value);

// Fills the launch shape of `p` for the current device (queries its CU count
// and occupancy).  `req_waves` > 0 forces the waves per workgroup.
// `req_shape` > 0 forces the matrix sweep's (bands, row blocks) per wave as
// 10 * bands + blocks.  hipErrorInvalidConfiguration: a forced matrix sweep
// has no shape that fits.
hipError_t configure_launch(Plan &p, int req_waves, int req_publish, int req_shape = 0);

// Register-ring length (= unroll length) of the sweep kernels for a band.
int unroll_for_band(int band);
// Step unroll of the chain kernel; `deep`: its streaming form, which launches
// whose bands all fit one workgroup use when there are at most
// kChainDeepBands of them (the memory-bound regime of small k), with at most
// kChainDeepWaves waves per workgroup.
constexpr int kChainDeepBands = 4;
constexpr int kChainDeepWaves = 8;
int chain_unroll(int band, bool deep);
size_t chain_lds_bytes(int band, int waves, int esize, bool deep = false);
hipError_t chain_occupancy(int band, int arith, int esize, int waves, size_t lds, int *blocks,
                           bool batch = false, bool deep = false);
hipError_t launch_chain(const Plan &p, void *A, const void *ws, hipStream_t stream);

// Matrix-instruction sweep (rotseq_mfma.hip).
constexpr int kMfmaFlagStride = 32;  // ints between progress flags (128 bytes)
bool mfma_shape_supported(int nb_wave, int rows);
int mfma_wave_stride(int nb_wave);
int mfma_waves();
int mfma_seg_delay(int nb_wave);
size_t mfma_lds_bytes(int rows);
hipError_t mfma_occupancy(int nb_wave, int rows, size_t lds, int *blocks);
hipError_t launch_mfma_prep(const Plan &p, const void *C, const void *S, void *ws, hipStream_t stream);
hipError_t launch_mfma(const Plan &p, void *A, const void *ws, hipStream_t stream);

// Launchers (rotseq_kernels.hip).  All are asynchronous on `stream` and
// return the hipError_t of the launch.
// p[0 .. count) = 0 by a kernel (also under graph capture).
hipError_t launch_prep(const Plan &p, const void *C, const void *S, void *ws,
                       hipStream_t stream);
hipError_t launch_sweep(const Plan &p, void *A, const void *ws, hipStream_t stream);
// dst (cols x rows, leading dimension ldd) = transpose of src (rows x cols,
// leading dimension lds_src); both column-major, esize 8 or 4.
hipError_t launch_transpose(const void *src, int64_t rows, int64_t cols, int64_t lds_src, void *dst,
                            int64_t ldd, int esize, hipStream_t stream);

}  // namespace rotseq
