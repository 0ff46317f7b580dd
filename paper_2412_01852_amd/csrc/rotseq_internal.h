// Internal interfaces between the host runtime and the HIP kernels of
// librotseq.  Not installed; the public interface is include/rotseq.h.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace rotseq {

// Per-rotation arithmetic (values of rotseq_opts.arith after resolving AUTO).
enum Arith : int { kExact = 1, kFma = 2, kLift = 3 };

// Shape of one call after dispatch decisions: A is m x n (column-major, lda),
// the k sequences are cut into `npass` bands of `band` sequences (the last
// band is padded with identity rotations), and every sweep over the columns
// takes `steps` wavefront steps (n + band - 1 rounded up to the kernel's
// unroll length; steps past the last real one are identity).
struct Plan {
    int64_t m, n, k, lda, ldc, lds;
    int band;    // sequences per band (K)
    int npass;   // number of bands
    int steps;   // padded wavefront steps per band
    int unroll;  // kernel unroll length (register ring size)
    int arith;
    int esize;   // sizeof element: 8 (double) or 4 (float)
    // Workspace layout (byte offsets from the workspace base, 256-aligned).
    size_t off_coef, off_negmask, off_parity, off_sign, total;
};

// Fills the dispatch fields of `p` (band, npass, steps, unroll, offsets)
// from its shape and the requested band (0 = auto).  Returns false when the
// requested band is not supported.
bool make_plan(Plan &p, int req_band);

// Register-ring length (= unroll length) of the sweep kernel for a band.
int unroll_for_band(int band);

// Launchers (rotseq_kernels.hip).  All are asynchronous on `stream` and
// return the hipError_t of the launch.
hipError_t launch_prep(const Plan &p, const void *C, const void *S, void *ws,
                       hipStream_t stream);
hipError_t launch_sweep(const Plan &p, void *A, const void *ws, hipStream_t stream);

}  // namespace rotseq
