// Internal interface of the 3x3 reflector sweep (rotseq_refl3.hip) for the
// host runtime.  Not installed; the public interface is include/rotseq.h.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace rotseq {

// Sequences of 3x3 reflectors (rotseq_refl3_*): bands of `band` sequences,
// one wave per band, at most `waves` bands per launch; records of
// (tau, nu1, nu2) in wavefront order, `steps` local steps per band.
struct Refl3Plan {
    int64_t m, n, k, lda;
    int esize, band, nbands, steps, waves;
    int64_t rec_elems;  // elements of the record buffer
    int64_t nrefl;      // reflectors per sequence: n-2 (n-1 for 2x2 ones, nu2 = 0)
    size_t total;       // workspace bytes
};
// Fills `p` for a call with work (m > 0, n >= width, k > 0) of reflectors
// `width` columns wide (3, or 2: 2x2 reflectors run as 3x3 ones with
// nu2 = 0); false if the shape is outside what the kernel indexes with
// 32-bit integers.  Host-only.
bool refl3_plan(Refl3Plan &p, int64_t m, int64_t n, int64_t k, int64_t lda, int esize,
                int width = 3);
// cj: step between the records of reflectors j and j+1 in TAU, NU1, NU2
// (1, or -1 with negative leading dimensions: the inverse order).
hipError_t launch_refl3_prep(const Refl3Plan &p, const void *TAU, int64_t ldt, const void *NU1,
                             int64_t ld1, const void *NU2, int64_t ld2, int64_t cj, void *ws,
                             hipStream_t stream);
// rev: A is a column-reversed view (negative lda) and the reflectors are
// read in the inverse order, so each one's unit component is its third column.
hipError_t launch_refl3_sweep(const Refl3Plan &p, void *A, const void *ws, bool rev,
                              hipStream_t stream);

}  // namespace rotseq
