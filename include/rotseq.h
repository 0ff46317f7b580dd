/*
 * librotseq: apply sequences of plane (Givens) rotations to a matrix on an
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (Steel & Langou, "Communication efficient application of
 * sequences of planar rotations to a matrix", Section 1, Algorithms 1 and 2):
 * given an m x n matrix A and k sequences of n-1 rotations stored as cosine
 * and sine matrices C and S of size (n-1) x k, overwrite A with
 *
 *     A <- A * G(0,0) G(1,0) ... G(n-2,0) G(0,1) ... G(n-2,k-1)
 *
 * where G(j,p) is the identity except in rows/columns j and j+1:
 *     G[j][j] = G[j+1][j+1] = c,  G[j+1][j] = s,  G[j][j+1] = -s,
 * with c = C(j,p), s = S(j,p).  Per row of A, rotation (j,p) does
 *     x' = c*x + s*y,   y' = -s*x + c*y      (x = A(i,j), y = A(i,j+1)).
 * Sequence p is applied after sequence p-1; within a sequence j ascends.
 * The library applies the rotations in a reordered but dependency-preserving
 * order (the wavefront of Section 1.1 and the blocks of Section 2), which
 * gives the same result up to rounding.
 *
 * Storage: all matrices are column-major with a leading dimension:
 *     A(i,j) = A[i + j*lda],  C(j,p) = C[j + p*ldc],  S(j,p) = S[j + p*lds].
 *
 * Pointers named "device" must be device memory of the current HIP device
 * (hipMalloc, or a torch CUDA/HIP tensor's data pointer); they stay owned by
 * the caller.  Calls are asynchronous and ordered on `stream` (0 = the null
 * stream); device inputs must stay valid until the stream has passed the call.
 * A must not overlap C, S or the workspace.  NaN or Inf inputs propagate.
 *
 * Return codes: 0 on success; -i if argument i (1-based) is invalid; a
 * positive ROTSEQ_E_* code for runtime failures.  rotseq_strerror() names them.
 */
#ifndef ROTSEQ_H
#define ROTSEQ_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ROTSEQ_SUCCESS        0
#define ROTSEQ_E_HIP          1  /* a HIP runtime call failed                   */
#define ROTSEQ_E_NOMEM        2  /* device workspace could not be allocated     */
#define ROTSEQ_E_WORKSPACE    3  /* caller workspace too small or misaligned    */
#define ROTSEQ_E_UNSUPPORTED  4  /* option combination not supported           */
#define ROTSEQ_E_TIMEOUT      5  /* a device-side wait exceeded its spin limit,
                                      or a server wait ran out of time           */
#define ROTSEQ_E_BUDGET       6  /* a matrix alone exceeds the server's budget  */
#define ROTSEQ_E_INVAL        7  /* unknown matrix id or ticket                 */
#define ROTSEQ_E_CLOSED       8  /* the matrix was closed                       */
#define ROTSEQ_E_FAILED       9  /* an earlier sweep of this matrix failed      */
#define ROTSEQ_E_TOO_LARGE   10  /* the problem's workspace exceeds the fixed
                                      scratch of rotseq_noalloc_d               */

/* Bit of the device status word (rotseq_device_status) set by the
 * preparation kernels of rotseq_refl_ex_{d,s} when a reflector with tau != 0
 * is not orthogonal (|tau (1 + nu^2) - 2| > 64 eps of the element type):
 * the result of that call is then not A H. */
#define ROTSEQ_STATUS_NOT_ORTHOGONAL (1 << 16)

/* Arithmetic used for one rotation (options.arith). */
#define ROTSEQ_ARITH_AUTO   0  /* library choice (currently ROTSEQ_ARITH_LIFT) */
/* Algorithm 1 exactly: two rounded products and one rounded sum per output,
 * no fused multiply-add.  Bitwise equal to a plain loop of Algorithm 2. */
#define ROTSEQ_ARITH_EXACT  1
/* Algorithm 1 with fused multiply-adds: x' = fma(c,x,s*y), y' = fma(c,y,-s*x). */
#define ROTSEQ_ARITH_FMA    2
/* Three fused multiply-adds per entry (shear/lifting factorisation of the
 * rotation, not from the paper):  x += a*y;  y += b*x;  x += a*y  with
 * a = s/(1+c), b = -s for c >= 0.  Rotations with c < 0 are applied as
 * (-c, -s) followed by negating both columns; the negations are tracked as
 * column signs and undone when A is written back, so |a| <= 1 always. */
#define ROTSEQ_ARITH_LIFT   3

/* Kernel family (options.kernel). */
#define ROTSEQ_KERNEL_AUTO      0
/* One wave per 64-row tile sweeps all k sequences in passes of `band`
 * sequences, reading and writing A once per pass. */
#define ROTSEQ_KERNEL_MULTIPASS 1
/* Chains of (tile, band) waves: consecutive bands of a tile hand columns to
 * each other through LDS inside a workgroup and through A (with device-scope
 * progress counters) across workgroups; one workgroup per CU.  Default. */
#define ROTSEQ_KERNEL_CHAIN     2
/* FP64 matrix instructions (v_mfma_f64_16x16x4f64): every band of 8
 * sequences is applied 8 wavefront steps at a time as a 16 x 16 window
 * matrix, accumulated once per call from C and S (the paper's GEMM-based
 * variant, Section 8); 4/3 of the counted flops are issued, on the matrix
 * units.  For FP64 right application of rotations in the forward order
 * (also left application, which runs it on a packed copy) with automatic
 * arithmetic; ROTSEQ_E_UNSUPPORTED otherwise.  ROTSEQ_KERNEL_AUTO picks it
 * where its modelled time is lower.  Results agree with the other kernels
 * up to rounding (not bitwise). */
#define ROTSEQ_KERNEL_MFMA      3

/*
 * Tuning options; zero-initialise for library defaults.
 *   arith   ROTSEQ_ARITH_*
 *   kernel  ROTSEQ_KERNEL_*
 *   band    sequences applied per wave per sweep over the columns
 *           (the paper's k_b, Section 2); 0 = auto.  MULTIPASS: 1, 2, 4,
 *           8 or 16; CHAIN: 2, 4, 6 or 8 (bands of 2 for single calls
 *           only, not batches).
 *   waves   CHAIN only: waves (bands) per workgroup, 1..16; 0 = auto
 *           (sized so the workgroups match the CU count).
 *   publish CHAIN only: columns between progress updates across
 *           workgroups (rounded up to a power of 2); 0 = auto (32).
 *   inverse nonzero: apply the inverse product instead,
 *               A <- A * (G(0,0) ... G(n-2,k-1))^T
 *                  = A * G(n-2,k-1)^T ... G(0,0)^T,
 *           i.e. the rotations in reverse order (p and j descending) with
 *           s negated; it undoes a forward call up to rounding.  In
 *           exact mode it equals that loop bitwise.  Not for batches.
 *   left    nonzero: the rotations mix adjacent ROWS of A instead of
 *           columns (application from the left, Section 4.3 of the paper).
 *           A is still m x n column-major with lda >= max(1,m), but C and S
 *           are (m-1) x k (ldc, lds >= max(1,m-1)), and rotation (j,p)
 *           applies the same per-pair formula to x = A(j,i), y = A(j+1,i)
 *           for every column i, in the order of Algorithm 2:
 *               A <- (G(0,0) ... G(m-2,k-1))^T A     (m x m rotations),
 *           and with `inverse` A <- G(0,0) ... G(m-2,k-1) A.
 *           A right application to a row-major r x q matrix B (row stride
 *           ldb) is a left application to the column-major q x r matrix
 *           with leading dimension ldb that is the same memory.
 *           The library packs A transposed into the workspace (m*n more
 *           elements, see rotseq_workspace_bytes), sweeps the packed copy
 *           and unpacks it.  Quick return if n == 0, m <= 1 or k == 0.
 *           Not for batches.
 *   shape   MFMA only: 10 * (bands chained in one wave, 1..3) + (blocks
 *           of 16 rows per wave), e.g. 35; 0 = auto.  Shapes without a
 *           compiled kernel return ROTSEQ_E_UNSUPPORTED.  With MFMA,
 *           `waves` (1..4) is the waves per workgroup.
 */
typedef struct rotseq_opts {
    int32_t arith;
    int32_t kernel;
    int32_t band;
    int32_t waves;
    int32_t publish;
    int32_t inverse;
    int32_t left;
    int32_t shape;
} rotseq_opts;

/*
 * The launch a call with these arguments would make on the current device
 * (kernel family, band, workgroup shape and workspace), without launching
 * anything.  Arguments 1-5 and `opts` as for rotseq_ex_d/_s with dtype 'd'
 * or 's' (pointers are not needed: the shape decides).  Returns 0, -i for
 * an invalid argument i (1 dtype, 2 m, 3 n, 4 k, 5 lda, 7 out), or
 * ROTSEQ_E_UNSUPPORTED / ROTSEQ_E_HIP.
 */
typedef struct rotseq_launch_info {
    int32_t kernel;         /* ROTSEQ_KERNEL_* that runs                    */
    int32_t band;           /* sequences per band                           */
    int32_t waves;          /* waves per workgroup                          */
    int32_t workgroups;     /* workgroups of the sweep launch               */
    int32_t bands_per_wave; /* MFMA: bands chained in one wave              */
    int32_t rows_per_wave;  /* MFMA: rows of A per wave                     */
    int32_t segments;       /* MFMA: workgroups along one tile's chain      */
    int32_t reserved;
    uint64_t workspace_bytes;
} rotseq_launch_info;
int rotseq_launch_describe(char dtype, int64_t m, int64_t n, int64_t k, int64_t lda,
                           const rotseq_opts *opts, rotseq_launch_info *out);

/*
 * rotseq_d: FP64 rotation sequence, A <- A * prod G(j,p) (Algorithms 1-2).
 *   1 m     rows of A, m >= 0
 *   2 n     columns of A, n >= 0
 *   3 k     number of rotation sequences, k >= 0
 *   4 A     device, m x n, lda >= max(1,m); updated in place
 *   5 lda   leading dimension of A
 *   6 C     device, (n-1) x k cosines, ldc >= max(1,n-1)
 *   7 ldc
 *   8 S     device, (n-1) x k sines, lds >= max(1,n-1)
 *   9 lds
 *  10 stream
 * Quick return (nothing is dereferenced) if m == 0, n <= 1 or k == 0.
 * The library keeps one cached device workspace per (device, stream); use
 * rotseq_ex_d with a caller workspace under HIP graph capture.
 */
int rotseq_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda,
             const double *C, int64_t ldc, const double *S, int64_t lds,
             hipStream_t stream);

/* rotseq_s: FP32 version of rotseq_d, same arguments and semantics. */
int rotseq_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda,
             const float *C, int64_t ldc, const float *S, int64_t lds,
             hipStream_t stream);

/*
 * rotseq_noalloc_d: rotseq_d for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, semantics, layouts and return codes as
 * rotseq_d, same kernels and launch shape (bitwise the same result), but
 * the call allocates nothing: its workspace lives in a fixed 128 MiB array
 * in device memory that the library holds on each device it runs on until
 * the process ends (the first 256 bytes hold this entry point's error
 * word, reported by rotseq_device_status).  A problem whose workspace
 * (rotseq_workspace_bytes('d', m, n, k, NULL)) exceeds 128 MiB - 256 bytes
 * returns ROTSEQ_E_TOO_LARGE before anything is launched; m = n = 10240
 * with k = 192 needs 71 MB.  The first call on a device looks up the
 * array's device address and clears its error word with a kernel on
 * `stream`.  Every call on a device uses that device's one array, so calls
 * that overlap on one device (on different streams, or from several host
 * threads) race and give wrong results: order them on one stream.
 */
int rotseq_noalloc_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda,
                     const double *C, int64_t ldc, const double *S, int64_t lds,
                     hipStream_t stream);

/*
 * rotseq_ex_d / rotseq_ex_s: as rotseq_d / rotseq_s with
 *  11 opts        tuning options or NULL for defaults
 *  12 workspace   device memory of at least rotseq_workspace_bytes(...)
 *                 bytes, 256-byte aligned, or NULL to use the cached pool
 *  13 ws_bytes    size of `workspace`
 * With a caller workspace nothing is allocated, so the call can be captured
 * into a HIP graph.  The workspace is in use until the stream passes the call.
 */
int rotseq_ex_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda,
                const double *C, int64_t ldc, const double *S, int64_t lds,
                hipStream_t stream, const rotseq_opts *opts,
                void *workspace, size_t ws_bytes);
int rotseq_ex_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda,
                const float *C, int64_t ldc, const float *S, int64_t lds,
                hipStream_t stream, const rotseq_opts *opts,
                void *workspace, size_t ws_bytes);

/*
 * rotseq_refl_ex_d / rotseq_refl_ex_s: sequences of 2x2 reflectors instead
 * of rotations (Section 6 of the paper: a reflector does the job of a
 * rotation with 3 multiplications and 3 additions per entry).  Reflector
 * (j,p) is LAPACK's elementary reflector with unit first component,
 *     H(j,p) = I - tau v v^T,   v = e_j + nu e_{j+1},
 *     tau = TAU(j,p) = TAU[j + p*ldt],  nu = NU(j,p) = NU[j + p*ldn],
 * and the call computes A <- A H(0,0) H(1,0) ... H(n-2,k-1) (per row:
 * w = x + nu*y, x' = x - tau*w, y' = y - tau*nu*w on columns j, j+1).
 * Arguments 1-13 as for rotseq_ex_d with TAU, ldt, NU, ldn in place of
 * C, ldc, S, lds; `opts` may ask for the inverse order (the same reflectors
 * with p and j descending) and for left application (rows j, j+1; TAU and
 * NU are then (m-1) x k).
 * Every reflector must be orthogonal: tau = 0 (the identity) or
 * tau * (1 + nu^2) = 2 up to rounding, as LAPACK's dlarfg produces.  The
 * library applies each one as a rotation followed by negating one column
 * (the negations are tracked and undone as in ROTSEQ_ARITH_LIFT), so
 * other values give results that are not A H.  The preparation kernels
 * check every reflector on the device and set ROTSEQ_STATUS_NOT_ORTHOGONAL
 * in the device status word (rotseq_device_status) when one is not
 * orthogonal to within 64 eps; the call itself returns before that check
 * runs.
 * ROTSEQ_ARITH_AUTO / ROTSEQ_ARITH_LIFT use that form (workspace as for
 * rotseq_ex_d).  ROTSEQ_ARITH_EXACT applies the formula as written, so any
 * (tau, nu) is accepted: the reflectors run on the 3x3 sweep as 3x3 ones
 * with nu2 = 0 (workspace: rotseq_refl3_ex_workspace_bytes for the same m,
 * n, k and `left`); forward order only, on either side (the inverse order,
 * or any other field set, gives ROTSEQ_E_UNSUPPORTED).  ROTSEQ_ARITH_FMA is
 * ROTSEQ_E_UNSUPPORTED.
 */
int rotseq_refl_ex_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda,
                     const double *TAU, int64_t ldt, const double *NU, int64_t ldn,
                     hipStream_t stream, const rotseq_opts *opts,
                     void *workspace, size_t ws_bytes);
int rotseq_refl_ex_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda,
                     const float *TAU, int64_t ldt, const float *NU, int64_t ldn,
                     hipStream_t stream, const rotseq_opts *opts,
                     void *workspace, size_t ws_bytes);

/*
 * rotseq_refl3_d / rotseq_refl3_s: sequences of 3x3 reflectors, as the
 * double-shift variant of the implicit QR algorithm needs (named among the
 * paper's future work, Section 9).  Reflector (j,p), 0 <= j < n-2, acts on
 * columns j, j+1, j+2:
 *     H(j,p) = I - tau v v^T,   v = e_j + nu1 e_{j+1} + nu2 e_{j+2},
 *     tau = TAU[j + p*ldt],  nu1 = NU1[j + p*ld1],  nu2 = NU2[j + p*ld2],
 * and the call computes A <- A H(0,0) H(1,0) ... H(n-3,0) H(0,1) ...
 * H(n-3,k-1).  Per row, with (x, y, z) = (A(i,j), A(i,j+1), A(i,j+2)):
 *     w = x + nu1*y + nu2*z;  x -= tau*w;  y -= tau*nu1*w;  z -= tau*nu2*w.
 * The formula is applied as written, so any (tau, nu1, nu2) is accepted
 * (orthogonal reflectors have tau*(1 + nu1^2 + nu2^2) = 2, or tau = 0).
 * Arguments: 1 m, 2 n, 3 k (>= 0); 4 A (device, m x n, column-major);
 * 5 lda >= max(1, m); 6 TAU (device, (n-2) x k); 7 ldt >= max(1, n-2);
 * 8 NU1, 9 ld1, 10 NU2, 11 ld2 likewise; 12 stream.  Quick return (nothing
 * launched) when m == 0, n <= 2 or k == 0; device pointers may then be NULL.
 * 13-14: optional device workspace of at least
 * rotseq_refl3_workspace_bytes() bytes, 256-byte aligned (NULL: the library
 * keeps one per device and stream; ROTSEQ_E_WORKSPACE if too small or
 * misaligned).  ROTSEQ_E_UNSUPPORTED if m > 2^31 - 65 or n > 2^30 - 1.
 * Right application in the forward order; rotseq_refl3_ex_* below also
 * takes the inverse order and application from the left.
 */
int rotseq_refl3_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda,
                   const double *TAU, int64_t ldt, const double *NU1, int64_t ld1,
                   const double *NU2, int64_t ld2, hipStream_t stream,
                   void *workspace, size_t ws_bytes);
int rotseq_refl3_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda,
                   const float *TAU, int64_t ldt, const float *NU1, int64_t ld1,
                   const float *NU2, int64_t ld2, hipStream_t stream,
                   void *workspace, size_t ws_bytes);
/* Workspace bytes of rotseq_refl3_{d,s} for this shape (dtype 'd' or 's');
 * 0 for quick-return shapes.  Host-only. */
size_t rotseq_refl3_workspace_bytes(char dtype, int64_t m, int64_t n, int64_t k);

/*
 * rotseq_refl3_ex_d / rotseq_refl3_ex_s: rotseq_refl3_{d,s} with options
 * (Section 4.3 of the paper for the side; the inverse order as for
 * rotations).  Arguments 1-12 and the workspace (14-15) as for
 * rotseq_refl3_d; 13 opts (host, may be NULL = forward, right), of which
 * only `inverse` and `left` may be set (every other field 0, else
 * ROTSEQ_E_UNSUPPORTED):
 *   inverse  A <- A * (H(0,0) ... H(n-3,k-1))^T = A * H(n-3,k-1) ... H(0,0),
 *            the same reflectors with p and j descending (each H is
 *            symmetric); for orthogonal reflectors it undoes a forward call.
 *   left     reflector (j,p) mixes ROWS j, j+1, j+2 (TAU, NU1, NU2 are then
 *            (m-2) x k, leading dimensions >= max(1, m-2)), with the same
 *            per-column formula:  A <- (H(0,0) ... H(m-3,k-1))^T A
 *            = H(m-3,k-1) ... H(0,0) A, and with `inverse`
 *            A <- H(0,0) ... H(m-3,k-1) A.  The library packs A transposed
 *            into the workspace (m*n more elements), sweeps the packed copy
 *            and unpacks it.  Quick return if n == 0, m <= 2 or k == 0.
 */
int rotseq_refl3_ex_d(int64_t m, int64_t n, int64_t k, double *A, int64_t lda,
                      const double *TAU, int64_t ldt, const double *NU1, int64_t ld1,
                      const double *NU2, int64_t ld2, hipStream_t stream,
                      const rotseq_opts *opts, void *workspace, size_t ws_bytes);
int rotseq_refl3_ex_s(int64_t m, int64_t n, int64_t k, float *A, int64_t lda,
                      const float *TAU, int64_t ldt, const float *NU1, int64_t ld1,
                      const float *NU2, int64_t ld2, hipStream_t stream,
                      const rotseq_opts *opts, void *workspace, size_t ws_bytes);
/* Workspace bytes of rotseq_refl3_ex_{d,s} for this shape and options (A with
 * lda = m); 0 for quick-return shapes and unsupported options.  Host-only. */
size_t rotseq_refl3_ex_workspace_bytes(char dtype, int64_t m, int64_t n, int64_t k,
                                       const rotseq_opts *opts);

/*
 * Device workspace bytes needed by rotseq_ex_{d,s} and rotseq_refl_ex_{d,s}
 * for this shape and options; dtype is 'd' or 's'.  Returns 0 for
 * quick-return shapes and for invalid arguments.  Host-only; never touches
 * the GPU.
 */
size_t rotseq_workspace_bytes(char dtype, int64_t m, int64_t n, int64_t k,
                              const rotseq_opts *opts);

/*
 * Argument check of rotseq_d/rotseq_s without launching anything: returns 0
 * or -i for the first invalid argument i as documented for rotseq_d.
 * Host-only; pointers are only compared with NULL.
 */
int rotseq_check_args(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                      const void *C, int64_t ldc, const void *S, int64_t lds);

/*
 * Kernel timing for benchmarks.  While enabled, every call records HIP
 * events on its own stream around the coefficient-preparation kernels and
 * around the sweep kernel.  rotseq_profile_read waits for the recorded events
 * (host-blocking), accumulates their durations into `out` and, if `reset` is
 * nonzero, clears the totals.  Not for use under HIP graph capture.
 */
typedef struct rotseq_profile {
    int64_t calls;        /* calls timed since the last reset            */
    double prep_ms;       /* total time of the preparation kernels       */
    double sweep_ms;      /* total time of the sweep kernel              */
    double sweep_ms_min;  /* fastest single sweep                        */
    double sweep_ms_max;  /* slowest single sweep                        */
} rotseq_profile;
int rotseq_profile_enable(int on);
int rotseq_profile_read(rotseq_profile *out, int reset);

/*
 * Sticky device-side error word of the current device, written by the
 * kernels of the plain calls (rotseq_d/_s, rotseq_ex_*, rotseq_refl_ex_*):
 * its low byte is ROTSEQ_E_TIMEOUT once a bounded wait between workgroups
 * has given up (the results of that call are then invalid; bits 8-15 say
 * which kind of wait), and ROTSEQ_STATUS_NOT_ORTHOGONAL is set when a
 * reflector call was given a reflector that is not orthogonal.  The word of
 * rotseq_noalloc_d (in its fixed array) is ORed in and reset with it.  Batch
 * plans and the server keep their own words (rotseq_batch_status, ticket
 * statuses).  This call synchronizes the device, returns the word and, if
 * `reset` is nonzero, clears it.
 */
int rotseq_device_status(int reset);

/*
 * Test hook for the error paths of the bounded waits.  Every chain sweep
 * launched after this call (plain calls, batch executions, server batches)
 * gives up a wait between workgroups after `spin_limit` polls (0 restores
 * the default, 2^22; -1 for a negative value), and with `unreachable`
 * nonzero every such wait asks for a column count no producer reaches, so
 * each one gives up: the kernels still run to completion, their results
 * are wrong, and the failure surfaces as documented for each call
 * (rotseq_device_status, rotseq_batch_status and rotseq_batched_*'s
 * return value, ticket statuses).  Process-wide; not for production use.
 */
int rotseq_test_set_waits(int32_t spin_limit, int32_t unreachable);

/*
 * Batches (many independent problems in one launch sequence).
 *
 * A batch is a host array of problem descriptors.  Each entry is a full
 * rotseq_d/rotseq_s call (same arguments, same semantics, same layouts);
 * the entries are independent and their A matrices must not overlap each
 * other (C and S may be shared).  All pointers are device pointers owned by
 * the caller.  Entries with nothing to do (m == 0, n <= 1 or k == 0) are
 * skipped.  The result equals a loop of rotseq_d/rotseq_s over the entries,
 * up to rounding (Section 1: each entry is Algorithm 2 on its own matrix).
 *
 * An invalid entry makes the call return -(1000*(idx+1) + argpos), where idx
 * is the 0-based entry and argpos the 1-based position of the offending
 * field in the rotseq_d argument list (1 m, 2 n, 3 k, 4 A, 5 lda, 6 C, 7 ldc,
 * 8 S, 9 lds); argpos 4 also flags an A that overlaps another entry's A.
 * count < 0 returns -1; probs == NULL with count > 0 returns -2.
 */
typedef struct rotseq_problem_d {
    int64_t m, n, k;
    double *A;
    int64_t lda;
    const double *C;
    int64_t ldc;
    const double *S;
    int64_t lds;
} rotseq_problem_d;

typedef struct rotseq_problem_s {
    int64_t m, n, k;
    float *A;
    int64_t lda;
    const float *C;
    int64_t ldc;
    const float *S;
    int64_t lds;
} rotseq_problem_s;

/*
 * rotseq_batched_d / rotseq_batched_s: one-shot batch.  Builds a batch plan,
 * runs it on `stream`, waits for the stream and frees the plan, so it blocks
 * until the batch is done.  Returns ROTSEQ_E_TIMEOUT if a bounded wait of
 * the sweep gave up (the results are then invalid).  For repeated batches
 * or HIP graph capture use the plan calls below.
 */
int rotseq_batched_d(int32_t count, const rotseq_problem_d *probs, hipStream_t stream);
int rotseq_batched_s(int32_t count, const rotseq_problem_s *probs, hipStream_t stream);

/*
 * Batch plans.  rotseq_batch_create_{d,s} validates the entries, sorts them
 * by decreasing work (longest chains are dispatched first), allocates and
 * fills the plan's device memory (descriptors and workspace; this call
 * synchronizes the device) and keeps the pointers: later executions use the
 * same A, C and S buffers, whose contents may change between executions.
 * `opts` as for rotseq_ex_d (kernel must be AUTO or CHAIN; band 4, 6 or 8;
 * waves 0 = planned); NULL for defaults.
 *
 * rotseq_batch_execute launches the whole batch on `stream`: one launch per
 * preparation stage over all entries, then one sweep launch over all
 * entries.  It allocates nothing and never synchronizes, so it can be
 * captured into a HIP graph; executions of one plan must not overlap.
 *
 * rotseq_batch_tune times the batch on `stream` for each candidate number of
 * waves per workgroup (`reps` timed executions each, after one warm-up) and
 * keeps the fastest.  It applies the rotations (1 + reps) times per
 * candidate, so the A buffers change; it blocks until done.
 *
 * rotseq_batch_destroy frees the plan (waits for the device first).
 */
typedef struct rotseq_batch rotseq_batch;

typedef struct rotseq_batch_info {
    int32_t count;      /* entries with work                                */
    int32_t band;       /* sequences per band                               */
    int32_t waves;      /* waves (bands) per workgroup of the sweep launch  */
    int32_t reserved;
    int64_t workgroups; /* workgroups of the sweep launch                   */
    int64_t waves_total;/* band-waves over all entries                      */
    double flops;       /* 6 m (n-1) k summed over entries                  */
    double bytes;       /* compulsory bytes: w (2 m n + 2 (n-1) k) summed   */
    size_t device_bytes;/* device memory held by the plan                   */
} rotseq_batch_info;

int rotseq_batch_create_d(int32_t count, const rotseq_problem_d *probs, const rotseq_opts *opts,
                          rotseq_batch **out);
int rotseq_batch_create_s(int32_t count, const rotseq_problem_s *probs, const rotseq_opts *opts,
                          rotseq_batch **out);
int rotseq_batch_execute(rotseq_batch *batch, hipStream_t stream);
/*
 * rotseq_batch_update_{d,s}: point an existing plan at other buffers.
 * `probs` lists the same entries as at creation, in the same order and with
 * the same m, n and k; A, C, S and the leading dimensions may change (and
 * are checked as at creation, overlap of the A ranges included).  Later
 * executions, and replays of a graph that captured rotseq_batch_execute,
 * use the new buffers.
 *   1 batch   the plan (-1 if NULL)
 *   2 count   entries (-2 unless it equals the plan's count, or if probs is
 *             NULL with count > 0; also -2 for a plan of the other type)
 *   3 probs   host array
 * An entry whose shape differs returns -(1000*(idx+1) + 1, 2 or 3) for m, n
 * or k; other invalid entries as rotseq_batch_create_d.  The item table is
 * rewritten after synchronizing the device, so no execution of the plan may
 * be in flight.  The plan is unchanged when an error is returned.
 */
int rotseq_batch_update_d(rotseq_batch *batch, int32_t count, const rotseq_problem_d *probs);
int rotseq_batch_update_s(rotseq_batch *batch, int32_t count, const rotseq_problem_s *probs);
int rotseq_batch_tune(rotseq_batch *batch, hipStream_t stream, int32_t reps);
/*
 * rotseq_batch_status: error words of a plan's entries.  Every entry keeps
 * a sticky word (zero at creation) into which its sweep records
 * ROTSEQ_E_TIMEOUT when a bounded wait between workgroups gives up, which
 * leaves that entry's A invalid.  Synchronizes the device, then writes each
 * entry's ROTSEQ_E_* code (0 if none) to per_problem[i] for the entries in
 * creation order (per_problem may be NULL; else it holds `count` entries)
 * and, if `reset` is nonzero, clears the words.  Returns 0, ROTSEQ_E_TIMEOUT
 * if any entry failed, -1 for a NULL plan or ROTSEQ_E_HIP.
 */
int rotseq_batch_status(rotseq_batch *batch, int32_t *per_problem, int reset);
int rotseq_batch_info_get(const rotseq_batch *batch, rotseq_batch_info *info);
int rotseq_batch_destroy(rotseq_batch *batch);

/*
 * Serving: resident matrices, each swept many times.
 *
 * A server keeps matrices resident in device memory (the paper keeps A
 * packed across repeated applications, Section 4; the setting is repeated
 * sweeps over the same matrix as in QR-type iterations, Section 5).  Clients
 * open a matrix (its host data is copied at the call), submit sweeps (k
 * sequences each; C and S are host arrays copied at the call, so the caller
 * may reuse them at once), wait for tickets, read the matrix back and close
 * it.  Sweeps of one matrix run in submission order; sweeps of different
 * matrices are batched together (one preparation launch per stage and one
 * sweep launch per batch, the batch path above) by a worker thread, with
 * the host-to-device copies of the next batch overlapping the current one.
 *
 * Admission: an opened matrix stays pending until its bytes (8*lda*n) fit
 * in the budget next to the resident ones; opens are admitted in order.
 * FP64 only.  All calls are thread-safe.  Host pointers are read during the
 * call only (open, submit) or written during the call (read).
 */
typedef struct rotseq_server rotseq_server;
typedef int64_t rotseq_matrix_id;
typedef int64_t rotseq_ticket;

typedef struct rotseq_server_config {
    uint64_t hbm_budget_bytes; /* resident matrices; 0 = 64 GiB              */
    int32_t max_batch;         /* sweeps per launch; 0 = 512                 */
    int32_t reserved[5];
} rotseq_server_config;

typedef struct rotseq_sweep_info {
    int32_t status;            /* 0, or the ROTSEQ_E_* code of the failure
                                  (ROTSEQ_E_TIMEOUT: a bounded wait of the
                                  sweep kernel gave up, so A is invalid;
                                  the matrix's later sweeps then fail with
                                  ROTSEQ_E_FAILED)                          */
    int32_t reserved;
    double submit_us;          /* host clock, microseconds since create      */
    double start_us;           /* its batch was launched                     */
    double end_us;             /* its batch was seen complete                */
} rotseq_sweep_info;

typedef struct rotseq_server_stats {
    int64_t sweeps_done;
    int64_t sweeps_failed;
    int64_t batches;
    int64_t matrices_resident;
    int64_t matrices_pending;
    uint64_t resident_bytes;
    uint64_t peak_resident_bytes;
    double flops;              /* 6 m (n-1) k over completed sweeps          */
    double busy_s;             /* first submit to last completion            */
    double gflops;             /* flops / busy_s / 1e9                       */
    double p50_us, p99_us;     /* sweep latency (submit to completion)       */
    double mean_batch;         /* sweeps per launch                          */
} rotseq_server_stats;

/* Creates a server on the current device (its worker thread starts here).
 * cfg NULL = defaults.  Returns 0, -1 (bad cfg) or -2 (out NULL), or an
 * ROTSEQ_E_* code. */
int rotseq_server_create(const rotseq_server_config *cfg, rotseq_server **out);
/* Opens an m x n matrix (column-major host data, lda >= max(1,m)); returns
 * at once with its id, admission may come later.  -i for a bad argument i,
 * ROTSEQ_E_BUDGET if 8*max(1,m)*n exceeds the whole budget. */
int rotseq_server_open(rotseq_server *srv, int64_t m, int64_t n, const double *A_host,
                       int64_t lda, rotseq_matrix_id *id);
/* Appends a sweep of k sequences (C, S host, (n-1) x k, column-major with
 * ldc, lds >= max(1,n-1)) to matrix `id`; returns its ticket. */
int rotseq_server_submit(rotseq_server *srv, rotseq_matrix_id id, int64_t k, const double *C_host,
                         int64_t ldc, const double *S_host, int64_t lds, rotseq_ticket *ticket);
/* Waits up to timeout_us (< 0: forever) for a ticket; fills `info` (may be
 * NULL).  Returns the sweep's status, or ROTSEQ_E_TIMEOUT / ROTSEQ_E_INVAL. */
int rotseq_server_wait(rotseq_server *srv, rotseq_ticket ticket, int64_t timeout_us,
                       rotseq_sweep_info *info);
/* Waits for every sweep submitted to `id` before this call, then copies the
 * matrix to A_host (lda >= max(1,m)).  Blocks. */
int rotseq_server_read(rotseq_server *srv, rotseq_matrix_id id, double *A_host, int64_t lda);
/* Closes `id`: its queued sweeps still run, then its device memory is freed.
 * Later submits and reads of `id` return ROTSEQ_E_CLOSED. */
int rotseq_server_close(rotseq_server *srv, rotseq_matrix_id id);
int rotseq_server_stats_get(rotseq_server *srv, rotseq_server_stats *stats);
/* Runs everything queued, stops the worker and frees all device memory. */
int rotseq_server_destroy(rotseq_server *srv);

/*
 * Measured FP64 ceilings of the current device (a synchronous diagnostic).
 * Launches one workgroup of `waves` waves (1..16) per CU; every wave runs 8
 * independent dependency chains for `iters` iterations (a positive multiple
 * of 4) of
 *   mode 1: v_fmac_f64 with register operands,
 *   mode 2: v_fmac_f64 with one operand broadcast by DPP row_newbcast (the
 *           form of the rotation sweep's coefficients),
 *   mode 3: v_mfma_f64_16x16x4f64 (2048 flops each),
 *   mode 4: half the waves mode 2, half mode 3, both kinds on every SIMD
 *           (`waves` a multiple of 8), which shows whether the vector and
 *           matrix units overlap,
 *   mode 5: mode 3 with, after every 8 matrix instructions, 8 doubles per
 *           lane written to LDS and read back into the next B operands (the
 *           LDS traffic of a sweep built on matrix instructions).
 * Fills `out` with the kernel time (HIP events), the FP64 flops done by each
 * kind of instruction and the average shader clock over the run (shader
 * cycle counter against the 100 MHz real-time counter).  Returns 0, -i for
 * a bad argument i, or ROTSEQ_E_NOMEM / ROTSEQ_E_HIP.  Allocates and frees
 * small device buffers; blocks until done.
 */
typedef struct rotseq_ceiling_result {
    double ms;          /* kernel duration                                  */
    double valu_flops;  /* FP64 flops of the vector FMAs                    */
    double mfma_flops;  /* FP64 flops of the matrix instructions            */
    double clock_mhz;   /* average shader clock during the kernel           */
} rotseq_ceiling_result;
int rotseq_fp64_ceiling(int32_t mode, int32_t waves, int64_t iters, rotseq_ceiling_result *out);

/* Static description of a return code. */
const char *rotseq_strerror(int code);

/* Library version as major*10000 + minor*100 + patch. */
int rotseq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ROTSEQ_H */
