/*
 * CPU oracle for applying sequences of plane rotations to a matrix.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * Build (done by oracle/build.py):
 *   gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread
 *
 * -ffp-contract=off keeps every product and sum separately rounded (IEEE
 * binary64, round to nearest even), exactly as the formulas below are written.
 *
 * Storage convention (the paper only says "matrices of size (n-1) x k"; the
 * reading taken here is the BLAS/LAPACK column-major one):
 *   A(i, j) = A[i + j*lda],  0 <= i < m, 0 <= j < n,  lda >= max(1, m)
 *   C(j, p) = C[j + p*ldc],  0 <= j < n-1, 0 <= p < k,  ldc >= max(1, n-1)
 *   S(j, p) = S[j + p*lds],  same shape as C
 * Column p of C/S is rotation sequence p; row j is the rotation that mixes the
 * adjacent columns j and j+1 of A.
 *
 * Parity pins: every function here is pinned by CPU tests against brute
 * force (dense product of rotation matrices), exact rational arithmetic,
 * the BLAS drot routine, closed forms (swap, identity, reflection, n = 2
 * composition), norm invariants and a round trip.
 */
#include <stdint.h>
#include <stdlib.h>
#include <pthread.h>

/*
 * Algorithm 1 (rot): apply one rotation (c, s) to the column pair (x, y) of
 * length m.  Per entry:  t = c*x + s*y;  y = -s*x + c*y;  x = t.
 * That is 4 multiplications and 2 additions (6 flops) per entry.
 */
static void rot(int64_t m, double *x, double *y, double c, double s)
{
    for (int64_t i = 0; i < m; ++i) {
        double t = c * x[i] + s * y[i];
        y[i] = -s * x[i] + c * y[i];
        x[i] = t;
    }
}

/*
 * Algorithm 2 (rot_sequence): for p = 0..k-1, for j = 0..n-2, apply
 * rotation (j, p) to columns j and j+1 of A, i.e.
 *   A <- A * G(0,0) G(1,0) ... G(n-2,0) G(0,1) ... G(n-2,k-1)
 * where G(j,p) is the identity except G[j][j] = G[j+1][j+1] = c,
 * G[j+1][j] = s, G[j][j+1] = -s  (rotation applied from the right).
 * Only rows [0, m) of A are touched; rows are independent.
 */
void oracle_rotseq_d(int64_t m, int64_t n, int64_t k,
                     double *A, int64_t lda,
                     const double *C, int64_t ldc,
                     const double *S, int64_t lds)
{
    for (int64_t p = 0; p < k; ++p)
        for (int64_t j = 0; j + 1 < n; ++j)
            rot(m, &A[j * lda], &A[(j + 1) * lda], C[j + p * ldc], S[j + p * lds]);
}

/*
 * Inverse of oracle_rotseq_d: each G(j,p) is orthogonal with inverse
 * G(j,p)^T, which is the rotation (c, -s).  The product is undone by
 * applying the transposes in reverse order: p = k-1..0, j = n-2..0.
 */
void oracle_rotseq_inverse_d(int64_t m, int64_t n, int64_t k,
                             double *A, int64_t lda,
                             const double *C, int64_t ldc,
                             const double *S, int64_t lds)
{
    for (int64_t p = k - 1; p >= 0; --p)
        for (int64_t j = n - 2; j >= 0; --j)
            rot(m, &A[j * lda], &A[(j + 1) * lda], C[j + p * ldc], -S[j + p * lds]);
}

/*
 * Row-partitioned driver.  Rows of A never interact (every rotation mixes two
 * columns of the same row), so running Algorithm 2 on disjoint row ranges in
 * separate threads gives a bitwise identical result for any thread count.
 * Used only to time the oracle on all host cores.
 */
struct rows_job {
    int64_t m, n, k, lda, ldc, lds;
    double *A;
    const double *C, *S;
};

static void *rows_worker(void *arg)
{
    struct rows_job *j = (struct rows_job *)arg;
    oracle_rotseq_d(j->m, j->n, j->k, j->A, j->lda, j->C, j->ldc, j->S, j->lds);
    return NULL;
}

int oracle_rotseq_threads_d(int nthreads, int64_t m, int64_t n, int64_t k,
                            double *A, int64_t lda,
                            const double *C, int64_t ldc,
                            const double *S, int64_t lds)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    if ((int64_t)nthreads > m)
        nthreads = m > 0 ? (int)m : 1;
    pthread_t tid[256];
    struct rows_job job[256];
    int64_t per = (m + nthreads - 1) / nthreads;
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        int64_t r0 = (int64_t)t * per;
        int64_t r1 = r0 + per < m ? r0 + per : m;
        if (r0 >= r1)
            break;
        job[t].m = r1 - r0;
        job[t].n = n;
        job[t].k = k;
        job[t].lda = lda;
        job[t].ldc = ldc;
        job[t].lds = lds;
        job[t].A = A + r0;
        job[t].C = C;
        job[t].S = S;
        if (pthread_create(&tid[t], NULL, rows_worker, &job[t]) != 0)
            return -1;
        ++started;
    }
    for (int t = 0; t < started; ++t)
        pthread_join(tid[t], NULL);
    return started;
}
