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
 * composition), norm invariants and a round trip.  The left application is
 * pinned by dense products Q^T A and Q A, column-norm invariance, a row swap
 * closed form and bitwise agreement with the right application on A^T; the
 * reflector sequences by dense products of I - tau v v^T (orthogonal and
 * arbitrary tau), annihilation of a row into its last entry, the tau = 0 and
 * (tau, nu) = (2, 0) closed forms, norm invariance and a round trip; the
 * 3x3 reflector sequences by dense products, a norm transfer into entry n-2,
 * the tau = 0 and (tau, nu1, nu2) = (2, 0, 0) closed forms, bitwise agreement
 * with the 2x2 reflectors when nu2 = 0, and row-norm invariance.
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

/*
 * Left application (Section 4.3 of the paper names it as the row-wise twin of
 * the right application, equivalently a right application to a row-major
 * matrix).  Rotation (j, p) mixes the adjacent ROWS j and j+1 of A with the
 * same per-pair formula as Algorithm 1; per column i:
 *   t = c*A(j,i) + s*A(j+1,i);  A(j+1,i) = -s*A(j,i) + c*A(j+1,i);  A(j,i) = t.
 * For p = 0..k-1, for j = 0..m-2 (the order of Algorithm 2).  In matrix form
 *   A <- (G(0,0) G(1,0) ... G(m-2,k-1))^T A
 * with m x m rotations G(j,p) as above; C and S are (m-1) x k.
 */
static void rot_rows(int64_t ncols, double *x, double *y, int64_t ld, double c, double s)
{
    for (int64_t i = 0; i < ncols; ++i) {
        double t = c * x[i * ld] + s * y[i * ld];
        y[i * ld] = -s * x[i * ld] + c * y[i * ld];
        x[i * ld] = t;
    }
}

void oracle_rotseq_left_d(int64_t m, int64_t n, int64_t k,
                          double *A, int64_t lda,
                          const double *C, int64_t ldc,
                          const double *S, int64_t lds)
{
    for (int64_t p = 0; p < k; ++p)
        for (int64_t j = 0; j + 1 < m; ++j)
            rot_rows(n, &A[j], &A[j + 1], lda, C[j + p * ldc], S[j + p * lds]);
}

/*
 * Inverse of oracle_rotseq_left_d: A <- G(0,0) ... G(m-2,k-1) A.  The
 * rightmost factor acts first, and G(j,p) acting on a row pair from the left
 * is the per-pair formula with (c, -s): p = k-1..0, j = m-2..0.
 */
void oracle_rotseq_left_inverse_d(int64_t m, int64_t n, int64_t k,
                                  double *A, int64_t lda,
                                  const double *C, int64_t ldc,
                                  const double *S, int64_t lds)
{
    for (int64_t p = k - 1; p >= 0; --p)
        for (int64_t j = m - 2; j >= 0; --j)
            rot_rows(n, &A[j], &A[j + 1], lda, C[j + p * ldc], -S[j + p * lds]);
}

/*
 * Sequences of 2x2 reflectors (Section 6 of the paper: a reflector plays the
 * role of a rotation at 3 multiplications and 3 additions per entry).  The
 * paper does not fix a parametrisation; the one read here is LAPACK's
 * elementary reflector with unit first component:
 *   H(j,p) = I - tau v v^T,  v = e_j + nu e_{j+1},
 *   tau = TAU(j,p) = TAU[j + p*ldt],  nu = NU(j,p) = NU[j + p*ldn].
 * Applied from the right to the column pair (x, y) = (A(i,j), A(i,j+1)):
 *   w = x + nu*y;  x' = x - tau*w;  y' = y - (tau*nu)*w
 * which is the 3 + 3 operation count (tau*nu is formed once per reflector).
 * H is orthogonal (and its own inverse) when tau = 0 or tau*(1 + nu^2) = 2;
 * the functions below apply the formula as written for any tau and nu.
 */
static void refl(int64_t len, double *x, double *y, int64_t stride, double tau, double nu)
{
    double tn = tau * nu;
    for (int64_t i = 0; i < len; ++i) {
        double w = x[i * stride] + nu * y[i * stride];
        x[i * stride] = x[i * stride] - tau * w;
        y[i * stride] = y[i * stride] - tn * w;
    }
}

/* A <- A H(0,0) H(1,0) ... H(n-2,k-1), in the order of Algorithm 2. */
void oracle_reflseq_d(int64_t m, int64_t n, int64_t k,
                      double *A, int64_t lda,
                      const double *TAU, int64_t ldt,
                      const double *NU, int64_t ldn)
{
    for (int64_t p = 0; p < k; ++p)
        for (int64_t j = 0; j + 1 < n; ++j)
            refl(m, &A[j * lda], &A[(j + 1) * lda], 1, TAU[j + p * ldt], NU[j + p * ldn]);
}

/*
 * A <- A H(n-2,k-1) ... H(0,0): the same reflectors in reverse order
 * (p = k-1..0, j = n-2..0).  For orthogonal reflectors (H^-1 = H^T = H) this
 * undoes oracle_reflseq_d.
 */
void oracle_reflseq_inverse_d(int64_t m, int64_t n, int64_t k,
                              double *A, int64_t lda,
                              const double *TAU, int64_t ldt,
                              const double *NU, int64_t ldn)
{
    for (int64_t p = k - 1; p >= 0; --p)
        for (int64_t j = n - 2; j >= 0; --j)
            refl(m, &A[j * lda], &A[(j + 1) * lda], 1, TAU[j + p * ldt], NU[j + p * ldn]);
}

/*
 * Reflectors mixing adjacent ROWS: the per-pair formula above with
 * (x, y) = (A(j,i), A(j+1,i)) for every column i, p = 0..k-1, j = 0..m-2;
 * A <- (H(0,0) ... H(m-2,k-1))^T A.  TAU and NU are (m-1) x k.
 */
void oracle_reflseq_left_d(int64_t m, int64_t n, int64_t k,
                           double *A, int64_t lda,
                           const double *TAU, int64_t ldt,
                           const double *NU, int64_t ldn)
{
    for (int64_t p = 0; p < k; ++p)
        for (int64_t j = 0; j + 1 < m; ++j)
            refl(n, &A[j], &A[j + 1], lda, TAU[j + p * ldt], NU[j + p * ldn]);
}

/*
 * Sequences of 3x3 reflectors, the double-shift QR case of Section 9 (the
 * paper's outlook).  Reflector (j, p) mixes columns j, j+1, j+2:
 *   H(j,p) = I - tau v v^T,  v = e_j + nu1 e_{j+1} + nu2 e_{j+2},
 *   tau = TAU(j,p), nu1 = NU1(j,p), nu2 = NU2(j,p); TAU, NU1, NU2 are
 *   (n-2) x k with leading dimensions ldt, ld1, ld2.
 * Per row, with (x, y, z) = (A(i,j), A(i,j+1), A(i,j+2)):
 *   w = x + nu1*y + nu2*z;  x -= tau*w;  y -= (tau*nu1)*w;  z -= (tau*nu2)*w.
 * In the order of Algorithm 2: for p = 0..k-1, for j = 0..n-3;
 * A <- A H(0,0) H(1,0) ... H(n-3,k-1).
 */
void oracle_refl3seq_d(int64_t m, int64_t n, int64_t k,
                       double *A, int64_t lda,
                       const double *TAU, int64_t ldt,
                       const double *NU1, int64_t ld1,
                       const double *NU2, int64_t ld2)
{
    for (int64_t p = 0; p < k; ++p)
        for (int64_t j = 0; j + 2 < n; ++j) {
            double tau = TAU[j + p * ldt], nu1 = NU1[j + p * ld1], nu2 = NU2[j + p * ld2];
            double t1 = tau * nu1, t2 = tau * nu2;
            double *x = &A[j * lda], *y = &A[(j + 1) * lda], *z = &A[(j + 2) * lda];
            for (int64_t i = 0; i < m; ++i) {
                double w = x[i] + nu1 * y[i] + nu2 * z[i];
                x[i] = x[i] - tau * w;
                y[i] = y[i] - t1 * w;
                z[i] = z[i] - t2 * w;
            }
        }
}

/*
 * The inverse order: A <- A * (H(0,0) ... H(n-3,k-1))^T
 *                     = A * H(n-3,k-1) ... H(1,0) H(0,0)
 * (each H is symmetric), i.e. p descending and, within p, j descending,
 * with the per-row formula above.  For orthogonal reflectors it undoes a
 * forward call.
 */
void oracle_refl3seq_inverse_d(int64_t m, int64_t n, int64_t k,
                               double *A, int64_t lda,
                               const double *TAU, int64_t ldt,
                               const double *NU1, int64_t ld1,
                               const double *NU2, int64_t ld2)
{
    for (int64_t p = k - 1; p >= 0; --p)
        for (int64_t j = n - 3; j >= 0; --j) {
            double tau = TAU[j + p * ldt], nu1 = NU1[j + p * ld1], nu2 = NU2[j + p * ld2];
            double t1 = tau * nu1, t2 = tau * nu2;
            double *x = &A[j * lda], *y = &A[(j + 1) * lda], *z = &A[(j + 2) * lda];
            for (int64_t i = 0; i < m; ++i) {
                double w = x[i] + nu1 * y[i] + nu2 * z[i];
                x[i] = x[i] - tau * w;
                y[i] = y[i] - t1 * w;
                z[i] = z[i] - t2 * w;
            }
        }
}

/*
 * Application from the left (reflector (j, p) mixes ROWS j, j+1, j+2;
 * TAU, NU1, NU2 are (m-2) x k):
 *   forward: A <- (H(0,0) ... H(m-3,k-1))^T A = H(m-3,k-1) ... H(0,0) A,
 *            so H(0,0) meets A first: p ascending, j ascending;
 *   inverse: A <- H(0,0) ... H(m-3,k-1) A: p descending, j descending.
 * Per column i, with (x, y, z) = (A(j,i), A(j+1,i), A(j+2,i)), the same
 * formula as above.
 */
void oracle_refl3seq_left_d(int64_t m, int64_t n, int64_t k, int inverse,
                            double *A, int64_t lda,
                            const double *TAU, int64_t ldt,
                            const double *NU1, int64_t ld1,
                            const double *NU2, int64_t ld2)
{
    for (int64_t pp = 0; pp < k; ++pp)
        for (int64_t jj = 0; jj + 2 < m; ++jj) {
            const int64_t p = inverse ? k - 1 - pp : pp;
            const int64_t j = inverse ? m - 3 - jj : jj;
            double tau = TAU[j + p * ldt], nu1 = NU1[j + p * ld1], nu2 = NU2[j + p * ld2];
            double t1 = tau * nu1, t2 = tau * nu2;
            for (int64_t i = 0; i < n; ++i) {
                double *col = &A[i * lda];
                double w = col[j] + nu1 * col[j + 1] + nu2 * col[j + 2];
                col[j] = col[j] - tau * w;
                col[j + 1] = col[j + 1] - t1 * w;
                col[j + 2] = col[j + 2] - t2 * w;
            }
        }
}

