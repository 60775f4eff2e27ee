/*
 * ST-HOSVD reference oracle: plain, slow, obviously correct FP64 CPU code.
 *
 * This is TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header or
 * constant with the GPU library; the GPU library never calls it.
 *
 * Layout convention (paper Sec. 4.1, eq. idxtolin): a tensor of sizes
 * J_0 x ... x J_{N-1} is a flat array in which element (j_0,...,j_{N-1}) sits
 * at sum_n j_n * prod_{k<n} J_k  (mode 0 fastest, "natural descending").
 * For a mode n write L = prod_{k<n} J_k and Rt = prod_{k>n} J_k; then
 * element (row a of the mode-n unfolding, block r, offset l) sits at
 * l + L*a + L*J_n*r  (paper Sec. 4.2: Rt row-major blocks of size J_n x L).
 *
 * Matrices are column-major unless stated.  All functions return 0 on
 * success and a negative value on invalid arguments.
 */
#ifndef TUCKER_ORACLE_H
#define TUCKER_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sum of squares of n values, accumulated sequentially (paper Sec. 2.2.2). */
double oracle_norm2(const double* x, int64_t n);

/* Materialise the mode-n unfolding Y_(n) (J_n x prod_{k!=n}J_k, row-major
 * output) from the index map of paper Sec. 2.2.1 / Sec. 4.2.  Test aid. */
int oracle_unfold(const double* Y, const int64_t* dims, int N, int n, double* out);

/* Gram matrix S = Y_(n) Y_(n)^T (paper Alg. 2), J_n x J_n, full symmetric,
 * written row-major (== column-major: it is symmetric).  Each entry is a
 * sum over the unfolding's columns in increasing column order. */
int oracle_gram(const double* Y, const int64_t* dims, int N, int n, double* S, int nthreads);

/* Symmetric eigendecomposition by cyclic-by-row two-sided Jacobi
 * (Golub & Van Loan, Matrix Computations, Sec. 8.5).  S is J x J (read
 * only).  On return lam[0..J) holds the eigenvalues in descending order and
 * V (column-major J x J) the matching eigenvectors.  Returns the number of
 * sweeps used, or -1 if max_sweeps was exceeded (not converged). */
int oracle_jacobi_eig(const double* S, int J, double* lam, double* V, int max_sweeps);

/* Truncation rule of paper eq. Un / Alg. 1: smallest R in {1..J} with
 * sum_{i>=R} max(lam_i,0) <= thr (lam descending, 0-based).  Writes the
 * discarded sum to *disc.  Returns R. */
int oracle_truncate(const double* lam, int J, double thr, double* disc);

/* Sign convention for factor columns: in each of the R columns of the
 * column-major I x R matrix U, the entry of largest magnitude (lowest row on
 * ties) is made positive by flipping the column if needed. */
void oracle_sign_fix(double* U, int64_t I, int64_t R);

/* Mode-n product Z = Y x_n M (paper Sec. 2.2.3 and Alg. 3), with M a K x J_n
 * matrix given by element (k,j) = M[k*msk + j*msj].  Z has the sizes of Y
 * with J_n replaced by K. */
int oracle_ttm(const double* Y, const int64_t* dims, int N, int n, const double* M,
               int64_t K, int64_t msk, int64_t msj, double* Z, int nthreads);

/* Sum of max(lam_i, 0) for i = R..J-1, accumulated from the last (smallest)
 * value upward: the energy discarded by keeping R leading eigenvectors. */
double oracle_tail(const double* lam, int J, int R);

/* Hyperslice statistics of mode n (paper Sec. 3.5): for every index i of
 * mode n, over the prod_{k!=n} J_k elements of that slice, stats[s*J_n + i]
 * holds s = 0 mean, 1 standard deviation (divided by the count), 2 minimum,
 * 3 maximum, 4 1-norm, 5 2-norm. */
int oracle_slice_stats(const double* Y, const int64_t* dims, int N, int n, double* stats);

/* Per-hyperslice affine map along mode n (paper Sec. 3.5): inverse == 0 gives
 * Z = (Y - shift_i) / scale_i, inverse != 0 gives Z = fma(Y, scale_i, shift_i). */
int oracle_slice_transform(const double* Y, const int64_t* dims, int N, int n, const double* shift,
                           const double* scale, int inverse, double* Z);

#ifdef __cplusplus
}
#endif
#endif
