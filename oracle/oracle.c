/*
 * ST-HOSVD reference oracle: plain FP64 CPU loops.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the GPU library never
 * calls it and shares no code with it.
 *
 * Every output entry is produced by exactly one thread with a fixed
 * summation order, so results do not depend on the thread count.
 * Built with -O2 and without -ffast-math: the compiler may not reassociate.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* L = prod_{k<n} J_k, Rt = prod_{k>n} J_k (paper Sec. 2.1, the "left" and
 * "right" products; both are 1 at the ends). */
static void left_right(const int64_t* dims, int N, int n, int64_t* L, int64_t* Rt) {
  int64_t l = 1, r = 1;
  for (int k = 0; k < n; ++k) l *= dims[k];
  for (int k = n + 1; k < N; ++k) r *= dims[k];
  *L = l;
  *Rt = r;
}

static int check_shape(const int64_t* dims, int N, int n) {
  if (!dims || N < 1 || n < 0 || n >= N) return -1;
  for (int k = 0; k < N; ++k)
    if (dims[k] < 1) return -1;
  return 0;
}

double oracle_norm2(const double* x, int64_t n) {
  /* paper Sec. 2.2.2: ||X||^2 is the sum of squares of all elements */
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += x[i] * x[i];
  return s;
}

int oracle_unfold(const double* Y, const int64_t* dims, int N, int n, double* out) {
  /* Element (j_0..j_{N-1}) goes to row j_n and column
   * sum_{k<n} j_k L_k + sum_{k>n} j_k L_k / J_n   (paper Sec. 2.2.1),
   * where L_k = prod_{m<k} J_m.  Enumerating the tensor in storage order and
   * decoding the multi-index keeps this literal. */
  if (check_shape(dims, N, n)) return -1;
  int64_t total = 1;
  for (int k = 0; k < N; ++k) total *= dims[k];
  const int64_t Jn = dims[n];
  const int64_t cols = total / Jn;
  for (int64_t lin = 0; lin < total; ++lin) {
    int64_t rem = lin, Lk = 1, col = 0, row = 0;
    for (int k = 0; k < N; ++k) {
      int64_t jk = rem % dims[k];
      rem /= dims[k];
      if (k < n) col += jk * Lk;
      else if (k > n) col += jk * (Lk / Jn);
      else row = jk;
      Lk *= dims[k];
    }
    out[row * cols + col] = Y[lin];
  }
  return 0;
}

int oracle_gram(const double* Y, const int64_t* dims, int N, int n, double* S, int nthreads) {
  /* paper Alg. 2: S = sum over the Rt block columns of (block)(block)^T, each
   * block the J_n x L row-major submatrix at offset L*J_n*r.  Column (r,l) of
   * the unfolding holds Y[l + L*a + L*J_n*r] in row a.  Each S[a][b] is the
   * sum over columns in increasing (r, l) order. */
  if (check_shape(dims, N, n) || !Y || !S) return -1;
  int64_t L, Rt;
  left_right(dims, N, n, &L, &Rt);
  const int64_t J = dims[n];
  memset(S, 0, sizeof(double) * (size_t)(J * J));
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    int T = 1, t = 0;
#ifdef _OPENMP
    T = omp_get_num_threads();
    t = omp_get_thread_num();
#endif
    double* y = (double*)malloc(sizeof(double) * (size_t)J);
    /* thread t owns the rows a = t, t+T, ... of the upper triangle */
    for (int64_t r = 0; r < Rt; ++r)
      for (int64_t l = 0; l < L; ++l) {
        for (int64_t a = 0; a < J; ++a) y[a] = Y[l + L * a + L * J * r];
        for (int64_t a = t; a < J; a += T)
          for (int64_t b = a; b < J; ++b) S[a * J + b] += y[a] * y[b];
      }
    free(y);
  }
  for (int64_t a = 0; a < J; ++a)
    for (int64_t b = 0; b < a; ++b) S[a * J + b] = S[b * J + a];
  return 0;
}

int oracle_jacobi_eig(const double* S, int J, double* lam, double* V, int max_sweeps) {
  /* Cyclic-by-row two-sided Jacobi (Golub & Van Loan Sec. 8.5): sweep over
   * all pairs p<q in row order; for each, the 2x2 symmetric Schur
   * decomposition picks (c,s) that zero A[p][q]; A <- J^T A J, V <- V J.
   * A pair is skipped when |a_pq| is negligible against sqrt(|a_pp a_qq|)
   * (unit roundoff) or against 1e-30*||S||_F; a sweep with no rotation ends
   * the iteration. */
  if (J < 1 || !S || !lam || !V) return -1;
  const size_t JJ = (size_t)J * (size_t)J;
  double* A = (double*)malloc(sizeof(double) * JJ);
  memcpy(A, S, sizeof(double) * JJ);
  for (size_t i = 0; i < JJ; ++i) V[i] = 0.0;
  for (int i = 0; i < J; ++i) V[(size_t)i * J + i] = 1.0;
  double fro = 0.0;
  for (size_t i = 0; i < JJ; ++i) fro += A[i] * A[i];
  fro = sqrt(fro);
  const double abs_floor = 1e-30 * fro;

  int sweeps = 0, converged = (J == 1);
  while (!converged) {
    if (sweeps >= max_sweeps) break;
    ++sweeps;
    int rotated = 0;
    for (int p = 0; p < J - 1; ++p)
      for (int q = p + 1; q < J; ++q) {
        const double apq = A[(size_t)p * J + q];
        const double app = A[(size_t)p * J + p];
        const double aqq = A[(size_t)q * J + q];
        if (fabs(apq) <= DBL_EPSILON * sqrt(fabs(app)) * sqrt(fabs(aqq)) || fabs(apq) <= abs_floor)
          continue;
        ++rotated;
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = t * c;
        for (int k = 0; k < J; ++k) {
          if (k == p || k == q) continue;
          const double akp = A[(size_t)k * J + p], akq = A[(size_t)k * J + q];
          const double nkp = c * akp - s * akq, nkq = s * akp + c * akq;
          A[(size_t)k * J + p] = nkp;
          A[(size_t)p * J + k] = nkp;
          A[(size_t)k * J + q] = nkq;
          A[(size_t)q * J + k] = nkq;
        }
        A[(size_t)p * J + p] = app - t * apq;
        A[(size_t)q * J + q] = aqq + t * apq;
        A[(size_t)p * J + q] = 0.0;
        A[(size_t)q * J + p] = 0.0;
        for (int k = 0; k < J; ++k) { /* V <- V J, V column-major */
          const double vkp = V[(size_t)p * J + k], vkq = V[(size_t)q * J + k];
          V[(size_t)p * J + k] = c * vkp - s * vkq;
          V[(size_t)q * J + k] = s * vkp + c * vkq;
        }
      }
    if (!rotated) converged = 1;
  }

  /* eigenvalues = diagonal; stable sort descending (ties keep index order) */
  int* idx = (int*)malloc(sizeof(int) * (size_t)J);
  for (int i = 0; i < J; ++i) idx[i] = i;
  for (int i = 1; i < J; ++i) {
    int v = idx[i], k = i - 1;
    const double dv = A[(size_t)v * J + v];
    while (k >= 0 && A[(size_t)idx[k] * J + idx[k]] < dv) {
      idx[k + 1] = idx[k];
      --k;
    }
    idx[k + 1] = v;
  }
  double* W = (double*)malloc(sizeof(double) * JJ);
  for (int i = 0; i < J; ++i) {
    lam[i] = A[(size_t)idx[i] * J + idx[i]];
    memcpy(W + (size_t)i * J, V + (size_t)idx[i] * J, sizeof(double) * (size_t)J);
  }
  memcpy(V, W, sizeof(double) * JJ);
  free(W);
  free(idx);
  free(A);
  return converged ? sweeps : -1;
}

int oracle_truncate(const double* lam, int J, double thr, double* disc) {
  /* paper eq. Un: discard the trailing eigenvalues whose sum is <= thr.
   * Negative round-off eigenvalues are clamped to 0; the tail sums are
   * accumulated from the smallest value upward; R = J always qualifies
   * (empty tail), and R is at least 1. */
  if (J < 1 || !lam) return -1;
  double* tail = (double*)malloc(sizeof(double) * (size_t)(J + 1));
  tail[J] = 0.0;
  for (int i = J - 1; i >= 0; --i) tail[i] = tail[i + 1] + (lam[i] > 0.0 ? lam[i] : 0.0);
  int R = J;
  for (int r = 1; r <= J; ++r)
    if (tail[r] <= thr) {
      R = r;
      break;
    }
  if (disc) *disc = tail[R];
  free(tail);
  return R;
}

void oracle_sign_fix(double* U, int64_t I, int64_t R) {
  for (int64_t r = 0; r < R; ++r) {
    double* u = U + r * I;
    int64_t best = 0;
    for (int64_t i = 1; i < I; ++i)
      if (fabs(u[i]) > fabs(u[best])) best = i;
    if (u[best] < 0.0)
      for (int64_t i = 0; i < I; ++i) u[i] = -u[i];
  }
}

int oracle_ttm(const double* Y, const int64_t* dims, int N, int n, const double* M,
               int64_t K, int64_t msk, int64_t msj, double* Z, int nthreads) {
  /* paper Sec. 2.2.3 / Alg. 3: Z_(n) = M Y_(n), block by block:
   * Z[l + L*k + L*K*r] = sum_j M(k,j) * Y[l + L*j + L*J*r], j increasing. */
  if (check_shape(dims, N, n) || K < 1 || !Y || !M || !Z) return -1;
  int64_t L, Rt;
  left_right(dims, N, n, &L, &Rt);
  const int64_t J = dims[n];
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for collapse(2) schedule(static)
#endif
  for (int64_t r = 0; r < Rt; ++r)
    for (int64_t k = 0; k < K; ++k)
      for (int64_t l = 0; l < L; ++l) {
        double s = 0.0;
        for (int64_t j = 0; j < J; ++j) s += M[k * msk + j * msj] * Y[l + L * j + L * J * r];
        Z[l + L * k + L * K * r] = s;
      }
  return 0;
}

int oracle_slice_stats(const double* Y, const int64_t* dims, int N, int n, double* stats) {
  /* paper Sec. 3.5: statistics of every hyperslice of mode n.  Slice i holds
   * the elements Y[l + L*i + L*J*r] (l < L, r < Rt).  Two plain passes: the
   * sum, extremes and norms first, then the squared deviations from the
   * mean.  The standard deviation divides by the element count. */
  if (check_shape(dims, N, n) || !Y || !stats) return -1;
  int64_t L, Rt;
  left_right(dims, N, n, &L, &Rt);
  const int64_t J = dims[n];
  const double cnt = (double)(L * Rt);
  for (int64_t i = 0; i < J; ++i) {
    double sum = 0.0, mn = INFINITY, mx = -INFINITY, n1 = 0.0, n2 = 0.0;
    for (int64_t r = 0; r < Rt; ++r)
      for (int64_t l = 0; l < L; ++l) {
        const double v = Y[l + L * i + L * J * r];
        sum += v;
        if (v < mn) mn = v;
        if (v > mx) mx = v;
        n1 += fabs(v);
        n2 += v * v;
      }
    const double mean = sum / cnt;
    double m2 = 0.0;
    for (int64_t r = 0; r < Rt; ++r)
      for (int64_t l = 0; l < L; ++l) {
        const double d = Y[l + L * i + L * J * r] - mean;
        m2 += d * d;
      }
    stats[0 * J + i] = mean;
    stats[1 * J + i] = sqrt(m2 / cnt);
    stats[2 * J + i] = mn;
    stats[3 * J + i] = mx;
    stats[4 * J + i] = n1;
    stats[5 * J + i] = sqrt(n2);
  }
  return 0;
}

int oracle_slice_transform(const double* Y, const int64_t* dims, int N, int n, const double* shift,
                           const double* scale, int inverse, double* Z) {
  /* paper Sec. 3.5: one affine map per hyperslice of mode n.  Forward:
   * Z = (Y - shift_i) / scale_i; inverse: Z = Y * scale_i + shift_i with a
   * single rounding (fused multiply-add). */
  if (check_shape(dims, N, n) || !Y || !Z || !shift || !scale) return -1;
  int64_t L, Rt;
  left_right(dims, N, n, &L, &Rt);
  const int64_t J = dims[n];
  for (int64_t r = 0; r < Rt; ++r)
    for (int64_t i = 0; i < J; ++i)
      for (int64_t l = 0; l < L; ++l) {
        const int64_t e = l + L * i + L * J * r;
        Z[e] = inverse ? fma(Y[e], scale[i], shift[i]) : (Y[e] - shift[i]) / scale[i];
      }
  return 0;
}

double oracle_tail(const double* lam, int J, int R) {
  /* sum of the clamped eigenvalues lam[R..J) (0-based), accumulated from the
   * smallest upward, as in oracle_truncate: the energy a rank-R truncation
   * of the mode discards (paper Corollary 1). */
  double t = 0.0;
  for (int i = J - 1; i >= R; --i) t += (lam[i] > 0.0 ? lam[i] : 0.0);
  return t;
}
