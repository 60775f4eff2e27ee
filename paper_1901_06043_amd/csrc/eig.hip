// FP64 symmetric eigensolver with the truncation rule of ST-HOSVD
// (paper Alg. 1: eigenvalues in descending order; R_n = smallest R whose
// discarded eigenvalues sum to at most eps^2 ||X||^2 / N, eq. Un; only the
// leading R_n eigenvectors are formed).
//
// The paper calls LAPACK syev on the CPU (Sec. 5.2) and notes that computing
// all eigenvalues first and then only the leading eigenvectors is cheaper.
// This GPU version does exactly that, with published methods:
//  1. Householder reduction to tridiagonal form T = Q^T S Q (one workgroup;
//     p = tau A v, w = p - (tau/2)(p.v) v, A <- A - v w^T - w v^T per step).
//  2. All eigenvalues of T by Sturm-count bisection, here multisection: the P
//     lanes of a group test P interior points at once (one group per eigenvalue).
//  3. Truncation: tail sums of the clamped eigenvalues from the smallest upward.
//  4. Leading R eigenvectors of T by inverse iteration (tridiagonal LU with
//     partial pivoting), one thread per vector; eigenvalues closer than
//     1e-10 ||T|| are handled as one cluster by one thread with Gram-Schmidt
//     inside the iteration.
//  5. Re-orthogonalisation (classical Gram-Schmidt, twice) of each vector
//     against the preceding ones whose eigenvalue lies within 1e-2 ||T||;
//     beyond that gap inverse iteration already yields orthogonality at the
//     level of rounding.
//  6. Back-transformation V = Q Z, one wave per vector, followed by the sign
//     convention (largest-magnitude entry positive, lowest index on ties).
#include <cfloat>

#include "common.hpp"
#include "kernels.hpp"

namespace tk {

namespace {

constexpr int kEigThreads = 1024;

// Block-wide fixed-order sum for 1024 threads (16 waves); all threads get it.
__device__ __forceinline__ double block_sum_1024(double v, double* sred) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < 16; ++w) s += sred[w];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double block_max_1024(double v, double* sred) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double s = sred[0];
#pragma unroll
  for (int w = 1; w < 16; ++w) s = fmax(s, sred[w]);
  __syncthreads();
  return s;
}

__device__ __forceinline__ double block_min_1024(double v, double* sred) {
  return -block_max_1024(-v, sred);
}

// ---------------------------------------------------------------- 1. tridiagonalisation
// A: J x J symmetric (row-major == column-major), overwritten.  On exit row k
// holds the Householder vector v_k in positions k+2..J-1 (v_k has an implicit
// 1 at position k+1); d, e, tau receive the tridiagonal and the reflector scalars.
__global__ __launch_bounds__(kEigThreads) void eig_tridiag_kernel(double* __restrict__ A, int J,
                                                                  double* __restrict__ d, double* __restrict__ e,
                                                                  double* __restrict__ tau) {
  extern __shared__ double sh[];
  double* sv = sh;          // J
  double* sp = sh + J;      // J
  double* sred = sh + 2 * J;  // 16
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int k = 0; k + 2 < J; ++k) {
    const int m = J - k - 1;
    const double* rowk = A + (int64_t)k * J + (k + 1);
    double part = 0.0;
    for (int i = tid; i < m; i += kEigThreads) {
      const double x = rowk[i];
      sv[i] = x;
      if (i >= 1) part += x * x;
    }
    const double sigma = block_sum_1024(part, sred);
    const double alpha = sv[0];
    double beta, tk;
    if (sigma == 0.0) {
      tk = 0.0;
      beta = alpha;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
      tk = (beta - alpha) / beta;
    }
    if (tid == 0) {
      d[k] = A[(int64_t)k * J + k];
      e[k] = beta;
      tau[k] = tk;
    }
    __syncthreads();
    if (tk == 0.0) continue;
    const double scale = 1.0 / (alpha - beta);
    for (int i = tid; i < m; i += kEigThreads) {
      const double v = (i == 0) ? 1.0 : sv[i] * scale;
      sv[i] = v;
      if (i >= 1) A[(int64_t)k * J + k + 1 + i] = v;
    }
    __syncthreads();
    // p = tau * A22 v
    for (int i = wave; i < m; i += 16) {
      const double* row = A + (int64_t)(k + 1 + i) * J + (k + 1);
      double s = 0.0;
      for (int j = lane; j < m; j += 64) s += row[j] * sv[j];
      s = wave_sum(s);
      if (lane == 0) sp[i] = tk * s;
    }
    __syncthreads();
    double pv = 0.0;
    for (int i = tid; i < m; i += kEigThreads) pv += sp[i] * sv[i];
    pv = block_sum_1024(pv, sred);
    const double cc = 0.5 * tk * pv;
    for (int i = tid; i < m; i += kEigThreads) sp[i] -= cc * sv[i];
    __syncthreads();
    // A22 <- A22 - v w^T - w v^T
    for (int i = wave; i < m; i += 16) {
      double* row = A + (int64_t)(k + 1 + i) * J + (k + 1);
      const double vi = sv[i], wi = sp[i];
      for (int j = lane; j < m; j += 64) row[j] -= vi * sp[j] + wi * sv[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (J >= 2) {
      d[J - 2] = A[(int64_t)(J - 2) * J + (J - 2)];
      e[J - 2] = A[(int64_t)(J - 2) * J + (J - 1)];
      d[J - 1] = A[(int64_t)(J - 1) * J + (J - 1)];
    } else {
      d[0] = A[0];
    }
  }
}

// ---------------------------------------------------------------- 2-3. eigenvalues + truncation
// scal[0] <- ||T|| (Gershgorin bound), scal[1] <- pivmin.
// The truncation threshold is thr, or thr * (*nx2) when nx2 is non-null (so
// that eps^2 ||X||^2 / N can be formed on the device without a host round trip).
__global__ __launch_bounds__(kEigThreads) void eig_bisect_kernel(const double* __restrict__ d,
                                                                 const double* __restrict__ e, int J, double thr,
                                                                 const double* __restrict__ nx2,
                                                                 double* __restrict__ lam, int64_t* __restrict__ Rout,
                                                                 double* __restrict__ disc, double* __restrict__ scal) {
  extern __shared__ double sh[];
  double* sd = sh;          // J
  double* se2 = sh + J;     // J
  double* sred = sh + 2 * J;  // 16
  const int tid = threadIdx.x, lane = tid & 63;
  double glo = DBL_MAX, ghi = -DBL_MAX, e2max = 0.0;
  for (int i = tid; i < J; i += kEigThreads) {
    const double di = d[i];
    const double em = (i > 0) ? fabs(e[i - 1]) : 0.0;
    const double ep = (i + 1 < J) ? fabs(e[i]) : 0.0;
    sd[i] = di;
    se2[i] = (i + 1 < J) ? e[i] * e[i] : 0.0;
    e2max = fmax(e2max, se2[i]);
    glo = fmin(glo, di - em - ep);
    ghi = fmax(ghi, di + em + ep);
  }
  glo = block_min_1024(glo, sred);
  ghi = block_max_1024(ghi, sred);
  e2max = block_max_1024(e2max, sred);
  const double pivmin = DBL_MIN * fmax(1.0, e2max);
  const double tnorm = fmax(fabs(glo), fabs(ghi));
  const double widen = 2.1 * DBL_EPSILON * tnorm * J + 4.2 * pivmin;
  glo -= widen;
  ghi += widen;
  const double atol = 2.0 * DBL_EPSILON * tnorm + 4.0 * pivmin;

  // group size P: power of two, P * J <= 1024, P <= 32
  int P = 1;
  while (P < 32 && 2 * P * J <= kEigThreads) P *= 2;
  const int G = kEigThreads / P;
  const int q = tid % P, gbase = (lane / P) * P;
  const uint64_t gmask = (P == 64) ? ~0ull : ((1ull << P) - 1ull);
  for (int a = tid / P; a < J; a += G) {
    double lo = glo, hi = ghi;
    for (int it = 0; it < 128 && (hi - lo) > atol; ++it) {
      const double h = (hi - lo) / (P + 1);
      const double sig = lo + h * (q + 1);
      // Sturm count: number of eigenvalues < sig
      int cnt = 0;
      double qq = sd[0] - sig;
      if (fabs(qq) < pivmin) qq = -pivmin;
      cnt += (qq < 0.0);
      for (int i = 1; i < J; ++i) {
        qq = (sd[i] - sig) - se2[i - 1] / qq;
        if (fabs(qq) < pivmin) qq = -pivmin;
        cnt += (qq < 0.0);
      }
      const uint64_t bal = __ballot(cnt > a);
      const uint64_t m = (bal >> gbase) & gmask;
      const int f = m ? (__ffsll((long long)m) - 1) : P;
      const double nlo = (f == 0) ? lo : lo + h * f;
      const double nhi = (f == P) ? hi : lo + h * (f + 1);
      lo = nlo;
      hi = nhi;
    }
    if (q == 0) lam[J - 1 - a] = 0.5 * (lo + hi);
  }
  __syncthreads();
  if (tid == 0) {
    scal[0] = tnorm;
    scal[1] = pivmin;
    if (nx2 != nullptr) thr *= *nx2;
    // smallest R in 1..J with sum_{i>=R} max(lam_i, 0) <= thr (lam descending)
    double tail = 0.0, tailR = 0.0;
    int R = J;
    for (int r = J - 1; r >= 1; --r) {
      tail += fmax(lam[r], 0.0);
      if (tail <= thr) {
        R = r;
        tailR = tail;
      } else {
        break;
      }
    }
    *Rout = R;
    *disc = tailR;
  }
}

// ---------------------------------------------------------------- 4. inverse iteration
__device__ __forceinline__ double hash_unit(uint32_t a, uint32_t b) {
  uint32_t x = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return (double)x * (2.0 / 4294967296.0) - 1.0;
}

// work layout: array a (0..5), element i, thread slot t  ->  work[(a*J + i)*ld + t]
__global__ __launch_bounds__(64) void eig_invit_kernel(const double* __restrict__ d, const double* __restrict__ e, int J,
                                                       const double* __restrict__ lam, const int64_t* __restrict__ Rp,
                                                       const double* __restrict__ scal, double* __restrict__ Zt,
                                                       double* __restrict__ work, int ld) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  const int R = (int)*Rp;
  if (t >= R) return;
  const double tnorm = scal[0];
  const double ctol = 1e-10 * tnorm;
  if (t > 0 && lam[t - 1] - lam[t] <= ctol) return;  // handled by its cluster leader
  if (tnorm == 0.0) {
    // zero matrix: unit vectors
    for (int vec = t; vec < R && (vec == t || lam[vec - 1] - lam[vec] <= ctol); ++vec)
      for (int i = 0; i < J; ++i) Zt[(int64_t)vec * J + i] = (i == vec) ? 1.0 : 0.0;
    return;
  }
  const double inv = 1.0 / tnorm;
  const double eps = DBL_EPSILON;
  double* dl = work + (int64_t)0 * J * ld + t;
  double* dd = work + (int64_t)1 * J * ld + t;
  double* du = work + (int64_t)2 * J * ld + t;
  double* du2 = work + (int64_t)3 * J * ld + t;
  double* pv = work + (int64_t)4 * J * ld + t;
  double* x = work + (int64_t)5 * J * ld + t;
#define W(arr, i) arr[(int64_t)(i) * ld]
  double prev_shift = 0.0;
  for (int vec = t; vec < R; ++vec) {
    if (vec > t && !(lam[vec - 1] - lam[vec] <= ctol)) break;
    double shift = lam[vec] * inv;
    if (vec > t && prev_shift - shift < 10.0 * eps) shift = prev_shift - 10.0 * eps;
    prev_shift = shift;
    // LU with partial pivoting of (T - lambda I) / ||T||
    for (int i = 0; i < J; ++i) {
      W(dd, i) = d[i] * inv - shift;
      W(dl, i) = (i + 1 < J) ? e[i] * inv : 0.0;
      W(du, i) = (i + 1 < J) ? e[i] * inv : 0.0;
      W(du2, i) = 0.0;
    }
    for (int i = 0; i + 1 < J; ++i) {
      const double di = W(dd, i), li = W(dl, i);
      if (fabs(di) >= fabs(li)) {
        W(pv, i) = 0.0;
        const double f = (di != 0.0) ? li / di : 0.0;
        W(dl, i) = f;
        W(dd, i + 1) = W(dd, i + 1) - f * W(du, i);
      } else {
        W(pv, i) = 1.0;
        const double f = di / li;
        const double ddn = W(dd, i + 1), dui = W(du, i);
        W(dd, i) = li;
        W(dl, i) = f;
        W(du, i) = ddn;
        W(dd, i + 1) = dui - f * ddn;
        if (i + 2 < J) {
          const double dun = W(du, i + 1);
          W(du2, i) = dun;
          W(du, i + 1) = -f * dun;
        }
      }
    }
    for (int i = 0; i < J; ++i)
      if (fabs(W(dd, i)) < eps) W(dd, i) = (W(dd, i) < 0.0) ? -eps : eps;
    // start vector
    double nrm = 0.0;
    for (int i = 0; i < J; ++i) {
      const double v = hash_unit((uint32_t)i, (uint32_t)vec);
      W(x, i) = v;
      nrm += v * v;
    }
    for (int it = 0; it < 3; ++it) {
      // forward: row interchanges and multipliers
      for (int i = 0; i + 1 < J; ++i) {
        if (W(pv, i) != 0.0) {
          const double tmp = W(x, i);
          W(x, i) = W(x, i + 1);
          W(x, i + 1) = tmp;
        }
        W(x, i + 1) = W(x, i + 1) - W(dl, i) * W(x, i);
      }
      // backward substitution with U (diag dd, superdiagonals du, du2)
      double y1 = 0.0, y2 = 0.0;
      for (int i = J - 1; i >= 0; --i) {
        double s = W(x, i);
        if (i + 1 < J) s -= W(du, i) * y1;
        if (i + 2 < J) s -= W(du2, i) * y2;
        const double yi = s / W(dd, i);
        W(x, i) = yi;
        y2 = y1;
        y1 = yi;
      }
      // Gram-Schmidt against the finished members of this cluster
      for (int j = t; j < vec; ++j) {
        const double* zj = Zt + (int64_t)j * J;
        double h = 0.0;
        for (int i = 0; i < J; ++i) h += zj[i] * W(x, i);
        for (int i = 0; i < J; ++i) W(x, i) = W(x, i) - h * zj[i];
      }
      nrm = 0.0;
      double amax = 0.0;
      for (int i = 0; i < J; ++i) amax = fmax(amax, fabs(W(x, i)));
      const double sc = (amax > 0.0) ? 1.0 / amax : 1.0;
      for (int i = 0; i < J; ++i) {
        const double v = W(x, i) * sc;
        W(x, i) = v;
        nrm += v * v;
      }
      const double rn = 1.0 / sqrt(nrm);
      for (int i = 0; i < J; ++i) W(x, i) = W(x, i) * rn;
    }
    for (int i = 0; i < J; ++i) Zt[(int64_t)vec * J + i] = W(x, i);
  }
#undef W
}

// ---------------------------------------------------------------- 5. re-orthogonalisation
__global__ __launch_bounds__(kEigThreads) void eig_orth_kernel(double* __restrict__ Zt, int J,
                                                               const double* __restrict__ lam,
                                                               const int64_t* __restrict__ Rp,
                                                               const double* __restrict__ scal) {
  extern __shared__ double sh[];
  double* hs = sh;           // J
  double* sred = sh + J;     // 16
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R = (int)*Rp;
  const double otol = 1e-2 * scal[0];
  int jlo = 0;
  for (int i = 1; i < R; ++i) {
    while (jlo < i && lam[jlo] - lam[i] >= otol) ++jlo;
    if (jlo == i) continue;  // uniform
    double* zi = Zt + (int64_t)i * J;
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = jlo + wave; j < i; j += 16) {
        const double* zj = Zt + (int64_t)j * J;
        double h = 0.0;
        for (int r = lane; r < J; r += 64) h += zj[r] * zi[r];
        h = wave_sum(h);
        if (lane == 0) hs[j - jlo] = h;
      }
      __syncthreads();
      for (int r = tid; r < J; r += kEigThreads) {
        double v = zi[r];
        for (int j = jlo; j < i; ++j) v -= hs[j - jlo] * Zt[(int64_t)j * J + r];
        zi[r] = v;
      }
      __syncthreads();
    }
    double nn = 0.0;
    for (int r = tid; r < J; r += kEigThreads) nn += zi[r] * zi[r];
    nn = block_sum_1024(nn, sred);
    const double rn = 1.0 / sqrt(nn);
    for (int r = tid; r < J; r += kEigThreads) zi[r] *= rn;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- 6. back-transformation + signs
template <int Q>
__global__ __launch_bounds__(256) void eig_back_kernel(const double* __restrict__ A, const double* __restrict__ tau,
                                                       int J, const double* __restrict__ Zt,
                                                       const int64_t* __restrict__ Rp, double* __restrict__ U) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int vec = blockIdx.x * 4 + wave;
  if (vec >= (int)*Rp) return;
  double z[Q], v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = lane + 64 * q;
    z[q] = (r < J) ? Zt[(int64_t)vec * J + r] : 0.0;
  }
  for (int k = J - 3; k >= 0; --k) {
    const double tk = tau[k];
    if (tk == 0.0) continue;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int r = lane + 64 * q;
      const double vq = (r == k + 1) ? 1.0 : ((r > k + 1 && r < J) ? A[(int64_t)k * J + r] : 0.0);
      v[q] = vq;
      s += vq * z[q];
    }
    s = wave_sum(s) * tk;
#pragma unroll
    for (int q = 0; q < Q; ++q) z[q] -= s * v[q];
  }
  // sign convention: entry of largest magnitude (lowest index on ties) positive
  double ba = -1.0, bv = 0.0;
  int bi = J;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = lane + 64 * q;
    if (r < J && fabs(z[q]) > ba) {
      ba = fabs(z[q]);
      bv = z[q];
      bi = r;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double oa = __shfl_xor(ba, off, 64);
    const double ov = __shfl_xor(bv, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (oa > ba || (oa == ba && oi < bi)) {
      ba = oa;
      bv = ov;
      bi = oi;
    }
  }
  const double sgn = (bv < 0.0) ? -1.0 : 1.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = lane + 64 * q;
    if (r < J) U[(int64_t)vec * J + r] = sgn * z[q];
  }
}

template <int Q>
void launch_back(const EigWork& w, int J, const int64_t* R, double* U, hipStream_t s) {
  hipLaunchKernelGGL((eig_back_kernel<Q>), dim3(ceil_div(J, 4)), dim3(256), 0, s, w.A, w.tau, J, w.Zt, R, U);
}

}  // namespace

int64_t eig_work_doubles(int64_t J) { return 2 * J * J + 6 * J * J + 3 * J + 8; }

void eig_work_carve(double* base, int64_t J, EigWork& w) {
  w.A = base;
  w.Zt = w.A + J * J;
  w.work = w.Zt + J * J;
  w.d = w.work + 6 * J * J;
  w.e = w.d + J;
  w.tau = w.e + J;
  w.scal = w.tau + J;
}

hipError_t launch_eig_truncate(const double* S, int J, double thr, const double* nx2, const EigWork& w,
                               double* lam, double* U, int64_t* R, double* disc, hipStream_t stream) {
  hipError_t err = hipMemcpyAsync(w.A, S, sizeof(double) * (size_t)J * J, hipMemcpyDeviceToDevice, stream);
  if (err != hipSuccess) return err;
  const size_t sh2 = sizeof(double) * (2 * (size_t)J + 16);
  hipLaunchKernelGGL(eig_tridiag_kernel, dim3(1), dim3(kEigThreads), sh2, stream, w.A, J, w.d, w.e, w.tau);
  hipLaunchKernelGGL(eig_bisect_kernel, dim3(1), dim3(kEigThreads), sh2, stream, w.d, w.e, J, thr, nx2, lam, R,
                     disc, w.scal);
  hipLaunchKernelGGL(eig_invit_kernel, dim3(ceil_div(J, 64)), dim3(64), 0, stream, w.d, w.e, J, lam, R, w.scal,
                     w.Zt, w.work, J);
  const size_t sh1 = sizeof(double) * ((size_t)J + 16);
  hipLaunchKernelGGL(eig_orth_kernel, dim3(1), dim3(kEigThreads), sh1, stream, w.Zt, J, lam, R, w.scal);
  const int q = (int)ceil_div(J, 64);
  if (q <= 1) launch_back<1>(w, J, R, U, stream);
  else if (q <= 2) launch_back<2>(w, J, R, U, stream);
  else if (q <= 4) launch_back<4>(w, J, R, U, stream);
  else if (q <= 8) launch_back<8>(w, J, R, U, stream);
  else if (q <= 11) launch_back<11>(w, J, R, U, stream);
  else launch_back<16>(w, J, R, U, stream);
  return hipGetLastError();
}

}  // namespace tk
