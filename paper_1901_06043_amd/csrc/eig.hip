// FP64 symmetric eigensolver with the truncation rule of ST-HOSVD
// (paper Alg. 1: eigenvalues in descending order; R_n = smallest R whose
// discarded eigenvalues sum to at most eps^2 ||X||^2 / N, eq. Un; only the
// leading R_n eigenvectors are formed).
//
// The paper calls LAPACK syev on the CPU (Sec. 5.2) and notes that computing
// all eigenvalues first and then only the leading eigenvectors is cheaper.
// This GPU version does exactly that, with published methods:
//  1. Householder reduction to tridiagonal form T = Q^T S Q.  Per step:
//     p = tau A v, w = p - (tau/2)(p.v) v, A <- A - v w^T - w v^T.
//     Once the trailing matrix has at most 208 rows, one workgroup keeps it in
//     registers (each matrix row on 16 lanes of a wave), in phases of shrinking
//     register layouts; the matrix-vector products and the rank-2 updates run
//     from registers, with look-ahead (the owner of the next row publishes it
//     and its reflector scalars during the update).  The phases of at most
//     128 rows share one launch and hand the trailing block on through LDS.
//     Larger matrices first take steps of two launches each over row blocks
//     in global memory.
//  2. All eigenvalues of T by Sturm-count multisection: one workgroup per
//     eigenvalue tests 256 interior points at once; many workgroups.
//  3. Truncation: tail sums of the clamped eigenvalues from the smallest upward.
//  4. Leading R eigenvectors of T by two steps of inverse iteration
//     (tridiagonal LU with partial pivoting, factors in LDS), one thread per
//     vector, every vector from its own pseudo-random start.  For eigenvalues
//     that coincide to rounding the iterates are independent random vectors of
//     the common invariant subspace.
//  5. Re-orthogonalisation (classical Gram-Schmidt, twice) of each vector
//     against the preceding ones whose eigenvalue lies within 1e-2 ||T||;
//     this turns such iterates into an orthonormal basis of the subspace, and
//     beyond that gap inverse iteration already yields orthogonality at the
//     level of rounding.  Large clusters are processed in blocks with FP64
//     MFMA products.
//  6. Back-transformation V = Q Z, one wave per vector, followed by the sign
//     convention (largest-magnitude entry positive, lowest index on ties).
#include <cfloat>

#include "common.hpp"
#include "kernels.hpp"

namespace tk {

namespace {

constexpr int kEigThreads = 1024;

// A launch that the runtime rejects (for instance for its LDS request) is
// returned to the caller at once.
#define LAUNCH_OK()                              \
  do {                                           \
    const hipError_t launch_err_ = hipGetLastError(); \
    if (launch_err_ != hipSuccess) return launch_err_; \
  } while (0)

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

template <int NW>
__device__ __forceinline__ double block_max(double v, double* sred) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double s = sred[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) s = fmax(s, sred[w]);
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- 1a. tridiagonalisation, J <= 208
// The full symmetric matrix is held in registers.  Each row of 16 lanes of a
// wave holds one matrix row: lane l serves row slot l >> 4 and the columns
// (l & 15) + 16 c, c < NC; wave w, group g, slot s holds row 4 (NW g + w) + s.
// Every reduction (row sums, norms, dot products) is then a 16-lane DPP
// reduction, bit-identical in all lanes, and the barriers order LDS only.
// Row groups that are already reduced are skipped; reduced columns carry
// v_j = w_j = 0 and are processed without branches.
// Output: d, e, tau and, in row k of H, the Householder vector v_k at
// positions k+2..J-1 (implicit 1 at k+1).
constexpr int kRegMaxJ = 208;

// Householder scalars of a step from alpha = a_k,k+1 and sigma =
// sum_{j >= k+2} a_kj^2: beta = -sign(alpha) sqrt(alpha^2 + sigma),
// tau = (beta - alpha) / beta, scale = 1 / (alpha - beta); tau = scale = 0
// when sigma = 0.  When alpha^2 + sigma falls below kTinyNorm2 its square root
// would lose precision in the subnormal range (rows of a strongly graded
// matrix), so the caller passes the values of the row scaled by kRowScale and
// reflector() unscales beta and scale (tau is scale-free), as LAPACK's
// reflector generator does.
constexpr double kTinyNorm2 = 0x1p-900;
constexpr double kRowScale = 0x1p+600;
__device__ __forceinline__ bool row_is_tiny(double alpha, double sigma) {
  return sigma != 0.0 && alpha * alpha + sigma < kTinyNorm2;
}
__device__ __forceinline__ void reflector(double alpha, double sigma, bool scaled, double& beta, double& tk,
                                          double& scale) {
  beta = alpha;
  tk = 0.0;
  scale = 0.0;
  if (sigma != 0.0) {
    beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
    tk = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  if (scaled) {
    beta *= 1.0 / kRowScale;
    scale *= kRowScale;
  }
}

// Sum of (kRowScale x_j)^2 over this lane's columns j >= kk + 2 of the row x in LDS.
template <int NC>
__device__ __forceinline__ double scaled_tail(const double* x, int c, int kk, int J) {
  double part = 0.0;
#pragma unroll
  for (int cc = 0; cc < NC; ++cc) {
    const int j = c + 16 * cc;
    const double y = x[j] * kRowScale;
    part += (j >= kk + 2 && j < J) ? y * y : 0.0;
  }
  return part;
}

// Row kk of the matrix becomes the column of step kk: its owner wave writes
// it to LDS and computes that step's reflector scalars from the values in its
// registers (sigma = sum_{j >= kk+2} a_kk,j^2, alpha = a_kk,kk+1,
// beta = -sign(alpha) sqrt(alpha^2 + sigma), tau = (beta - alpha) / beta,
// scale = 1 / (alpha - beta)), published in ssn[0..2].  Called by every wave;
// only the owner acts.
template <int NW, int NG, int NC>
__device__ __forceinline__ void publish_row(int kk, int J, int wave, int rs, int c, const double (&a)[NG][NC],
                                            double* sxn, double* ssn) {
  const int blk = kk >> 2;
  if (wave != blk % NW) return;  // uniform
  const int gk = blk / NW;
  const bool mine = (rs == (kk & 3));
  double part = 0.0;
#pragma unroll
  for (int g = 0; g < NG; ++g)
    if (g == gk) {
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const int j = c + 16 * cc;
        const double x = a[g][cc];
        if (mine) sxn[j] = x;
        part += (j >= kk + 2 && j < J) ? x * x : 0.0;
      }
    }
  double sigma = row16_sum(part);  // the owner slot's 16 lanes hold row kk
  if (kk + 1 >= J) return;
  double alpha = sxn[kk + 1];  // written above by this wave (LDS operations of a wave are ordered)
  const bool tiny = row_is_tiny(alpha, sigma);  // uniform within each 16-lane row
  if (tiny) sigma = row16_sum(scaled_tail<NC>(sxn, c, kk, J)), alpha *= kRowScale;
  double beta, tk, scale;
  reflector(alpha, sigma, tiny, beta, tk, scale);
  if (mine && c == 0) {
    ssn[0] = beta;
    ssn[1] = tk;
    ssn[2] = scale;
  }
}

// Phase of the reduction: the J x J block at S (leading dimension lds) is
// reduced for at most `nsteps` steps; if rows remain, the trailing block
// (rows and columns >= nsteps) is written to Aout (leading dimension lda,
// indices relative to that block) for the next, smaller, phase, which may
// read it in place.  d, e, tau and H (leading dimension ldh) start at the
// block's first row.  Waves numbered NW and above hold no rows: they only
// take part in the barriers.
// Look-ahead: during the update of step k the wave owning row k + 1 (in its
// first live group) writes that row to LDS as soon as it is updated and
// computes the scalars of step k + 1 from its registers, so a step starts
// from LDS values instead of a reduction, square root and divisions on every
// wave.  Columns and scalars are double-buffered by the parity of k: one
// barrier after the matrix-vector product and one at the end of each step.
template <int NW, int NG, int NC>
__device__ __forceinline__ void tridiag_reg_body(const double* S, int lds, int J, int nsteps, double* Aout, int lda,
                                                 double* __restrict__ H, int ldh, double* __restrict__ d,
                                                 double* __restrict__ e, double* __restrict__ tau) {
  __shared__ double sxb[2][16 * NC];  // column k of the current matrix (by parity of k)
  __shared__ double ssc[2][4];        // beta, tau, scale of step k (by parity of k)
  __shared__ double sp[16 * NC];      // p = tau A v
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane & 15, rs = lane >> 4;
  if (wave >= NW) {  // uniform: one barrier after the first row, two per step
    lds_barrier();
    for (int k = 0; k + 2 < J && k < nsteps; ++k) {
      lds_barrier();
      lds_barrier();
    }
    return;
  }

  double a[NG][NC];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      const int i = 4 * (NW * g + wave) + rs, j = c + 16 * cc;
      a[g][cc] = (i < J && j < J) ? S[(int64_t)i * lds + j] : 0.0;
    }
  for (int j = tid; j < 16 * NC; j += 64 * NW) sp[j] = 0.0;
  publish_row<NW, NG, NC>(0, J, wave, rs, c, a, sxb[0], ssc[0]);
  lds_barrier();

  int k = 0;
  for (; k + 2 < J && k < nsteps; ++k) {
    const double* sx = sxb[k & 1];
    double* sxn = sxb[(k + 1) & 1];
    double* ssn = ssc[(k + 1) & 1];
    const double beta = ssc[k & 1][0], tk = ssc[k & 1][1], scale = ssc[k & 1][2];
    if (tid == 0) {
      d[k] = sx[k];
      e[k] = beta;
      tau[k] = tk;
    }
    if (wave == 0)
      for (int j = k + 2 + lane; j < J; j += 64) H[(int64_t)k * ldh + j] = sx[j] * scale;
    // (tau = 0 needs no special case: p, w and the update vanish).  LDS reads
    // are unconditional (then selected) so that they are issued together.
    double vj[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      const int j = c + 16 * cc;
      const double x = sx[j];
      vj[cc] = (j <= k || j >= J) ? 0.0 : (j == k + 1 ? 1.0 : x * scale);
    }
    // p_i = tau * sum_j a_ij v_j
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int i = 4 * (NW * g + wave) + rs;
      if (4 * (NW * g + wave) + 3 <= k) {  // whole group reduced (uniform): p = 0 there
        if (c == 0 && i < J) sp[i] = 0.0;
        continue;
      }
      // columns <= k have v_j = 0 and contribute nothing
      double t = 0.0;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) t += a[g][cc] * vj[cc];
      t = row16_sum(t);
      if (c == 0 && i < J) sp[i] = (i > k) ? tk * t : 0.0;
    }
    lds_barrier();
    double pv = 0.0;
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) pv += sp[c + 16 * cc] * vj[cc];
    pv = row16_sum(pv);
    const double c2 = 0.5 * tk * pv;
    // A <- A - v w^T - w v^T on the live rows and column slots, w = p - c2 v.
    // The owner of row k + 1 (whose first live group holds it) writes that row
    // to LDS as soon as it is updated and sums the squares of its tail.
    const int kn = k + 1, blkn = kn >> 2;
    const int gkn = (wave == blkn % NW) ? blkn / NW : -1;  // uniform
    const bool slot = (rs == (kn & 3));
    double part = 0.0;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      if (4 * (NW * g + wave) + 3 <= k) continue;  // uniform
      const int i = 4 * (NW * g + wave) + rs;
      const int ic = min(i, 16 * NC - 1);  // rows beyond the columns are padding
      const double sxi = sx[ic], spi = sp[ic];
      const double vi = (i <= k || i >= J) ? 0.0 : (i == k + 1 ? 1.0 : sxi * scale);
      const double wi = (i < J) ? spi - c2 * vi : 0.0;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const double wj = sp[c + 16 * cc] - c2 * vj[cc];  // w_j; zero for reduced columns
        a[g][cc] = fma(-vi, wj, fma(-wi, vj[cc], a[g][cc]));
      }
      if (g == gkn) {
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
          const int j = c + 16 * cc;
          if (slot) sxn[j] = a[g][cc];
          part += (j >= kn + 2 && j < J) ? a[g][cc] * a[g][cc] : 0.0;
        }
      }
    }
    if (gkn >= 0 && kn + 1 < J) {
      // scalars of step k + 1 from the owner slot's 16 lanes
      double sigma = row16_sum(part);
      double alpha = sxn[kn + 1];  // written above by this wave (LDS operations of a wave are ordered)
      const bool tiny = row_is_tiny(alpha, sigma);  // uniform within each 16-lane row
      if (tiny) sigma = row16_sum(scaled_tail<NC>(sxn, c, kn, J)), alpha *= kRowScale;
      double nbeta, ntk, nscale;
      reflector(alpha, sigma, tiny, nbeta, ntk, nscale);
      if (slot && c == 0) {
        ssn[0] = nbeta;
        ssn[1] = ntk;
        ssn[2] = nscale;
      }
    }
    lds_barrier();
  }
  const double* sx = sxb[k & 1];
  if (k + 2 < J) {
    // stopped early: hand the trailing block (rows and columns >= k) to the next phase
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int i = 4 * (NW * g + wave) + rs;
      if (i < k || i >= J) continue;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const int j = c + 16 * cc;
        if (j >= k && j < J) Aout[(int64_t)(i - k) * lda + (j - k)] = a[g][cc];
      }
    }
    return;
  }
  if (J >= 2) {
    if (tid == 0) {
      d[J - 2] = sx[J - 2];
      e[J - 2] = sx[J - 1];
    }
    const int kl = J - 1, blk = kl >> 2;
    if (wave == blk % NW && rs == (kl & 3) && c == (kl & 15)) {
      const int gk = blk / NW, ck = kl >> 4;
#pragma unroll
      for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int cc = 0; cc < NC; ++cc)
          if (g == gk && cc == ck) d[kl] = a[g][cc];
    }
  } else if (tid == 0) {
    d[0] = sx[0];
  }
}

// One phase on the trailing block of S (leading dimension ld) that starts at
// row and column k0; the block left after `nsteps` steps goes to A (same
// global indices).
template <int NW, int NG, int NC>
__global__ __launch_bounds__(64 * NW) void eig_tridiag_reg_kernel(const double* S, int ld, int k0, int J, int nsteps,
                                                                  double* A, double* __restrict__ H,
                                                                  double* __restrict__ d, double* __restrict__ e,
                                                                  double* __restrict__ tau) {
  const int kt = min(k0 + nsteps, ld - 1);  // origin of the block handed on (only written if rows remain)
  tridiag_reg_body<NW, NG, NC>(S + (int64_t)k0 * ld + k0, ld, J, nsteps, A + (int64_t)kt * ld + kt, ld,
                               H + (int64_t)k0 * ld + k0, ld, d + k0, e + k0, tau + k0);
}

// The phases of at most 128 rows in one workgroup of 16 waves: each phase
// hands its trailing block to the next through LDS (kTailHand doubles,
// dynamic) instead of global memory and a new launch.  Phases with fewer
// waves leave the others to wait at the barriers.
constexpr int kTailRows = 128;
constexpr int kTailHand = 96 * 96;
__global__ __launch_bounds__(1024) void eig_tridiag_tail_kernel(const double* S, int ld, int k0, int J,
                                                                double* __restrict__ H, double* __restrict__ d,
                                                                double* __restrict__ e, double* __restrict__ tau) {
  extern __shared__ double hand[];
  const double* src = S + (int64_t)k0 * ld + k0;
  int lsrc = ld, Jl = J - k0;
  H += (int64_t)k0 * ld + k0;
  d += k0;
  e += k0;
  tau += k0;
  // one phase that stops when `next` rows are left, handing them on through LDS
#define TAIL_PHASE(NW, NG, NC, next)                                                            \
  if (Jl > (next)) {                                                                            \
    const int ns = Jl - (next);                                                                 \
    tridiag_reg_body<NW, NG, NC>(src, lsrc, Jl, ns, hand, (next), H, ld, d, e, tau);            \
    __syncthreads();                                                                            \
    src = hand;                                                                                 \
    lsrc = (next);                                                                              \
    Jl = (next);                                                                                \
    H += (int64_t)ns * ld + ns;                                                                 \
    d += ns;                                                                                    \
    e += ns;                                                                                    \
    tau += ns;                                                                                  \
  }
  TAIL_PHASE(16, 2, 8, 96)
  TAIL_PHASE(16, 2, 6, 64)
  TAIL_PHASE(16, 1, 4, 32)
#undef TAIL_PHASE
  tridiag_reg_body<8, 1, 2>(src, lsrc, Jl, Jl, hand, 32, H, ld, d, e, tau);
}

// ---------------------------------------------------------------- 1b. tridiagonalisation steps, J > 208
// While the trailing matrix is larger than the register-resident form holds,
// each Householder step is a launch over blocks of kBigRows matrix rows
// (A: J x J in global memory, global indices).  A step needs two passes that
// depend on every row: p = tau A v (which needs v from the updated row k) and
// the rank-2 update A <- A - v w^T - w v^T with w = p - (tau/2)(p.v) v (which
// needs all of p).  eig_tri_big_step runs the update of step k - 1 and the
// product of step k in one pass; eig_tri_big_update applies the last step's
// update (every workgroup forms w in the same fixed order) and stores v_k in
// row k, the form the back-transformation reads.
constexpr int kBigRows = 16;
constexpr int kBigThreads = 256;

// Fixed-order sum over a workgroup of 256 threads; every thread gets it.
__device__ __forceinline__ double block_sum_256(double v, double* sred) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum_fast(v);
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  const double s = (sred[0] + sred[1]) + (sred[2] + sred[3]);
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(kBigThreads) void eig_tri_big_update(double* __restrict__ A, int J, int k,
                                                                  const double* __restrict__ V,
                                                                  const double* __restrict__ P,
                                                                  const double* __restrict__ sc,
                                                                  double* __restrict__ d, double* __restrict__ e,
                                                                  double* __restrict__ tau) {
  extern __shared__ double sh[];
  double* sv = sh;      // J
  double* sw = sh + J;  // J
  __shared__ double sred[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double tk = sc[1];
  double part = 0.0;
  for (int j = k + 1 + tid; j < J; j += kBigThreads) {
    const double v = V[j], pj = P[j];
    sv[j] = v;
    sw[j] = pj;
    part += pj * v;
  }
  const double c2 = 0.5 * tk * block_sum_256(part, sred);  // (the sum's barriers publish sv, sw)
  for (int j = k + 1 + tid; j < J; j += kBigThreads) sw[j] -= c2 * sv[j];
  __syncthreads();
  const int r0 = k + 1 + (int)blockIdx.x * kBigRows, r1 = min(r0 + kBigRows, J);
  for (int i = r0 + wave; i < r1; i += kBigThreads / 64) {
    double* row = A + (int64_t)i * J;
    const double vi = sv[i], wi = sw[i];
    for (int j = k + 1 + lane; j < J; j += 64) row[j] -= vi * sw[j] + wi * sv[j];
  }
  if (blockIdx.x == 0) {
    if (tid == 0 && d != nullptr) {  // null after eig_tri_big_step, which wrote them
      d[k] = A[(int64_t)k * J + k];
      e[k] = sc[0];
      tau[k] = tk;
    }
    for (int j = k + 2 + tid; j < J; j += kBigThreads) A[(int64_t)k * J + j] = sv[j];
  }
}

// The same steps with one launch each: launch k first applies the rank-2
// update of step k - 1 (v, p and tau of that step, from the previous launch)
// to the rows it owns, and forms row k as updated by every workgroup for
// itself (a fixed-order computation, the same in each), so that the update
// and the next reflector's matrix-vector product share one pass over the
// rows.  Row k is read in launch k and written by no one then; workgroup 0
// stores v_{k-1} into row k - 1 (which no launch reads again) and writes
// d_k, e_k and tau_k.  V, P and the scalars alternate between two buffers.
// After the last step, eig_tri_big_update (without d) applies its update.
// Fixed-order sum over a workgroup of NW waves; every thread gets it.
template <int NW>
__device__ __forceinline__ double block_sum_nw(double v, double* sred) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum_fast(v);
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += sred[w];
  __syncthreads();
  return s;
}

// NW waves, one matrix row each; RR = row entries per lane (J <= 64 RR), all
// loaded before the step's reductions so that their latency overlaps them.
template <int RR, int NW>
__global__ __launch_bounds__(64 * NW) void eig_tri_big_step(double* __restrict__ A, int J, int k,
                                                            const double* __restrict__ Vp,
                                                            const double* __restrict__ Pp,
                                                            const double* __restrict__ scp,
                                                            double* __restrict__ Vc, double* __restrict__ Pc,
                                                            double* __restrict__ scc, double* __restrict__ d,
                                                            double* __restrict__ e, double* __restrict__ tau) {
  constexpr int kStepThreads = 64 * NW;
  extern __shared__ double sh[];
  double* sv = sh;          // v of step k - 1 (indices >= k)
  double* sw = sh + J;      // w of step k - 1
  double* su = sh + 2 * J;  // row k after that update, then v of step k (indices >= k + 1)
  __shared__ double sred[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool upd = k > 0;  // uniform
  const double* rk = A + (int64_t)k * J;
  // this wave's row, loaded first (in bounds; used only if i < J)
  const int i = k + 1 + (int)blockIdx.x * NW + wave;
  double* row = A + (int64_t)min(i, J - 1) * J;
  constexpr int kRowRegs = RR;
  double a[kRowRegs];
#pragma unroll
  for (int u = 0; u < kRowRegs; ++u) {
    const int j = k + 1 + lane + 64 * u;
    a[u] = (j < J) ? row[j] : 0.0;
  }
  if (upd) {
    const double tp = scp[1];
    double part = 0.0;
    for (int j = k + tid; j < J; j += kStepThreads) {
      const double v = Vp[j], pj = Pp[j];
      sv[j] = v;
      sw[j] = pj;
      part += pj * v;
    }
    const double c2 = 0.5 * tp * block_sum_nw<NW>(part, sred);  // (the sum's barriers publish sv, sw)
    for (int j = k + tid; j < J; j += kStepThreads) sw[j] -= c2 * sv[j];
    __syncthreads();
  }
  const double vk = upd ? sv[k] : 0.0, wk = upd ? sw[k] : 0.0;
  double part = 0.0;
  for (int j = k + 1 + tid; j < J; j += kStepThreads) {
    const double x = upd ? rk[j] - (vk * sw[j] + wk * sv[j]) : rk[j];
    su[j] = x;
    if (j >= k + 2) part += x * x;
  }
  double sigma = block_sum_nw<NW>(part, sred);
  // alpha from the same expression as su[k + 1] (bit-identical), not from
  // su, whose entry k + 1 its owner rewrites below
  double alpha = upd ? rk[k + 1] - (vk * sw[k + 1] + wk * sv[k + 1]) : rk[k + 1];
  const bool tiny = row_is_tiny(alpha, sigma);  // uniform
  if (tiny) {
    part = 0.0;
    for (int j = k + 2 + tid; j < J; j += kStepThreads) {
      const double y = su[j] * kRowScale;
      part += y * y;
    }
    sigma = block_sum_nw<NW>(part, sred);
    alpha *= kRowScale;
  }
  double beta, tk, scale;
  reflector(alpha, sigma, tiny, beta, tk, scale);
  for (int j = k + 1 + tid; j < J; j += kStepThreads) {
    const double v = (j == k + 1) ? 1.0 : su[j] * scale;
    su[j] = v;  // each thread rewrites only its own entries
    if (blockIdx.x == 0) Vc[j] = v;
  }
  if (blockIdx.x == 0) {
    if (tid == 0) {
      scc[0] = beta;
      scc[1] = tk;
      d[k] = upd ? rk[k] - 2.0 * vk * wk : rk[k];
      e[k] = beta;
      tau[k] = tk;
    }
    if (upd)
      for (int j = k + 1 + tid; j < J; j += kStepThreads) A[(int64_t)(k - 1) * J + j] = sv[j];
  }
  __syncthreads();
  if (i < J) {  // uniform per wave
    const double vi = upd ? sv[i] : 0.0, wi = upd ? sw[i] : 0.0;
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < kRowRegs; ++u) {
      const int j = k + 1 + lane + 64 * u;
      if (j < J) {
        double x = a[u];
        if (upd) {
          x -= vi * sw[j] + wi * sv[j];
          row[j] = x;
        }
        t += x * su[j];
      }
    }
    t = wave_sum_fast(t);
    if (lane == 0) Pc[i] = tk * t;
  }
}

// ---------------------------------------------------------------- 2. eigenvalues
// Gershgorin interval and pivmin; every bisection workgroup recomputes them.
struct TriBounds {
  double glo, ghi, pivmin, tnorm, atol;
};

__device__ TriBounds tri_bounds(const double* __restrict__ d, const double* __restrict__ e, int J, double* sd,
                                double* se2, double* sred) {
  double glo = DBL_MAX, ghi = -DBL_MAX, e2max = 0.0;
  for (int i = threadIdx.x; i < J; i += blockDim.x) {
    const double di = d[i];
    const double em = (i > 0) ? fabs(e[i - 1]) : 0.0;
    const double ep = (i + 1 < J) ? fabs(e[i]) : 0.0;
    sd[i] = di;
    se2[i] = (i + 1 < J) ? e[i] * e[i] : 0.0;
    e2max = fmax(e2max, se2[i]);
    glo = fmin(glo, di - em - ep);
    ghi = fmax(ghi, di + em + ep);
  }
  TriBounds b;
  glo = -block_max<4>(-glo, sred);
  ghi = block_max<4>(ghi, sred);
  e2max = block_max<4>(e2max, sred);
  b.pivmin = DBL_MIN * fmax(1.0, e2max);
  b.tnorm = fmax(fabs(glo), fabs(ghi));
  const double widen = 2.1 * DBL_EPSILON * b.tnorm * J + 4.2 * b.pivmin;
  b.glo = glo - widen;
  b.ghi = ghi + widen;
  b.atol = 2.0 * DBL_EPSILON * b.tnorm + 4.0 * b.pivmin;
  return b;
}

// number of eigenvalues of T below sig (Sturm count of T - sig I)
__device__ __forceinline__ int sturm_count(const double* sd, const double* se2, int J, double sig, double pivmin) {
  int cnt = 0;
  double q = sd[0] - sig;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += (q < 0.0);
  for (int i = 1; i < J; ++i) {
    // 1/q by the hardware reciprocal refined with one Newton step
    double rq = __builtin_amdgcn_rcp(q);
    rq = fma(rq, fma(-q, rq, 1.0), rq);
    q = (sd[i] - sig) - se2[i - 1] * rq;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
  }
  return cnt;
}

// Starting intervals from geometric brackets: the Sturm counts at 0 and at
// tnorm * 10^-k, k = 15 .. 0 (one per lane of the first wave), after which
// eigenvalue a starts from the tightest bracket [x, y] with count(x) <= a <
// count(y) inside the Gershgorin interval.  A Gram matrix's eigenvalues span
// many decades and most are small, so each starts from an interval about its
// own size instead of the whole spectrum: several multisection rounds fewer
// for the small ones.
constexpr int kGeoPts = 17;
__device__ __forceinline__ void geo_brackets(const double* sd, const double* se2, int J, const TriBounds& b,
                                             double* sx, int* scnt) {
  const int tid = threadIdx.x;
  if (tid < kGeoPts) {
    double x = 0.0;
    if (tid > 0) {
      x = b.tnorm;  // tnorm * 10^-(kGeoPts - 1 - tid)
      for (int k = tid; k < kGeoPts - 1; ++k) x *= 0.1;
    }
    sx[tid] = x;
    scnt[tid] = sturm_count(sd, se2, J, x, b.pivmin);
  }
  __syncthreads();
}
__device__ __forceinline__ void geo_start(const double* sx, const int* scnt, int a, const TriBounds& b, double& lo,
                                          double& hi) {
  lo = b.glo;
  hi = b.ghi;
  for (int p = 0; p < kGeoPts; ++p) {
    const double x = sx[p];
    const int c = scnt[p];
    if (c <= a && x > lo) lo = x;
    if (c > a && x < hi) hi = x;
  }
}

// 256 threads, LANES per eigenvalue (LANES interior points per round), used
// by the batched form with 4 lanes: a batch holds thousands of eigenvalues,
// so the total number of Sturm counts (LANES x rounds: 4 x ~23 against
// 32 x ~11) decides, not the length of one eigenvalue's chain of rounds.
// The single-matrix form takes a whole workgroup per eigenvalue (fewer,
// latency-bound rounds; eig_bisect_wide_kernel).
constexpr int kBisLanesBatched = 4;
template <int LANES>
__device__ __forceinline__ void bisect_body(const double* __restrict__ d, const double* __restrict__ e, int J,
                                            double* __restrict__ lam, double* __restrict__ scal, int bx) {
  extern __shared__ double sh[];
  double* sd = sh;            // J
  double* se2 = sh + J;       // J
  double* sred = sh + 2 * J;  // 4
  __shared__ double sgx[kGeoPts];
  __shared__ int sgc[kGeoPts];
  const TriBounds b = tri_bounds(d, e, J, sd, se2, sred);
  geo_brackets(sd, se2, J, b, sgx, sgc);
  const int tid = threadIdx.x, lane = tid & 63;
  const int q = lane & (LANES - 1), gbase = lane & ~(LANES - 1);
  const int a = bx * (256 / LANES) + tid / LANES;  // ascending index
  if (bx == 0 && tid == 0) {
    scal[0] = b.tnorm;
    scal[1] = b.pivmin;
  }
  if (a >= J) return;
  double lo, hi;
  geo_start(sgx, sgc, a, b, lo, hi);
  for (int it = 0; it < 64 && (hi - lo) > b.atol; ++it) {
    const double h = (hi - lo) / (LANES + 1);
    const double sig = lo + h * (q + 1);
    const int cnt = sturm_count(sd, se2, J, sig, b.pivmin);
    const uint64_t bal = __ballot(cnt > a);
    const uint64_t m = (LANES == 64) ? bal : ((bal >> gbase) & ((1ull << (LANES & 63)) - 1));
    const int f = m ? (__ffsll((long long)m) - 1) : LANES;
    const double nlo = (f == 0) ? lo : lo + h * f;
    const double nhi = (f == LANES) ? hi : lo + h * (f + 1);
    lo = nlo;
    hi = nhi;
  }
  if (q == 0) lam[J - 1 - a] = 0.5 * (lo + hi);
}

// Single-matrix form with a whole workgroup per eigenvalue: its 256 threads
// test 256 interior points per round (257 subintervals instead of 65, so
// about 7 rounds instead of 9 reach the tolerance); the waves' ballots are
// combined through LDS.  Every thread holds the same interval (the same
// fixed-order data), so the loop is uniform over the workgroup.
__global__ __launch_bounds__(256) void eig_bisect_wide_kernel(const double* __restrict__ d,
                                                              const double* __restrict__ e, int J,
                                                              double* __restrict__ lam, double* __restrict__ scal) {
  extern __shared__ double sh[];
  double* sd = sh;            // J
  double* se2 = sh + J;       // J
  double* sred = sh + 2 * J;  // 4
  __shared__ uint64_t sbal[4];
  __shared__ double sgx[kGeoPts];
  __shared__ int sgc[kGeoPts];
  const TriBounds b = tri_bounds(d, e, J, sd, se2, sred);
  geo_brackets(sd, se2, J, b, sgx, sgc);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int a = blockIdx.x;  // ascending index
  if (a == 0 && tid == 0) {
    scal[0] = b.tnorm;
    scal[1] = b.pivmin;
  }
  double lo, hi;
  geo_start(sgx, sgc, a, b, lo, hi);
  for (int it = 0; it < 64 && (hi - lo) > b.atol; ++it) {
    const double h = (hi - lo) / 257.0;
    const double sig = lo + h * (tid + 1);
    const int cnt = sturm_count(sd, se2, J, sig, b.pivmin);
    const uint64_t bal = __ballot(cnt > a);
    if (lane == 0) sbal[wave] = bal;
    __syncthreads();
    int f = 256;  // first point with more than a eigenvalues below it
#pragma unroll
    for (int w = 3; w >= 0; --w)
      if (sbal[w]) f = 64 * w + __ffsll((long long)sbal[w]) - 1;
    __syncthreads();  // every thread has read sbal before the next round
    const double nlo = (f == 0) ? lo : lo + h * f;
    const double nhi = (f == 256) ? hi : lo + h * (f + 1);
    lo = nlo;
    hi = nhi;
  }
  if (tid == 0) lam[J - 1 - a] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------- 3. truncation
// The threshold is thr, or thr * (*nx2) when nx2 is non-null (so that
// eps^2 ||X||^2 / N is formed on the device without a host round trip).
// Tail sums: sum_{i>=R} max(lam_i, 0), accumulated from the smallest
// eigenvalue upward (eq. Un); R = J discards nothing.  fixed > 0 selects the
// fixed-rank variant instead: R = min(fixed, J), and disc is its tail.
__device__ __forceinline__ void truncate_body(const double* __restrict__ lam, int J, double thr,
                                              const double* __restrict__ nx2, int fixed,
                                              int64_t* __restrict__ Rout, double* __restrict__ disc) {
  if (nx2 != nullptr) thr *= *nx2;
  const int Rf = (fixed > 0) ? min(fixed, J) : 0;
  int R = J;
  double tailR = 0.0;
  // smallest R in 1..J with sum_{i>=R} max(lam_i, 0) <= thr (lam descending),
  // or R = Rf; the loop runs over all entries without an early exit, so that
  // the loads can be issued ahead (the tails are monotone in r)
  double tail = 0.0;
  bool ok = true;
#pragma unroll 8
  for (int r = J - 1; r >= 1; --r) {
    tail += fmax(lam[r], 0.0);
    ok = ok && (Rf > 0 ? r >= Rf : tail <= thr);
    R = ok ? r : R;
    tailR = ok ? tail : tailR;
  }
  *Rout = R;
  *disc = tailR;
}

// One workgroup of 64 threads: the eigenvalues are staged in LDS (dynamic,
// J doubles), then thread 0 runs the sequential tail sums over LDS.
__global__ void eig_truncate_kernel(const double* __restrict__ lam, int J, double thr,
                                    const double* __restrict__ nx2, int fixed, int64_t* __restrict__ Rout,
                                    double* __restrict__ disc) {
  extern __shared__ double sl[];
  for (int i = threadIdx.x; i < J; i += blockDim.x) sl[i] = lam[i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  truncate_body(sl, J, thr, nx2, fixed, Rout, disc);
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

// 1/x from the hardware reciprocal refined by one Newton step.
__device__ __forceinline__ double rcp_refined(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// Inverse iteration state in LDS, one thread per vector; every array holds J
// entries per vector, interleaved by thread (entry i of thread t at
// i * nvw + t) so that accesses are bank-conflict free.
constexpr int kInvitArrays = 7;
// vectors per workgroup: the arrays of all its vectors fit in 128 KB of LDS
inline int invit_vectors_per_group(int64_t J) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(64, (128 * 1024) / (8 * kInvitArrays * J)));
}

// Back substitution y = U^{-1} x (U upper triangular with two superdiagonals,
// reciprocal pivots) and ||y||^2.  x and y are distinct arrays, so that the
// loads of the unrolled loop are issued ahead of the stores.
__device__ __forceinline__ double invit_back(const double* __restrict__ x, const double* __restrict__ wr,
                                             const double* __restrict__ w1, const double* __restrict__ w2,
                                             double* __restrict__ y, int J, int nvw) {
  double y1 = 0.0, y2 = 0.0, nrm = 0.0;
#pragma unroll 8
  for (int i = J - 1; i >= 0; --i) {
    const size_t o = (size_t)i * nvw;
    const double yi = (x[o] - w1[o] * y1 - w2[o] * y2) * wr[o];
    y[o] = yi;
    nrm += yi * yi;
    y2 = y1;
    y1 = yi;
  }
  return nrm;
}

// Forward substitution with the stored multipliers and interchanges:
// y = L^{-1} P (s x).
__device__ __forceinline__ void invit_forward(const double* __restrict__ x, const double* __restrict__ wf,
                                              const double* __restrict__ wp, double* __restrict__ y, double s,
                                              int J, int nvw) {
  double xc = x[0] * s;
#pragma unroll 8
  for (int i = 0; i + 1 < J; ++i) {
    const size_t o = (size_t)i * nvw;
    const double xn = x[o + nvw] * s;
    const double f = wf[o];
    const bool sw = wp[o] != 0.0;
    y[o] = sw ? xn : xc;
    xc = sw ? fma(-f, xn, xc) : fma(-f, xc, xn);
  }
  y[(size_t)(J - 1) * nvw] = xc;
}

// One thread per vector; a workgroup of 64 threads serves `nvw` vectors.
// Two steps of inverse iteration with (T - lambda I)/||T|| from a pseudo-random
// start.  The first step factors it (LU with partial pivoting, rows i and i+1
// interchanged when |l_i| > |u_ii|; tiny pivots replaced by +-eps) while it
// forward-substitutes the start vector, keeping the reciprocal pivots, the two
// superdiagonals of U, the multipliers and the interchanges; the second step
// reuses them (one forward and one back substitution, no division).  The
// pivoting is written without branches, so the lanes of a wave stay together.
__device__ __forceinline__ void invit_body(const double* __restrict__ d, const double* __restrict__ e, int J,
                                           const double* __restrict__ lam, const int64_t* __restrict__ Rp,
                                           const double* __restrict__ scal, double* __restrict__ Zt, int nvw,
                                           double* sh, int bx) {
  const int tid = threadIdx.x;
  const int t = bx * nvw + tid;
  const int R = (int)*Rp;
  if (tid >= nvw || t >= R) return;
  const double tnorm = scal[0];
  if (tnorm == 0.0) {
    for (int i = 0; i < J; ++i) Zt[(int64_t)t * J + i] = (i == t) ? 1.0 : 0.0;
    return;
  }
  const double inv = 1.0 / tnorm;
  const double eps = DBL_EPSILON;
  const size_t JN = (size_t)J * nvw;
  double* Wr = sh + 0 * JN + tid;  // 1 / u_ii
  double* W1 = sh + 1 * JN + tid;  // u_{i,i+1}
  double* W2 = sh + 2 * JN + tid;  // u_{i,i+2}
  double* Wf = sh + 3 * JN + tid;  // multiplier of step i
  double* Wp = sh + 4 * JN + tid;  // 1 if rows i, i+1 were interchanged
  double* Xa = sh + 5 * JN + tid;  // iterates
  double* Xb = sh + 6 * JN + tid;
  const int vec = t;
  const double shift = lam[vec] * inv;
  // step 1: factor + forward substitution of the start vector; the running
  // row (dd, du) and its right-hand side xc are carried in registers
  double dd = d[0] * inv - shift;
  double du = (J > 1) ? e[0] * inv : 0.0;
  double xc = hash_unit(0u, (uint32_t)vec);
  for (int i = 0; i + 1 < J; ++i) {
    const size_t o = (size_t)i * nvw;
    const double li = e[i] * inv;
    const double dn = d[i + 1] * inv - shift;
    const double un = (i + 2 < J) ? e[i + 1] * inv : 0.0;
    const double xn = hash_unit((uint32_t)(i + 1), (uint32_t)vec);
    const bool sw = fabs(dd) < fabs(li);
    const double dg = (fabs(dd) < eps) ? ((dd < 0.0) ? -eps : eps) : dd;
    const double rp = rcp_refined(sw ? li : dg);
    const double f = (sw ? dd : li) * rp;
    Wr[o] = rp;
    W1[o] = sw ? dn : du;
    W2[o] = sw ? un : 0.0;
    Wf[o] = f;
    Wp[o] = sw ? 1.0 : 0.0;
    Xa[o] = sw ? xn : xc;
    const double ndd = sw ? du - f * dn : dn - f * du;
    const double ndu = sw ? -f * un : un;
    xc = sw ? xc - f * xn : xn - f * xc;
    dd = ndd;
    du = ndu;
  }
  if (fabs(dd) < eps) dd = (dd < 0.0) ? -eps : eps;
  {
    const size_t o = (size_t)(J - 1) * nvw;
    Wr[o] = rcp_refined(dd);
    W1[o] = 0.0;
    W2[o] = 0.0;
    Xa[o] = xc;
  }
  const double s1 = 1.0 / sqrt(invit_back(Xa, Wr, W1, W2, Xb, J, nvw));
  // step 2
  invit_forward(Xb, Wf, Wp, Xa, s1, J, nvw);
  const double s2 = 1.0 / sqrt(invit_back(Xa, Wr, W1, W2, Xb, J, nvw));
  for (int i = 0; i < J; ++i) Zt[(int64_t)vec * J + i] = Xb[(size_t)i * nvw] * s2;
}

__global__ __launch_bounds__(64) void eig_invit_kernel(const double* __restrict__ d, const double* __restrict__ e, int J,
                                                       const double* __restrict__ lam, const int64_t* __restrict__ Rp,
                                                       const double* __restrict__ scal, double* __restrict__ Zt,
                                                       int nvw) {
  extern __shared__ double sh[];
  invit_body(d, e, J, lam, Rp, scal, Zt, nvw, sh, blockIdx.x);
}

// ---------------------------------------------------------------- 5. re-orthogonalisation
// Classical Gram-Schmidt, twice, of vector i against the preceding vectors
// whose eigenvalue lies within otol of lambda_i, then normalisation.  Z points
// either to the vectors in global memory or to a copy in LDS.
__device__ __forceinline__ void orth_loop(double* __restrict__ Z, int J, int R, const double* __restrict__ lam,
                                          double otol, double* hs, double* sred) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int jlo = 0;
  for (int i = 1; i < R; ++i) {
    while (jlo < i && lam[jlo] - lam[i] >= otol) ++jlo;
    if (jlo == i) continue;  // uniform
    double* zi = Z + (int64_t)i * J;
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = jlo + wave; j < i; j += 16) {
        const double* zj = Z + (int64_t)j * J;
        double h = 0.0;
        for (int r = lane; r < J; r += 64) h += zj[r] * zi[r];
        h = wave_sum_fast(h);
        if (lane == 0) hs[j - jlo] = h;
      }
      __syncthreads();
      for (int r = tid; r < J; r += kEigThreads) {
        double v = zi[r];
        for (int j = jlo; j < i; ++j) v -= hs[j - jlo] * Z[(int64_t)j * J + r];
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

// Blocked form, for R * J beyond the LDS copy: blocks of kOB consecutive
// vectors.  A block is first projected, twice, against the preceding (final)
// vectors of its window, kOB of them at a time, with FP64 MFMA products: the
// chunk's coefficients C = Z_chunk Z_blk^T (masked to each vector's window),
// then Z_blk -= C^T Z_chunk.  Then each vector of the block is orthogonalised
// (classical Gram-Schmidt, twice) against the block's earlier vectors of its
// window and normalised.  In exact arithmetic this is the same projection as
// the vector-by-vector loop.  The chunks are read from global memory; the
// block lives in LDS (zero-padded rows of Jp) while kOB rows of J fit
// (J <= 1024), otherwise (GLB) it is updated in place in global memory, with
// the entries past the block's R - i0 vectors or past J masked to zero.
constexpr int kOB = 16;  // vectors per block
constexpr int kOC = 64;  // preceding vectors per chunk
__host__ __device__ constexpr int orth_ksplit(int J) { return J <= 960 ? 4 : 2; }
// LDS of the blocked forms (doubles); the LDS block runs while this stays
// within the 160 KB a gfx950 workgroup may use (every J up to 1024).
constexpr int kEigLdsMax = 160 * 1024 / 8;
__host__ __device__ constexpr int64_t orth_blocked_doubles(int64_t J, bool glb = false) {
  return J + 32 + (glb ? 0 : (int64_t)kOB * ((J + 15) & ~int64_t(15))) + (int64_t)orth_ksplit((int)J) * kOC * kOB;
}

template <bool GLB>
__device__ __forceinline__ void orth_blocked(double* __restrict__ Z, int J, int R, int first,
                                             const double* __restrict__ lam, double otol, double* sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int il = lane & 15, q = lane >> 4;
  const int Jp = (J + 15) & ~15;
  const int KS = orth_ksplit(J);
  const int ZS = GLB ? J : Jp;                        // row stride of the block
  double* hs = sh;                                    // kOB (in-block coefficients)
  double* sred = sh + J;                              // 16
  int* sjlo = reinterpret_cast<int*>(sh + J + 16);    // kOB window starts
  double* sC = sh + J + 32 + (GLB ? 0 : kOB * Jp);    // [KS][kOC][kOB] partial coefficients
  for (int i0 = first; i0 < R; i0 += kOB) {
    const int nb = min(kOB, R - i0);
    double* Zb = GLB ? Z + (int64_t)i0 * J : sh + J + 32;  // [kOB][ZS]
    if (tid < kOB) {
      // window start: smallest j <= i with lam_j - lam_i < otol (lam descending)
      const int i = i0 + tid;
      int lo = i < R ? 0 : i, hi = i;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (lam[mid] - lam[i] < otol) hi = mid;
        else lo = mid + 1;
      }
      sjlo[tid] = lo;
    }
    if (!GLB) {
      for (int x = tid; x < kOB * Jp; x += kEigThreads) {
        const int t = x / Jp, r = x - t * Jp;
        Zb[x] = (t < nb && r < J) ? Z[(int64_t)(i0 + t) * J + r] : 0.0;
      }
    }
    __syncthreads();
    const int jw = sjlo[0];  // window starts grow with i
    for (int pass = 0; pass < 2 && jw < i0; ++pass) {
      for (int jc = jw; jc < i0; jc += kOC) {
        const int nc = min(kOC, i0 - jc);
        // coefficients: wave -> (row tile a of the chunk, reduction split ks)
        {
          const int a = wave & 3, ks = wave >> 2;
          if (ks < KS) {
            const int nst = Jp / 4, s0 = nst * ks / KS, s1 = nst * (ks + 1) / KS;
            const int jj = 16 * a + il;
            const double* zr = Z + (int64_t)(jc + min(jj, nc - 1)) * J;
            const bool rowok = jj < nc;
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            // reduction steps in groups of 8 loads (in bounds, masked here); the
            // other waves of the SIMD cover a group's load latency
            for (int g0 = s0; g0 < s1; g0 += 8) {
              double x[8], y[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                x[u] = zr[min(4 * (g0 + u) + q, J - 1)];
                y[u] = GLB ? Zb[(int64_t)min(il, nb - 1) * J + min(4 * (g0 + u) + q, J - 1)] : 0.0;
              }
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                const int st = g0 + u, r = 4 * st + q;
                const double av = (rowok && st < s1 && r < J) ? x[u] : 0.0;
                const double bv = GLB ? ((il < nb && r < J) ? y[u] : 0.0) : Zb[il * Jp + min(r, Jp - 1)];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
              }
            }
            // D[(l >> 4) + 4v][l & 15]: chunk row 16 a + q + 4 v, block vector il
#pragma unroll
            for (int v = 0; v < 4; ++v) sC[(ks * kOC + 16 * a + q + 4 * v) * kOB + il] = acc[v];
          }
        }
        __syncthreads();
        {
          // one (chunk row, block vector) per thread: sum the splits, mask to the window
          const int jj = tid >> 4, t = tid & 15;
          double c = 0.0;
          for (int ks = 0; ks < KS; ++ks) c += sC[(ks * kOC + jj) * kOB + t];
          sC[jj * kOB + t] = (jj < nc && t < nb && jc + jj >= sjlo[t]) ? c : 0.0;
        }
        __syncthreads();
        // Z_blk -= C^T Z_chunk: wave -> 16-column tiles of the block
        for (int b = wave; b < Jp / 16; b += 16) {
          const int r = 16 * b + il;
          d4 acc;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int t = q + 4 * v;
            if (GLB) {
              const double zv = Zb[(int64_t)min(t, nb - 1) * J + min(r, J - 1)];  // in bounds; masked
              acc[v] = (t < nb && r < J) ? zv : 0.0;
            } else {
              acc[v] = Zb[t * Jp + r];
            }
          }
#pragma unroll
          for (int h = 0; h < 2; ++h) {  // two halves of 8 steps (bounds the loads in flight)
#pragma unroll
            for (int st = 8 * h; st < 8 * h + 8; ++st) {
              const int jj = 4 * st + q;
              const double x = Z[(int64_t)(jc + min(jj, nc - 1)) * J + min(r, J - 1)];  // in bounds; masked below
              const double bv = (jj < nc && r < J) ? x : 0.0;
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-sC[jj * kOB + il], bv, acc, 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int t = q + 4 * v;
            if (GLB) {
              if (t < nb && r < J) Zb[(int64_t)t * J + r] = acc[v];
            } else {
              Zb[t * Jp + r] = acc[v];
            }
          }
        }
        __syncthreads();
      }
    }
    // within the block, vector by vector
    for (int t = 0; t < nb; ++t) {
      const int i = i0 + t;
      if (sjlo[t] >= i) continue;  // uniform: no neighbour within otol
      double* zt = Zb + (int64_t)t * ZS;
      const int u0 = max(sjlo[t], i0) - i0;
      for (int pass = 0; pass < 2 && u0 < t; ++pass) {
        for (int u = u0 + wave; u < t; u += 16) {
          double h = 0.0;
          for (int r = lane; r < J; r += 64) h += Zb[(int64_t)u * ZS + r] * zt[r];
          h = wave_sum_fast(h);
          if (lane == 0) hs[u] = h;
        }
        __syncthreads();
        for (int r = tid; r < J; r += kEigThreads) {
          double v = zt[r];
          for (int u = u0; u < t; ++u) v -= hs[u] * Zb[(int64_t)u * ZS + r];
          zt[r] = v;
        }
        __syncthreads();
      }
      double nn = 0.0;
      for (int r = tid; r < J; r += kEigThreads) nn += zt[r] * zt[r];
      nn = block_sum_1024(nn, sred);
      const double rn = 1.0 / sqrt(nn);
      for (int r = tid; r < J; r += kEigThreads) zt[r] *= rn;
      __syncthreads();
    }
    if (!GLB) {
      for (int x = tid; x < nb * Jp; x += kEigThreads) {
        const int t = x / Jp, r = x - t * Jp;
        if (r < J) Z[(int64_t)(i0 + t) * J + r] = Zb[x];
      }
    }
    __syncthreads();
  }
}

// LDS capacity (doubles) for the LDS copy of the R leading vectors.
constexpr int kOrthCap = 14336;
constexpr int kOrthCapBatched = 4096;
__host__ __device__ inline int orth_cap_batched(int64_t Jmax) {
  return (int)(Jmax * Jmax < kOrthCapBatched ? Jmax * Jmax : kOrthCapBatched);
}
inline bool orth_blocked_fits(int64_t J) { return orth_blocked_doubles(J) <= kEigLdsMax; }
// the blocked form of a single matrix: 1 with the block in LDS, 2 in place
inline int orth_blocked_mode(int64_t J) { return orth_blocked_fits(J) ? 1 : 2; }
// LDS of eig_orth_kernel: the copy form, and the blocked form unless the
// right-looking launches (rl) take the matrices beyond the copy
inline size_t orth_lds_bytes(int64_t J, bool rl = false) {
  const int64_t copy = J + 16 + std::min<int64_t>(J * J, kOrthCap);
  return sizeof(double) *
         (size_t)std::max<int64_t>(copy, rl ? 0 : orth_blocked_doubles(J, orth_blocked_mode(J) == 2));
}

// The vectors are copied to LDS when R * J fits in `cap` doubles (the rounds
// then cost LDS latency instead of global-memory round trips), and only the
// vectors from the first one that changes onward are written back; otherwise
// the blocked form runs (`blocked` 1 or 2, which needs orth_lds_bytes of LDS),
// the right-looking launches that follow do the work (`blocked` 3), or the
// vector-by-vector loop on global memory (the batched form, whose workgroups
// keep their LDS small).
__device__ __forceinline__ void orth_body(double* __restrict__ Zt, int J, const double* __restrict__ lam,
                                          const int64_t* __restrict__ Rp, const double* __restrict__ scal,
                                          double* sh, int cap, int blocked) {
  double* hs = sh;        // J
  double* sred = sh + J;  // 16
  const int R = (int)*Rp;
  const double otol = 1e-2 * scal[0];
  int first = 1;  // first vector with a neighbour within otol
  while (first < R && lam[first - 1] - lam[first] >= otol) ++first;
  if (first >= R) return;  // uniform: nothing to do
  if ((int64_t)R * J > cap) {
    if (blocked == 1) orth_blocked<false>(Zt, J, R, first, lam, otol, sh);
    else if (blocked == 2) orth_blocked<true>(Zt, J, R, first, lam, otol, sh);
    else if (blocked == 3) return;
    else orth_loop(Zt, J, R, lam, otol, hs, sred);
    return;
  }
  double* Zs = sh + J + 16;
  for (int x = threadIdx.x; x < R * J; x += kEigThreads) Zs[x] = Zt[x];
  __syncthreads();
  orth_loop(Zs, J, R, lam, otol, hs, sred);
  for (int x = (first - 1) * J + threadIdx.x; x < R * J; x += kEigThreads) Zt[x] = Zs[x];
}

__global__ __launch_bounds__(kEigThreads) void eig_orth_kernel(double* __restrict__ Zt, int J,
                                                               const double* __restrict__ lam,
                                                               const int64_t* __restrict__ Rp,
                                                               const double* __restrict__ scal, int blocked) {
  extern __shared__ double sh[];
  orth_body(Zt, J, lam, Rp, scal, sh, (int)std::min<int64_t>((int64_t)J * J, kOrthCap), blocked);
}

// Right-looking form for single matrices of kRlMinJ <= J <= kRlMaxJ: a sweep
// of block modified Gram-Schmidt, one launch per block b = -1, 0, 1, ...,
// then a second sweep in one launch (eig_orth_rl2_kernel).  In the first,
// once block b is final, every later block c that holds
// vectors whose window reaches into b is projected against b by a workgroup
// of its own (coefficients C = Z_b Z_c^T masked to the windows, then
// Z_c -= C^T Z_b, FP64 MFMA products, Z_c in LDS, Z_b read from global
// memory), and the workgroup of block b + 1 then completes that block within
// itself.  The projections of all later blocks run side by side on many CUs
// instead of one after another on one.  This sweep leaves a loss of
// orthogonality of the order of u times the condition of the iterates
// (rounding in a later block's projection is not removed by an earlier one);
// the second sweep, over nearly orthonormal vectors, brings it to rounding,
// as the second pass of classical Gram-Schmidt does.  Within the block, the vectors
// from the first one whose window reaches a block vector onward are
// orthonormalised by two passes of Cholesky QR (G = Z Z^T = L L^T,
// Z <- L^{-1} Z), which gives the Gram-Schmidt result in that order; if a
// pivot shows a nearly dependent vector (L_tt^2 < 1e-8 G_tt) the block takes
// the vector-by-vector classical Gram-Schmidt instead.  Block vectors outside
// each other's window are already orthogonal to rounding (their eigenvalues
// differ by more than 1e-2 ||T||), so treating them together changes them at
// that level only.  Launches for blocks beyond R, and every launch when R * J
// fits the LDS copy of eig_orth_kernel, return at once.
constexpr int kRlWaves = 8;
constexpr int kRlThreads = 64 * kRlWaves;
constexpr int kRlMinJ = 384;
constexpr int kRlMaxJ = 1024;
__host__ __device__ constexpr int64_t orth_rl_doubles(int64_t J) {
  return (int64_t)kOB * ((J + 15) & ~int64_t(15)) + kRlWaves * 256 + 2 * 256 + 16 + 16 + 16;
}
// the single-launch second sweep: a 64 x 16 coefficient block instead of 16 x 16
__host__ __device__ constexpr int64_t orth_rl2_doubles(int64_t J) { return orth_rl_doubles(J) + 1024 - 256; }

// Fixed-order sum over a workgroup of kRlThreads threads; all threads get it.
__device__ __forceinline__ double block_sum_rl(double v, double* sred) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum_fast(v);
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kRlWaves; ++w) s += sred[w];
  __syncthreads();
  return s;
}

// Window starts of block c's vectors (window of vector i: the j <= i with
// lam_j - lam_i < otol; lam is descending, so the j < i outside the window
// form a prefix and the start is their count; each thread tests two j, as
// R <= J <= 1024), the smallest start (wmin) and the first block row whose
// window reaches a block vector (t0; kOB if none).
__device__ __forceinline__ void rl_block_windows(const double* __restrict__ lam, int R, int c0, int nb, double otol,
                                                 int* sjlo, int* scnt, int& wmin, int& t0) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double lj[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int j = tid + u * kRlThreads;
    lj[u] = (j < R) ? lam[j] : 0.0;
  }
#pragma unroll
  for (int t = 0; t < kOB; ++t) {
    const int i = c0 + t;
    const double li = lam[min(i, R - 1)];
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int j = tid + u * kRlThreads;
      cnt += __popcll(__ballot(j < i && lj[u] - li >= otol));
    }
    if (lane == 0) scnt[wave * kOB + t] = cnt;
  }
  __syncthreads();
  if (tid < kOB) {
    int cnt = 0;
#pragma unroll
    for (int w = 0; w < kRlWaves; ++w) cnt += scnt[w * kOB + tid];
    sjlo[tid] = (c0 + tid < R) ? cnt : c0 + tid;
  }
  __syncthreads();
  wmin = c0 + kOB;
  t0 = kOB;
  for (int t = 0; t < nb; ++t) {
    const int st = sjlo[t];
    wmin = min(wmin, st);
    if (st < c0 + t) t0 = min(t0, max(st, c0) - c0);
  }
}

// Orthonormalisation of a block of kOB vectors within itself, held in LDS
// (Zc, rows of Jp), from its row t0 on (shifted Cholesky QR3, or the
// vector-by-vector classical Gram-Schmidt within the windows if a pivot
// fails).  All kRlThreads threads call it.
__device__ __forceinline__ void rl_block_finish(double* Zc, int Jp, int J, int c0, int nb, int t0, const int* sjlo,
                                                double* sP, double* sL, double* sRd, double* shs, int* sflag) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int il = lane & 15, q = lane >> 4;
  const int nst = Jp / 4;
  const int s0 = nst * wave / kRlWaves, s1 = nst * (wave + 1) / kRlWaves;
  bool done = false;
  for (int pass = 0; pass < 2; ++pass) {
    {
      // G = Z_c Z_c^T: lane (il, q) supplies Z_c[il][4 st + q] as both operands
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int st = s0; st < s1; ++st) {
        const double v = Zc[il * Jp + 4 * st + q];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) sP[wave * 256 + (q + 4 * v) * 16 + il] = acc[v];
    }
    __syncthreads();
    if (wave == 0) {
      // Cholesky of the rows t0..nb-1 (the others: identity), lane t & 15
      // holding row t; right-looking, column k by column k
      const int t = lane & 15;
      const bool act = t >= t0 && t < nb;
      double a[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int x = t * 16 + j;
        double g = 0.0;
#pragma unroll
        for (int w = 0; w < kRlWaves; ++w) g += sP[w * 256 + x];
        const bool jact = j >= t0 && j < nb;
        a[j] = act ? (jact ? g : 0.0) : (j == t ? 1.0 : 0.0);
      }
      double gtt = 1.0;
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (j == t) gtt = a[j];
      double ratio = 1.0;
      bool okp = true;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const double dk = __shfl(a[k], k, 64);  // lane k's updated diagonal
        okp = okp && dk > 0.0;
        const double lkk = dk > 0.0 ? sqrt(dk) : 1.0;
        if (t == k) ratio = dk / gtt;
        const double lik = (t == k) ? lkk : ((t > k) ? a[k] / lkk : 0.0);
        a[k] = lik;
#pragma unroll
        for (int j = k + 1; j < 16; ++j) {
          const double ljk = __shfl(lik, j, 64);
          if (t >= j) a[j] -= lik * ljk;
        }
      }
      const double rmin = act ? ratio : 1.0;
      double m = rmin;
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off, 16));
      if (lane < 16) {
        double ltt = 1.0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          sL[t * 16 + j] = (j < t) ? a[j] : 0.0;
          if (j == t) ltt = a[j];
        }
        sRd[t] = 1.0 / ltt;
      }
      if (lane == 0) sflag[0] = (okp && m >= 1e-8) ? 1 : 0;
    }
    __syncthreads();
    if (!sflag[0]) break;  // uniform
    // Z_c <- L^{-1} Z_c, column by column
    for (int r = tid; r < J; r += kRlThreads) {
      double z[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) z[t] = Zc[t * Jp + r];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        double v = z[t];
#pragma unroll
        for (int u = 0; u < t; ++u) v -= sL[t * 16 + u] * z[u];
        z[t] = v * sRd[t];
      }
#pragma unroll
      for (int t = 0; t < 16; ++t) Zc[t * Jp + r] = z[t];
    }
    __syncthreads();
    done = pass == 1;
  }
  if (!done) {
    // classical Gram-Schmidt, twice, vector by vector within the windows
    for (int t = t0; t < nb; ++t) {
      const int i = c0 + t;
      if (sjlo[t] >= i) continue;  // uniform: no neighbour within otol
      double* zt = Zc + t * Jp;
      const int u0 = max(sjlo[t], c0) - c0;
      for (int pass = 0; pass < 2 && u0 < t; ++pass) {
        for (int u = u0 + wave; u < t; u += kRlWaves) {
          double h = 0.0;
          for (int r = lane; r < J; r += 64) h += Zc[u * Jp + r] * zt[r];
          h = wave_sum_fast(h);
          if (lane == 0) shs[u] = h;
        }
        __syncthreads();
        for (int r = tid; r < J; r += kRlThreads) {
          double v = zt[r];
          for (int u = u0; u < t; ++u) v -= shs[u] * Zc[u * Jp + r];
          zt[r] = v;
        }
        __syncthreads();
      }
      double nn = 0.0;
      for (int r = tid; r < J; r += kRlThreads) nn += zt[r] * zt[r];
      nn = block_sum_rl(nn, sP);
      const double rn = 1.0 / sqrt(nn);
      for (int r = tid; r < J; r += kRlThreads) zt[r] *= rn;
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kRlThreads) void eig_orth_rl_kernel(double* __restrict__ Z, int J,
                                                                 const double* __restrict__ lam,
                                                                 const int64_t* __restrict__ Rp,
                                                                 const double* __restrict__ scal, int b, int cap) {
  extern __shared__ double sh[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int il = lane & 15, q = lane >> 4;
  const int R = (int)*Rp;
  if ((int64_t)R * J <= cap) return;  // eig_orth_kernel's LDS copy form did it
  const int c = b + 1 + (int)blockIdx.x;
  const int c0 = kOB * c;
  if (c0 >= R) return;
  const int nb = min(kOB, R - c0);
  const int Jp = (J + 15) & ~15;
  double* Zc = sh;                                       // [kOB][Jp], zero-padded
  double* sP = Zc + kOB * Jp;                            // [kRlWaves][16][16] per-wave partial products
  double* sC = sP + kRlWaves * 256;                      // [16][16] coefficients
  double* sL = sC + 256;                                 // [16][16] Cholesky factor, row t = L_t*
  double* sRd = sL + 256;                                // [16] 1 / L_tt
  double* shs = sRd + 16;                                // [16] Gram-Schmidt coefficients
  int* sjlo = reinterpret_cast<int*>(shs + 16);          // [16] window starts
  int* sflag = sjlo + 16;                                // [1]
  const double otol = 1e-2 * scal[0];
  // Z_c (zero-padded to Jp columns) and the window data are loaded together
  constexpr int kZcRegs = kOB * kRlMaxJ / kRlThreads;
  double zr[kZcRegs];
#pragma unroll
  for (int u = 0; u < kZcRegs; ++u) {
    const int x = tid + u * kRlThreads;
    const int t = x / Jp, r = x - t * Jp;
    zr[u] = (x < kOB * Jp && t < nb && r < J) ? Z[(int64_t)(c0 + t) * J + r] : 0.0;
  }
  int wmin, t0;
  rl_block_windows(lam, R, c0, nb, otol, sjlo, reinterpret_cast<int*>(sP), wmin, t0);
  const int b0 = kOB * b;
  const bool proj = b >= 0 && wmin < b0 + kOB;
  const bool fin = (c == b + 1) && t0 < nb;
  if (!proj && !fin) return;  // uniform
#pragma unroll
  for (int u = 0; u < kZcRegs; ++u) {
    const int x = tid + u * kRlThreads;
    if (x < kOB * Jp) Zc[x] = zr[u];
  }
  __syncthreads();
  const int nst = Jp / 4;  // reduction steps of 4
  const int s0 = nst * wave / kRlWaves, s1 = nst * (wave + 1) / kRlWaves;
  if (proj) {
    {
      // C[i][j] = sum_r Z_b[i][r] Z_c[j][r] over this wave's steps, 16 loads of
      // Z_b in flight (Z_c is zero past J, so the clamped loads need no mask)
      const double* zb = Z + (int64_t)(b0 + il) * J;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int g0 = s0; g0 < s1; g0 += 16) {
        double x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) x[u] = zb[min(4 * (g0 + u) + q, J - 1)];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int st = g0 + u;
          const double av = (st < s1) ? x[u] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Zc[il * Jp + min(4 * st + q, Jp - 1)], acc, 0, 0, 0);
        }
      }
      // D[(l >> 4) + 4v][l & 15] = C[i][j], i = q + 4 v, j = il
#pragma unroll
      for (int v = 0; v < 4; ++v) sP[wave * 256 + (q + 4 * v) * 16 + il] = acc[v];
    }
    __syncthreads();
    if (tid < 256) {
      const int i = tid >> 4, j = tid & 15;
      double cv = 0.0;
#pragma unroll
      for (int w = 0; w < kRlWaves; ++w) cv += sP[w * 256 + tid];
      sC[tid] = (j < nb && b0 + i >= sjlo[j]) ? cv : 0.0;
    }
    __syncthreads();
    // Z_c[j][r] -= sum_i C[i][j] Z_b[i][r]: wave -> 16-column tiles T, all of
    // its tiles' Z_b values loaded first (at most 8 tiles for J <= 1024)
    {
      constexpr int kTiles = kRlMaxJ / 16 / kRlWaves;
      double x[kTiles][4];
#pragma unroll
      for (int tt = 0; tt < kTiles; ++tt) {
        const int r = 16 * (wave + kRlWaves * tt) + il;
#pragma unroll
        for (int st = 0; st < 4; ++st) x[tt][st] = Z[(int64_t)(b0 + 4 * st + q) * J + min(r, J - 1)];  // in bounds
      }
      double cq[4];
#pragma unroll
      for (int st = 0; st < 4; ++st) cq[st] = -sC[(4 * st + q) * 16 + il];
#pragma unroll
      for (int tt = 0; tt < kTiles; ++tt) {
        const int T = wave + kRlWaves * tt;
        if (T < Jp / 16) {  // uniform per wave
          const int r = 16 * T + il;
          d4 acc;
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[v] = Zc[(q + 4 * v) * Jp + r];
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            const double bv = (r < J) ? x[tt][st] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(cq[st], bv, acc, 0, 0, 0);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) Zc[(q + 4 * v) * Jp + r] = acc[v];
        }
      }
    }
    __syncthreads();
  }
  if (fin) rl_block_finish(Zc, Jp, J, c0, nb, t0, sjlo, sP, sL, sRd, shs, sflag);
  for (int x = tid; x < nb * Jp; x += kRlThreads) {
    const int t = x / Jp, r = x - t * Jp;
    if (r < J) Z[(int64_t)(c0 + t) * J + r] = Zc[x];
  }
}

// The second sweep in one launch: after the first sweep the vectors are
// orthonormal up to a small error e, so each block can be projected against
// all preceding vectors of its windows at once, reading them as the first
// sweep left them (Zs) and writing its result elsewhere (Zd): the error left
// is of order e^2 + u.  Workgroup c takes block c: projections against the
// preceding vectors in chunks of 64 (coefficients C = Z_chunk Z_c^T over two
// halves of the rows, masked to the windows, then Z_c -= C^T Z_chunk, FP64
// MFMA), then the block finish.  Every block is written to Zd (unchanged
// ones too), so that Zd holds all R vectors; when R * J fits the LDS copy
// form of eig_orth_kernel, which left its result in Zs, the blocks are only
// copied.
__global__ __launch_bounds__(kRlThreads) void eig_orth_rl2_kernel(const double* __restrict__ Zs,
                                                                  double* __restrict__ Zd, int J,
                                                                  const double* __restrict__ lam,
                                                                  const int64_t* __restrict__ Rp,
                                                                  const double* __restrict__ scal, int cap) {
  extern __shared__ double sh[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int il = lane & 15, q = lane >> 4;
  const int R = (int)*Rp;
  const int c0 = kOB * (int)blockIdx.x;
  if (c0 >= R) return;
  const int nb = min(kOB, R - c0);
  const int Jp = (J + 15) & ~15;
  double* Zc = sh;                                       // [kOB][Jp], zero-padded
  double* sP = Zc + kOB * Jp;                            // [2][64][16] partial coefficients (also the finish's)
  double* sC = sP + kRlWaves * 256;                      // [64][16] coefficients of a chunk
  double* sL = sC + 1024;                                // [16][16]
  double* sRd = sL + 256;                                // [16]
  double* shs = sRd + 16;                                // [16]
  int* sjlo = reinterpret_cast<int*>(shs + 16);          // [16]
  int* sflag = sjlo + 16;                                // [1]
  constexpr int kZcRegs = kOB * kRlMaxJ / kRlThreads;
  double zr[kZcRegs];
#pragma unroll
  for (int u = 0; u < kZcRegs; ++u) {
    const int x = tid + u * kRlThreads;
    const int t = x / Jp, r = x - t * Jp;
    zr[u] = (x < kOB * Jp && t < nb && r < J) ? Zs[(int64_t)(c0 + t) * J + r] : 0.0;
  }
  auto store_regs = [&]() {
#pragma unroll
    for (int u = 0; u < kZcRegs; ++u) {
      const int x = tid + u * kRlThreads;
      const int t = x / Jp, r = x - t * Jp;
      if (x < kOB * Jp && t < nb && r < J) Zd[(int64_t)(c0 + t) * J + r] = zr[u];
    }
  };
  if ((int64_t)R * J <= cap) {  // uniform: the copy form's result, as it is
    store_regs();
    return;
  }
  const double otol = 1e-2 * scal[0];
  int wmin, t0;
  rl_block_windows(lam, R, c0, nb, otol, sjlo, reinterpret_cast<int*>(sP), wmin, t0);
  if (wmin >= c0 + kOB) {  // uniform: no vector of the block has a window
    store_regs();
    return;
  }
#pragma unroll
  for (int u = 0; u < kZcRegs; ++u) {
    const int x = tid + u * kRlThreads;
    if (x < kOB * Jp) Zc[x] = zr[u];
  }
  __syncthreads();
  const int nst = Jp / 4;
  for (int jc = wmin; jc < c0; jc += 64) {
    const int nc = min(64, c0 - jc);
    {
      // C[jj][t] = sum_r Z[jc + jj][r] Z_c[t][r]: wave -> (16-row tile a of
      // the chunk, half ks of the reduction steps)
      const int a = wave & 3, ks = wave >> 2;
      const int s0 = nst * ks / 2, s1 = nst * (ks + 1) / 2;
      const int jj = 16 * a + il;
      const double* zr0 = Zs + (int64_t)(jc + min(jj, nc - 1)) * J;
      const bool rowok = jj < nc;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int g0 = s0; g0 < s1; g0 += 16) {
        double x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) x[u] = zr0[min(4 * (g0 + u) + q, J - 1)];  // in bounds; masked below
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int st = g0 + u;
          const double av = (rowok && st < s1) ? x[u] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Zc[il * Jp + min(4 * st + q, Jp - 1)], acc, 0, 0, 0);
        }
      }
      // D[(l >> 4) + 4v][l & 15]: chunk row 16 a + q + 4 v, block vector il
#pragma unroll
      for (int v = 0; v < 4; ++v) sP[(ks * 64 + 16 * a + q + 4 * v) * 16 + il] = acc[v];
    }
    __syncthreads();
    for (int e = tid; e < 1024; e += kRlThreads) {
      const int jj = e >> 4, t = e & 15;
      const double cv = sP[e] + sP[1024 + e];
      sC[e] = (jj < nc && t < nb && jc + jj >= sjlo[t]) ? cv : 0.0;
    }
    __syncthreads();
    // Z_c[t][r] -= sum_jj C[jj][t] Z[jc + jj][r]: wave -> 16-column tiles,
    // 16 steps of 4 chunk rows each
    for (int T = wave; T < Jp / 16; T += kRlWaves) {
      const int r = 16 * T + il;
      d4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = Zc[(q + 4 * v) * Jp + r];
      double x[16];
#pragma unroll
      for (int st = 0; st < 16; ++st) x[st] = Zs[(int64_t)(jc + min(4 * st + q, nc - 1)) * J + min(r, J - 1)];
#pragma unroll
      for (int st = 0; st < 16; ++st) {
        const int jj = 4 * st + q;
        const double bv = (jj < nc && r < J) ? x[st] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-sC[jj * 16 + il], bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) Zc[(q + 4 * v) * Jp + r] = acc[v];
    }
    __syncthreads();
  }
  if (t0 < nb) rl_block_finish(Zc, Jp, J, c0, nb, t0, sjlo, sP, sL, sRd, shs, sflag);
  for (int x = tid; x < nb * Jp; x += kRlThreads) {
    const int t = x / Jp, r = x - t * Jp;
    if (r < J) Zd[(int64_t)(c0 + t) * J + r] = Zc[x];
  }
}

// ---------------------------------------------------------------- 6. back-transformation + signs
// z <- H_0 H_1 ... H_{J-3} z, one wave per vector, four vectors per workgroup.
// The reflectors are staged through LDS in chunks of kc rows, double-buffered:
// the global loads of the next chunk are in flight (in registers) while the
// current chunk is applied, so the sequential loop reads LDS only.  Each
// reflector costs one dot product (VALU-only wave sum) and one axpy.
// cap: doubles of one chunk buffer (kc * J <= cap).
constexpr int kBackCap = 6400;

__host__ __device__ constexpr int back_rows_max(int Q) { return 32 / ((Q + 3) / 4); }
__host__ __device__ inline int back_chunk(int Q, int J, int cap) {
  const int k = cap / J;
  return k < 1 ? 1 : (k > back_rows_max(Q) ? back_rows_max(Q) : k);
}
__host__ __device__ constexpr size_t back_lds_bytes(int Q, int cap) {
  return sizeof(double) * (2 * (size_t)(cap + 64) + 2 * (size_t)back_rows_max(Q));
}

// Zt and U may be the same buffer: each wave reads its vector before it
// writes it, and no other wave touches it.
template <int Q>
__device__ __forceinline__ void back_body(const double* __restrict__ H, const double* __restrict__ tau, int J,
                                          const double* Zt, const int64_t* __restrict__ Rp, double* U, int bx,
                                          double* sh, int cap) {
  constexpr int UQ = (Q + 3) / 4;          // row entries per thread (256 threads)
  constexpr int KCM = back_rows_max(Q);    // rows per chunk, bounded by the register staging
  const int kStride = cap + 64;  // buffer stride (reads of the last row may run 63 past kc * J)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R = (int)*Rp;
  if (bx * 4 >= R || J < 1) return;  // uniform per workgroup
  const int vec = bx * 4 + wave;
  const bool active = vec < R;
  const int kc = back_chunk(Q, J, cap);
  double* stau = sh + 2 * kStride;  // [2][KCM]
  double z[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = lane + 64 * q;
    z[q] = (active && r < J) ? Zt[(int64_t)vec * J + r] : 0.0;
  }
  // chunk with first (highest) reflector hi: rows k = hi - kk, kk < kc, k >= 0;
  // row kk holds v_k (implicit 1 at k + 1, zero above)
  double stage[KCM][UQ];
  double stt = 0.0;
  // fetch() only issues the loads (the staged values are not touched until
  // put(), so the loads stay in flight while a chunk is applied); put() masks
  // on the bits (no select on a loaded value, which the compiler would turn
  // into a branch around the load) and stores every staged entry: entries
  // outside the chunk go to distinct padding slots past the data, which only
  // masked lanes ever read.
  auto fetch = [&](int hi) {
#pragma unroll
    for (int kk = 0; kk < KCM; ++kk) {
      const int kx = max(hi - kk, 0);
#pragma unroll
      for (int u = 0; u < UQ; ++u) stage[kk][u] = H[(int64_t)kx * J + min(tid + 256 * u, J - 1)];  // in bounds
    }
    stt = tau[max(hi - min(tid, kc - 1), 0)];
  };
  auto put = [&](int b, int hi) {
    double* buf = sh + b * kStride;
#pragma unroll
    for (int kk = 0; kk < KCM; ++kk) {
      const int k = hi - kk;
#pragma unroll
      for (int u = 0; u < UQ; ++u) {
        const int r = tid + 256 * u;
        const bool row = (kk < kc && k >= 0 && r < J);
        const unsigned long long keep = (row && r > k + 1) ? ~0ull : 0ull;
        const unsigned long long one = (row && r == k + 1) ? 0x3FF0000000000000ull : 0ull;
        buf[row ? kk * J + r : cap + (tid & 63)] =
            __longlong_as_double((__double_as_longlong(stage[kk][u]) & keep) | one);
      }
    }
    stau[b * KCM + min(tid, KCM - 1)] = stt;
  };
  int hi = J - 3;
  // unconditional, so that every path into the loop has waited for the loads
  // of z and of the first chunk (the loop then only waits on LDS)
  fetch(max(hi, 0));
  put(0, hi);
  __syncthreads();
  int b = 0;
  for (; hi >= 0; hi -= kc) {
    const int nhi = hi - kc;
    if (nhi >= 0) fetch(nhi);  // in flight while this chunk is applied
    if (active) {
      const double* buf = sh + b * kStride;
      const int n = min(kc, hi + 1);
      double v[Q], vn[Q];
      double tn = stau[b * KCM];
#pragma unroll
      for (int q = 0; q < Q; ++q) vn[q] = buf[lane + 64 * q];
      for (int kk = 0; kk < n; ++kk) {
        const double tk = tn;
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] = (lane + 64 * q < J) ? vn[q] : 0.0;
        if (kk + 1 < n) {  // next row, independent of z
          tn = stau[b * KCM + kk + 1];
#pragma unroll
          for (int q = 0; q < Q; ++q) vn[q] = buf[(kk + 1) * J + lane + 64 * q];
        }
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) s = fma(v[q], z[q], s);
        s = wave_sum_fast(s) * tk;
#pragma unroll
        for (int q = 0; q < Q; ++q) z[q] = fma(-s, v[q], z[q]);
      }
    }
    if (nhi >= 0) put(b ^ 1, nhi);
    __syncthreads();
    b ^= 1;
  }
  if (!active) return;
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
__global__ __launch_bounds__(256) void eig_back_kernel(const double* __restrict__ H, const double* __restrict__ tau,
                                                       int J, const double* Zt, const int64_t* __restrict__ Rp,
                                                       double* U) {
  extern __shared__ double sh[];
  back_body<Q>(H, tau, J, Zt, Rp, U, blockIdx.x, sh, kBackCap);
}

// Z: the tridiagonal eigenvectors (w.Zt, or U itself after the single-launch
// second re-orthogonalisation sweep)
template <int Q>
void launch_back(const EigWork& w, int J, const double* Z, const int64_t* R, double* U, hipStream_t s) {
  hipLaunchKernelGGL((eig_back_kernel<Q>), dim3(ceil_div(J, 4)), dim3(256), back_lds_bytes(Q, kBackCap), s, w.A,
                     w.tau, J, Z, R, U);
}

// Batched form (throughput over many small matrices): one thread per vector;
// a workgroup of 64 threads serves `nvw` vectors and keeps, per vector, the
// upper factor of the pivoted LU of (T - lambda I)/||T|| (reciprocal pivots,
// first and second superdiagonal) and the iterate in LDS, interleaved by
// thread so that accesses are bank-conflict free.  Each iteration factors and
// forward-substitutes in one pass (the multipliers and interchanges are
// applied to the right-hand side as they are produced) and back-substitutes
// in a second pass.  Only the kept vectors (typically a small fraction of
// the rows) take part, so a group serves few of them: its LDS stays small and
// many groups, each a latency-bound chain, are in flight per CU.
constexpr int kInvitBatchedRows = 512;  // vectors per group times rows: 16 KB of LDS per group
__device__ __forceinline__ void invit_body_lean(const double* __restrict__ d, const double* __restrict__ e, int J,
                                           const double* __restrict__ lam, const int64_t* __restrict__ Rp,
                                           const double* __restrict__ scal, double* __restrict__ Zt, int nvw,
                                           double* sh, int bx) {
  const int tid = threadIdx.x;
  const int t = bx * nvw + tid;
  const int R = (int)*Rp;
  if (tid >= nvw || t >= R) return;
  const double tnorm = scal[0];
  if (tnorm == 0.0) {
    for (int i = 0; i < J; ++i) Zt[(int64_t)t * J + i] = (i == t) ? 1.0 : 0.0;
    return;
  }
  const double inv = 1.0 / tnorm;
  const double eps = DBL_EPSILON;
  double* Wr = sh + 0 * (size_t)J * nvw + tid;  // 1 / u_ii
  double* W1 = sh + 1 * (size_t)J * nvw + tid;  // u_{i,i+1}
  double* W2 = sh + 2 * (size_t)J * nvw + tid;  // u_{i,i+2}
  double* Wx = sh + 3 * (size_t)J * nvw + tid;  // iterate
#define W(arr, i) arr[(size_t)(i) * nvw]
  {
    const int vec = t;
    const double shift = lam[vec] * inv;
    for (int i = 0; i < J; ++i) W(Wx, i) = hash_unit((uint32_t)i, (uint32_t)vec);
    double xscale = 1.0;
    for (int it = 0; it < 2; ++it) {
      // factor + forward substitution; the running row (dd, du) and its
      // right-hand side xc are carried in registers
      double dd = d[0] * inv - shift;
      double du = (J > 1) ? e[0] * inv : 0.0;
      double xc = W(Wx, 0) * xscale;
      for (int i = 0; i + 1 < J; ++i) {
        const double li = e[i] * inv;
        const double dn = d[i + 1] * inv - shift;
        const double un = (i + 2 < J) ? e[i + 1] * inv : 0.0;
        double xn = W(Wx, i + 1) * xscale;
        double u1, u2, ndd, ndu, rp;
        if (fabs(dd) >= fabs(li)) {
          if (fabs(dd) < eps) dd = (dd < 0.0) ? -eps : eps;
          rp = rcp_refined(dd);
          const double f = li * rp;
          u1 = du;
          u2 = 0.0;
          ndd = dn - f * du;
          ndu = un;
          xn -= f * xc;
        } else {  // interchange rows i and i+1
          rp = rcp_refined(li);
          const double f = dd * rp;
          u1 = dn;
          u2 = un;
          ndd = du - f * dn;
          ndu = -f * un;
          const double tmp = xc;
          xc = xn;
          xn = tmp - f * xn;
        }
        W(Wr, i) = rp;
        W(W1, i) = u1;
        W(W2, i) = u2;
        W(Wx, i) = xc;
        dd = ndd;
        du = ndu;
        xc = xn;
      }
      if (fabs(dd) < eps) dd = (dd < 0.0) ? -eps : eps;
      W(Wr, J - 1) = rcp_refined(dd);
      W(W1, J - 1) = 0.0;
      W(W2, J - 1) = 0.0;
      W(Wx, J - 1) = xc;
      // back substitution
      double y1 = 0.0, y2 = 0.0, nrm = 0.0;
      for (int i = J - 1; i >= 0; --i) {
        const double yi = (W(Wx, i) - W(W1, i) * y1 - W(W2, i) * y2) * W(Wr, i);
        W(Wx, i) = yi;
        nrm += yi * yi;
        y2 = y1;
        y1 = yi;
      }
      xscale = 1.0 / sqrt(nrm);
    }
    for (int i = 0; i < J; ++i) Zt[(int64_t)vec * J + i] = W(Wx, i) * xscale;
  }
#undef W
}

// One wave per vector reading the reflectors straight from global memory
// (the next one prefetched); many workgroups per CU hide the latency, and no
// LDS is used.
template <int Q>
__device__ __forceinline__ void back_body_direct(const double* __restrict__ H, const double* __restrict__ tau, int J,
                                          const double* __restrict__ Zt, const int64_t* __restrict__ Rp,
                                          double* __restrict__ U, int bx) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int vec = bx * 4 + wave;
  if (vec >= (int)*Rp) return;
  double z[Q], v[Q], vn[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = lane + 64 * q;
    z[q] = (r < J) ? Zt[(int64_t)vec * J + r] : 0.0;
  }
  auto load_v = [&](int k, double* dst) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int r = lane + 64 * q;
      dst[q] = (r == k + 1) ? 1.0 : ((r > k + 1 && r < J) ? H[(int64_t)k * J + r] : 0.0);
    }
  };
  double tn = 0.0;
  if (J >= 3) {
    load_v(J - 3, vn);
    tn = tau[J - 3];
  }
  for (int k = J - 3; k >= 0; --k) {
    const double tk = tn;
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = vn[q];
    if (k > 0) {  // prefetch the next reflector, independent of z
      load_v(k - 1, vn);
      tn = tau[k - 1];
    }
    if (tk == 0.0) continue;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) s += v[q] * z[q];
    s = wave_sum_fast(s) * tk;
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

// ---------------------------------------------------------------- batched form
// Many independent matrices of sizes J_m <= kBatchMaxJ in one launch per step:
// blockIdx.x selects the matrix, J_m is read from the device (0 = no matrix),
// and every per-matrix array sits at a fixed stride (Jmax^2 or Jmax) with the
// matrix stored contiguously (leading dimension J_m) at its start.
__device__ __forceinline__ bool batch_matrix(const EigBatch& b, int& m, int& J) {
  m = blockIdx.x;
  J = (m < b.count) ? b.J[m] : 0;
  return J > 0;
}

// Tridiagonalisation phase (hi, lo]: matrices with J_m > lo reduce the rows of
// their trailing block of size min(J_m, hi) down to lo (to the end for lo = 0).
template <int NW, int NG, int NC>
__global__ __launch_bounds__(64 * NW) void eig_tridiag_reg_batched(EigBatch b, int hi, int lo) {
  int m, J;
  if (!batch_matrix(b, m, J) || J <= lo) return;
  const int64_t o2 = (int64_t)m * b.Jmax * b.Jmax, o1 = (int64_t)m * b.Jmax;
  const int Jl = min(J, hi);
  const int k0 = J - Jl;
  const double* src = (J <= hi) ? b.S + o2 : b.A + o2;
  const int ns = lo > 0 ? Jl - lo : Jl;
  const int kt = min(k0 + ns, J - 1);  // origin of the block handed on (only written if rows remain)
  tridiag_reg_body<NW, NG, NC>(src + (int64_t)k0 * J + k0, J, Jl, ns, b.A + o2 + (int64_t)kt * J + kt, J,
                               b.A + o2 + (int64_t)k0 * J + k0, J, b.d + o1 + k0, b.e + o1 + k0, b.tau + o1 + k0);
}

// One workgroup per (matrix, group of 256 / kBisLanesBatched eigenvalues),
// the groups of a matrix consecutive: blockIdx.x = m * groups + g.
__global__ __launch_bounds__(256) void eig_bisect_batched(EigBatch b, int groups) {
  extern __shared__ double sh[];
  const int m = (int)(blockIdx.x / (unsigned)groups), g = (int)(blockIdx.x % (unsigned)groups);
  const int J = (m < b.count) ? b.J[m] : 0;
  if (J <= 0 || g * (256 / kBisLanesBatched) >= J) return;
  const int64_t o1 = (int64_t)m * b.Jmax;
  bisect_body<kBisLanesBatched>(b.d + o1, b.e + o1, J, b.lam + o1, b.scal + 8 * (int64_t)m, g);
}

__global__ void eig_truncate_batched(EigBatch b, double thr_mul) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= b.count) return;
  const int J = b.J[m];
  if (J <= 0) return;
  truncate_body(b.lam + (int64_t)m * b.Jmax, J, thr_mul, b.nx2 ? b.nx2 + m : nullptr, 0, b.R + m,
                b.disc + m);
}

__global__ __launch_bounds__(64) void eig_invit_batched(EigBatch b, int nvw) {
  extern __shared__ double sh[];
  int m, J;
  if (!batch_matrix(b, m, J)) return;
  const int64_t o2 = (int64_t)m * b.Jmax * b.Jmax, o1 = (int64_t)m * b.Jmax;
  invit_body_lean(b.d + o1, b.e + o1, J, b.lam + o1, b.R + m, b.scal + 8 * (int64_t)m, b.Zt + o2, nvw, sh,
                  blockIdx.y);
}

__global__ __launch_bounds__(kEigThreads) void eig_orth_batched(EigBatch b) {
  extern __shared__ double sh[];
  int m, J;
  if (!batch_matrix(b, m, J)) return;
  const int64_t o2 = (int64_t)m * b.Jmax * b.Jmax, o1 = (int64_t)m * b.Jmax;
  orth_body(b.Zt + o2, J, b.lam + o1, b.R + m, b.scal + 8 * (int64_t)m, sh, orth_cap_batched(b.Jmax), 0);
}

// Single matrices above 1024 rows: the register-staged LDS chunks of
// eig_back_kernel no longer fit beside a vector of Q > 16 values per lane, so
// the reflectors are read straight from global memory
// (each row k of H is read by all R vectors, from L2).
template <int Q>
__global__ __launch_bounds__(256) void eig_back_direct_kernel(const double* __restrict__ H,
                                                              const double* __restrict__ tau, int J,
                                                              const double* __restrict__ Zt,
                                                              const int64_t* __restrict__ Rp, double* __restrict__ U) {
  back_body_direct<Q>(H, tau, J, Zt, Rp, U, blockIdx.x);
}

// Batched back-transformation with one workgroup per matrix: its reflectors
// are read once into LDS, packed (v_k's entries k + 2 .. J - 1 only: at most
// 63 KB at J = 128, so that two matrices share a CU), then each of the 16
// waves applies them to every 16th vector from LDS.  Reading each reflector
// from global memory once per vector made every step of the sequence wait
// for a global load.
__host__ __device__ constexpr int back_packed_offset(int J, int k) { return k * (J - 2) - k * (k - 1) / 2; }
inline size_t back_batched_lds_bytes(int J) {
  return sizeof(double) * ((size_t)back_packed_offset(J, J - 2 > 0 ? J - 2 : 0) + (size_t)J);
}
__global__ __launch_bounds__(1024) void eig_back_batched_lds(EigBatch b) {
  extern __shared__ double sh[];
  int m, J;
  if (!batch_matrix(b, m, J)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R = (int)b.R[m];
  const int64_t o2 = (int64_t)m * b.Jmax * b.Jmax, o1 = (int64_t)m * b.Jmax;
  // sP[back_packed_offset(J, k) + r - k - 2] = v_k[r], r = k + 2 .. J - 1
  double* sP = sh;
  double* stau = sh + (J > 2 ? back_packed_offset(J, J - 2) : 0);  // [J]
  const double* H = b.A + o2;
  for (int k = wave; k + 2 < J; k += 16) {
    const int ok = back_packed_offset(J, k) - k - 2;
    for (int r = k + 2 + lane; r < J; r += 64) sP[ok + r] = H[(int64_t)k * J + r];
  }
  for (int x = tid; x < J; x += 1024) stau[x] = b.tau[o1 + x];
  __syncthreads();
  const double* Zt = b.Zt + o2;
  double* U = b.U + o2;
  for (int vec = wave; vec < R; vec += 16) {  // uniform per wave
    double z[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = lane + 64 * u;
      z[u] = (r < J) ? Zt[(int64_t)vec * J + r] : 0.0;
    }
    for (int k = J - 3; k >= 0; --k) {
      const double tk = stau[k];
      if (tk == 0.0) continue;  // uniform
      double v[2];
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int r = lane + 64 * u;
        v[u] = (r == k + 1) ? 1.0 : ((r > k + 1 && r < J) ? sP[back_packed_offset(J, k) - k - 2 + r] : 0.0);
        s = fma(v[u], z[u], s);
      }
      s = wave_sum_fast(s) * tk;
#pragma unroll
      for (int u = 0; u < 2; ++u) z[u] = fma(-s, v[u], z[u]);
    }
    // sign convention: entry of largest magnitude (lowest index on ties) positive
    double ba = -1.0, bv = 0.0;
    int bi = J;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = lane + 64 * u;
      if (r < J && fabs(z[u]) > ba) {
        ba = fabs(z[u]);
        bv = z[u];
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
    for (int u = 0; u < 2; ++u) {
      const int r = lane + 64 * u;
      if (r < J) U[(int64_t)vec * J + r] = sgn * z[u];
    }
  }
}

}  // namespace

int64_t eig_work_doubles(int64_t J) { return 2 * J * J + 3 * J + 8; }

void eig_work_carve(double* base, int64_t J, EigWork& w) {
  w.A = base;
  w.Zt = w.A + J * J;
  w.d = w.Zt + J * J;
  w.e = w.d + J;
  w.tau = w.e + J;
  w.scal = w.tau + J;
}

hipError_t launch_eig_values(const double* S, int J, double thr, const double* nx2, int fixed, const EigWork& w,
                             double* lam, int64_t* R, double* disc, hipStream_t stream) {
  {
    const double* src = S;
    int ld = J, k0 = 0;
    if (J > kRegMaxJ) {
      // steps over the whole device until the trailing block fits the registers
      hipError_t err = hipMemcpyAsync(w.A, S, sizeof(double) * (size_t)J * J, hipMemcpyDeviceToDevice, stream);
      if (err != hipSuccess) return err;
      // the eigenvector buffer is free until inverse iteration: V, P and the
      // step scalars, twice
      double* V[2] = {w.Zt, w.Zt + 3 * (size_t)J};
      double* P[2] = {w.Zt + J, w.Zt + 4 * (size_t)J};
      double* sc[2] = {w.Zt + 2 * (size_t)J, w.Zt + 5 * (size_t)J};
      const int nbig = J - kRegMaxJ;
      for (int k = 0; k < nbig; ++k) {
        const int c = k & 1, pv = c ^ 1;
        const size_t shs = sizeof(double) * 3 * (size_t)J;
#define STEP_LAUNCH(RR, NW)                                                                                   \
  hipLaunchKernelGGL((eig_tri_big_step<RR, NW>), dim3((int)ceil_div(J - k - 1, NW)), dim3(64 * NW), shs, stream, \
                     w.A, J, k, V[pv], P[pv], sc[pv], V[c], P[c], sc[c], w.d, w.e, w.tau)
        if (J <= 768) STEP_LAUNCH(12, 8);  // 8 waves: 0.25 ms less per J = 672 solve than 16
        else if (J <= 1536) STEP_LAUNCH(24, 8);
        else STEP_LAUNCH(kEigMaxJ / 64, 8);
#undef STEP_LAUNCH
        LAUNCH_OK();
      }
      {
        const int k = nbig - 1, c = k & 1;
        hipLaunchKernelGGL(eig_tri_big_update, dim3((int)ceil_div(J - k - 1, kBigRows)), dim3(kBigThreads),
                           sizeof(double) * 2 * (size_t)J, stream, w.A, J, k, V[c], P[c], sc[c], nullptr, w.e,
                           w.tau);
        LAUNCH_OK();
      }
      src = w.A;
      k0 = nbig;
    }
    // phases: each register configuration reduces until the trailing block
    // fits the next smaller one
    while (J - k0 > 2 || k0 == 0) {
      const int Jl = J - k0;
      int next;
#define TRI_LAUNCH(NW, NG, NC)                                                                                    \
  hipLaunchKernelGGL((eig_tridiag_reg_kernel<NW, NG, NC>), dim3(1), dim3(64 * NW), 0, stream, src, ld, k0, Jl, \
                     Jl - next, w.A, w.A, w.d, w.e, w.tau)
      if (Jl <= kTailRows) {
        next = 0;
        hipLaunchKernelGGL(eig_tridiag_tail_kernel, dim3(1), dim3(1024), sizeof(double) * kTailHand, stream, src, ld,
                           k0, J, w.A, w.d, w.e, w.tau);
      } else if (Jl <= 192) { next = 128; TRI_LAUNCH(8, 6, 12); }
      else { next = 192; TRI_LAUNCH(4, 13, 13); }  // Jl <= kRegMaxJ
#undef TRI_LAUNCH
      LAUNCH_OK();
      if (next == 0) break;
      src = w.A;
      k0 += Jl - next;
    }
  }
  const size_t shb = sizeof(double) * (2 * (size_t)J + 4);
  hipLaunchKernelGGL(eig_bisect_wide_kernel, dim3(J), dim3(256), shb, stream, w.d, w.e, J, lam, w.scal);
  LAUNCH_OK();
  hipLaunchKernelGGL(eig_truncate_kernel, dim3(1), dim3(64), sizeof(double) * (size_t)J, stream, lam, J, thr, nx2,
                     fixed, R, disc);
  return hipGetLastError();
}

hipError_t launch_eig_vectors(int J, const EigWork& w, const double* lam, const int64_t* R, double* U,
                              hipStream_t stream) {
  {
    const int nvw = invit_vectors_per_group(J);
    const size_t shi = sizeof(double) * kInvitArrays * (size_t)J * nvw;
    hipLaunchKernelGGL(eig_invit_kernel, dim3(ceil_div(J, nvw)), dim3(64), shi, stream, w.d, w.e, J, lam, R,
                       w.scal, w.Zt, nvw);
    LAUNCH_OK();
  }
  const bool rl = J >= kRlMinJ && J <= kRlMaxJ;
  hipLaunchKernelGGL(eig_orth_kernel, dim3(1), dim3(kEigThreads), orth_lds_bytes(J, rl), stream, w.Zt, J, lam, R,
                     w.scal, rl ? 3 : orth_blocked_mode(J));
  LAUNCH_OK();
  if (rl) {
    const int cap = (int)std::min<int64_t>((int64_t)J * J, kOrthCap);
    const int nblk = (int)ceil_div(J, kOB);
    const size_t shr = sizeof(double) * (size_t)orth_rl_doubles(J);
    for (int b = -1; b + 1 < nblk; ++b) {
      hipLaunchKernelGGL(eig_orth_rl_kernel, dim3(b < 0 ? 1 : nblk - b - 1), dim3(kRlThreads), shr, stream, w.Zt,
                         J, lam, R, w.scal, b, cap);
      LAUNCH_OK();
    }
    // second sweep into U, which the back-transformation then updates in place
    hipLaunchKernelGGL(eig_orth_rl2_kernel, dim3(nblk), dim3(kRlThreads), sizeof(double) * (size_t)orth_rl2_doubles(J),
                       stream, w.Zt, U, J, lam, R, w.scal, cap);
    LAUNCH_OK();
  }
  const double* Zv = rl ? U : w.Zt;
  const int q = (int)ceil_div(J, 64);
  if (q <= 1) launch_back<1>(w, J, Zv, R, U, stream);
  else if (q <= 2) launch_back<2>(w, J, Zv, R, U, stream);
  else if (q <= 4) launch_back<4>(w, J, Zv, R, U, stream);
  else if (q <= 8) launch_back<8>(w, J, Zv, R, U, stream);
  else if (q <= 11) launch_back<11>(w, J, Zv, R, U, stream);
  else if (q <= 16) launch_back<16>(w, J, Zv, R, U, stream);
  else if (q <= 24)
    hipLaunchKernelGGL((eig_back_direct_kernel<24>), dim3(ceil_div(J, 4)), dim3(256), 0, stream, w.A, w.tau, J,
                       w.Zt, R, U);
  else if (q <= kEigMaxJ / 64)
    hipLaunchKernelGGL((eig_back_direct_kernel<kEigMaxJ / 64>), dim3(ceil_div(J, 4)), dim3(256), 0, stream, w.A,
                       w.tau, J, w.Zt, R, U);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_eig_truncate(const double* S, int J, double thr, const double* nx2, int fixed, const EigWork& w,
                               double* lam, double* U, int64_t* R, double* disc, hipStream_t stream) {
  const hipError_t e = launch_eig_values(S, J, thr, nx2, fixed, w, lam, R, disc, stream);
  return e != hipSuccess ? e : launch_eig_vectors(J, w, lam, R, U, stream);
}

hipError_t launch_eig_truncate_batched(const EigBatch& b, double thr_mul, hipStream_t stream) {
  if (b.Jmax > kBatchMaxJ || b.count <= 0) return hipErrorInvalidValue;
  // The matrix index is blockIdx.x (up to 2^31 - 1 matrices): consecutive
  // workgroups take different matrices, which the dispatcher deals round the
  // XCDs, so the groups of a matrix that carry work (the first of a split
  // launch) spread over the whole chip instead of gathering on a few XCDs.
  // The bisection, whose groups mostly carry work, keeps a matrix's groups
  // consecutive instead (a 1-D grid, measured faster).
  const unsigned nb = (unsigned)b.count;
  // Tridiagonalisation phases, largest first (as in the single-matrix path).
  // From 96 rows down each lane holds more rows (NG) in fewer waves, so that
  // several matrices share a CU (the 96-row phase: 4 waves of 137 VGPRs,
  // 3 workgroups per CU); the 128-row phase is fastest with 16 waves.
  hipLaunchKernelGGL((eig_tridiag_reg_batched<16, 2, 8>), dim3(nb), dim3(64 * 16), 0, stream, b, 128, 96);
  hipLaunchKernelGGL((eig_tridiag_reg_batched<4, 6, 6>), dim3(nb), dim3(64 * 4), 0, stream, b, 96, 64);
  hipLaunchKernelGGL((eig_tridiag_reg_batched<4, 4, 4>), dim3(nb), dim3(64 * 4), 0, stream, b, 64, 32);
  hipLaunchKernelGGL((eig_tridiag_reg_batched<2, 4, 2>), dim3(nb), dim3(64 * 2), 0, stream, b, 32, 0);
  const int J = b.Jmax;
  const size_t shb = sizeof(double) * (2 * (size_t)J + 4);
  const int groups = (int)ceil_div(J, 256 / kBisLanesBatched);
  hipLaunchKernelGGL(eig_bisect_batched, dim3(nb * (unsigned)groups), dim3(256), shb, stream, b, groups);
  hipLaunchKernelGGL(eig_truncate_batched, dim3(ceil_div((int)nb, 64)), dim3(64), 0, stream, b, thr_mul);
  const int nvw = std::max(1, std::min(64, kInvitBatchedRows / J));
  hipLaunchKernelGGL(eig_invit_batched, dim3(nb, ceil_div(J, nvw)), dim3(64), sizeof(double) * 4 * (size_t)J * nvw,
                     stream, b, nvw);
  hipLaunchKernelGGL(eig_orth_batched, dim3(nb), dim3(kEigThreads),
                     sizeof(double) * ((size_t)J + 16 + (size_t)orth_cap_batched(J)), stream, b);
  hipLaunchKernelGGL(eig_back_batched_lds, dim3(nb), dim3(1024), back_batched_lds_bytes(J), stream, b);
  return hipGetLastError();
}

}  // namespace tk
