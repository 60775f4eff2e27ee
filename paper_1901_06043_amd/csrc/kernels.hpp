// Internal launch interfaces of the HIP kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace tk {

// ---------------------------------------------------------------- Gram
struct GramParams {
  const void* Y;
  int J;          // rows of the unfolding (size of mode n)
  uint32_t L;     // product of the sizes below mode n
  uint32_t K;     // columns of the unfolding (L * product of sizes above n)
  int ntiles;
  int npairs;
  int64_t nchunks;
  int64_t cps;    // chunks per split
  int64_t total;  // work items = nsplit * npairs
  double* part;   // nsplit * npairs * tile * tile partial tiles
  double* sq;     // nsplit * ntiles partial sums of squares (or null)
};

struct GramPlan {
  int tile;
  int ntiles;
  int npairs;
  int64_t nchunks;
  int64_t cps;
  int64_t nsplit;
  int64_t part_elems;  // doubles of partial-tile workspace
  int64_t sq_elems;    // doubles of sum-of-squares workspace
};

GramPlan plan_gram_f64(int J, uint64_t L, uint64_t K);
// `after_main` (may be null) is recorded right after the main Gram kernel.
template <typename T>
hipError_t launch_gram_f64(const T* Y, int J, uint64_t L, uint64_t K, const GramPlan& p, double* part,
                           double* sq, double* S, double* norm2, hipStream_t stream, hipEvent_t after_main);

// Mixed-precision Gram (FP32 inputs): FP32 MFMA or BF16x3 MFMA products,
// FP32 accumulation within a chunk group, FP64 across groups.
GramPlan plan_gram_mixed(int J, uint64_t L, uint64_t K);
hipError_t launch_gram_mixed(const float* Y, int J, uint64_t L, uint64_t K, int prec, const GramPlan& p,
                             double* part, double* sq, double* S, double* norm2, hipStream_t stream,
                             hipEvent_t after_main);

__global__ void sum_fixed_kernel(const double* __restrict__ x, int64_t n, double* __restrict__ out);

// ---------------------------------------------------------------- TTM
// Z_(n) = M Y_(n);  M is K x J with element (k,j) at M[k*msk + j*msj].
template <typename TI, typename TO>
hipError_t launch_ttm(const TI* Y, int J, uint64_t L, uint64_t cols, const double* M, int64_t msk, int64_t msj,
                      int K, TO* Z, hipStream_t stream);

// ---------------------------------------------------------------- eigensolver
struct EigWork {
  double* A;      // J*J   (copy of S, then Householder vectors in its rows)
  double* d;      // J
  double* e;      // J
  double* tau;    // J
  double* Zt;     // J*J   eigenvectors of the tridiagonal, column-major
  double* scal;   // 8 scalars (tnorm, ...)
};
int64_t eig_work_doubles(int64_t J);
void eig_work_carve(double* base, int64_t J, EigWork& w);
// S (J x J, device) -> lam (desc), U (J x J, first R columns), R, disc.
// Threshold: thr, or thr * (*nx2) if nx2 (device) is non-null.
hipError_t launch_eig_truncate(const double* S, int J, double thr, const double* nx2, const EigWork& w,
                               double* lam, double* U, int64_t* R, double* disc, hipStream_t stream);

}  // namespace tk
