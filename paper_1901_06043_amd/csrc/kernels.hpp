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
  int64_t cps;    // chunks per split (at most)
  int64_t nsplit; // splits; split s takes chunks s, s + nsplit, ...
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

// Gram for J > 128 with direct global-to-LDS staging (gram_dma.hip): float
// or double input, unit stride (L = 1) or row segments (L >= 64 or L a
// multiple of the chunk width 128 / sizeof(T)), 16-byte aligned base and
// column (L = 1) or row stride.  Partial blocks in the tile-pair layout of
// launch_gram_pair_reduce; norm2 (may be null) receives the FP64 sum of
// squares (trace(S) with FP64 products).
bool gram_dma_eligible(int J, uint64_t L, int elem_size, const void* Y);
// prec 0: FP64 products; prec 1: FP32 products, prec 3: BF16X6 products, both
// of float input with unit stride only (sq: one double per item,
// p.sq_elems).  Other combinations return hipErrorInvalidValue.
GramPlan plan_gram_dma(int J, uint64_t L, uint64_t K, int elem_size, int prec);
template <typename T>
hipError_t launch_gram_dma(const T* Y, int J, uint64_t L, uint64_t K, int prec, const GramPlan& p, double* part,
                           double* sq, double* S, double* norm2, hipStream_t stream, hipEvent_t after_main);
// Sums the partial 128 x 128 tile-pair blocks of nsplit splits into S (both
// triangles), in a fixed order.
void launch_gram_pair_reduce(const double* part, int ntiles, int npairs, int64_t nsplit, int J, double* S,
                             hipStream_t stream);

// FP64 Gram with the whole triangle per workgroup, J <= kTriMaxJ.
constexpr int kTriMaxJ = 240;
GramPlan plan_gram_f64(int J, uint64_t L, uint64_t K);
// `after_main` (may be null) is recorded right after the main Gram kernel.
template <typename T>
hipError_t launch_gram_f64(const T* Y, int J, uint64_t L, uint64_t K, const GramPlan& p, double* part,
                           double* sq, double* S, double* norm2, hipStream_t stream, hipEvent_t after_main);

// Gram in one of four arithmetic forms (0 FP64, 1 FP32 MFMA, 2 BF16x3,
// 3 BF16x6), FP32 accumulation within a chunk group and FP64 across groups
// for the reduced forms.  Handles any J (triangle mode J <= 128, 128-row tile
// pairs above).  T = float or double input.
GramPlan plan_gram_mp(int J, uint64_t K, int prec);
template <typename T>
hipError_t launch_gram_mp(const T* Y, int J, uint64_t L, uint64_t K, int prec, const GramPlan& p, double* part,
                          double* sq, double* S, double* norm2, hipStream_t stream, hipEvent_t after_main);

// Streaming Gram for J <= kStreamMaxJ (HBM-bound small modes): no LDS, the
// loaded values feed both MFMA operands; any arithmetic form.
constexpr int kStreamMaxJ = 64;
GramPlan plan_gram_stream(int J, uint64_t K, int prec);
template <typename T>
hipError_t launch_gram_stream(const T* Y, int J, uint64_t L, uint64_t K, int prec, const GramPlan& p, double* part,
                              double* sq, double* S, double* norm2, hipStream_t stream, hipEvent_t after_main);

// Range guard of a reduced-precision Gram over K columns (one workgroup): if
// S has a non-finite entry, |trace(S) - *sq| > 1e-3 *sq, or (K > 0) a diagonal
// entry with S_aa / K outside [2^-100, 2^100] (squares near the FP32
// underflow or overflow range, or an all-zero row, which cannot be told apart
// from one; K = 0 skips this check, for a Gram computed on scaled slices),
// zero S and set *flag = 1, else *flag = 0.
hipError_t launch_gram_guard(double* S, int J, double K, const double* sq, double* flag, hipStream_t stream);

__global__ void sum_fixed_kernel(const double* __restrict__ x, int64_t n, double* __restrict__ out);

// ---------------------------------------------------------------- TTM
// Z_(n) = M Y_(n);  M is K x J with element (k,j) at M[k*msk + j*msj].
// fp32_products: FP32 MFMA products (M and Y rounded to FP32), else FP64.
// FP64 mode product for more than 64 output rows with direct global-to-LDS
// staging (ttm_dma.hip): M with contiguous rows (msj = 1) or columns
// (msk = 1) and even stride, 16-byte aligned M and Y; L = 1 needs double Y
// and even J, L > 1 needs L a multiple of 16 / sizeof(TI); float Y only with
// contiguous rows of M and double output.  launch_ttm uses it when eligible.
bool ttm_dma_eligible(int J, uint64_t L, uint64_t cols, int K, int64_t msk, int64_t msj, int ysize, int zsize,
                      const void* Y, const void* M);
// Output of a mode product (L > 1) whose L covers a mode p of extent Pp on
// input and Rp on output: l = a + Lp (i_p + Pp h) on input is written to
// a + Lp (i_p + Rp h).  Rp < Pp drops the zero slices i_p >= Rp of a padded
// mode (from zero columns of that mode's factor), so that the output is the
// compact tensor; Rp = Pp + 1 appends a zero slice i_p = Pp (written with the
// slice before it), so that a later product over mode p meets an even
// extent.  Pp == Rp: no remap.
struct TtmOutRemap {
  int64_t Lp = 1, Pp = 1, Rp = 1;
};
template <typename TY, typename TZ>
hipError_t launch_ttm_dma(const TY* Y, int J, uint64_t L, uint64_t cols, const double* M, int64_t msk, int64_t msj,
                          int K, TZ* Z, hipStream_t stream, const TtmOutRemap& rm = TtmOutRemap{});
template <typename TI, typename TO>
hipError_t launch_ttm(const TI* Y, int J, uint64_t L, uint64_t cols, const double* M, int64_t msk, int64_t msj,
                      int K, TO* Z, bool fp32_products, hipStream_t stream);

// ---------------------------------------------------------------- eigensolver
// Largest matrix of the single-matrix eigensolver: the back-transformation
// holds a vector as J / 64 doubles per lane next to two reflectors (3 x 36
// doubles at 2304), and inverse iteration keeps seven arrays of J doubles of
// one vector in the 160 KB of LDS of a workgroup.
constexpr int kEigMaxJ = 2304;
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
// Threshold: thr, or thr * (*nx2) if nx2 (device) is non-null; fixed > 0
// takes R = min(fixed, J) instead of the threshold rule.
hipError_t launch_eig_truncate(const double* S, int J, double thr, const double* nx2, int fixed, const EigWork& w,
                               double* lam, double* U, int64_t* R, double* disc, hipStream_t stream);
// The same in two parts, so that R can be read back while the eigenvectors
// are being formed: the eigenvalues and the truncation (lam, R, disc; steps
// 1-3), then the leading R eigenvectors (U; steps 4-6), which only read w,
// lam and R.
hipError_t launch_eig_values(const double* S, int J, double thr, const double* nx2, int fixed, const EigWork& w,
                             double* lam, int64_t* R, double* disc, hipStream_t stream);
hipError_t launch_eig_vectors(int J, const EigWork& w, const double* lam, const int64_t* R, double* U,
                              hipStream_t stream);

// ---------------------------------------------------------------- batched form
// `count` independent matrices; matrix m has size J[m] (device; 0 = none),
// J[m] <= Jmax <= kBatchMaxJ, and occupies the first J[m]^2 (resp. J[m])
// entries of its slot of Jmax^2 (resp. Jmax) doubles in every array below.
constexpr int kBatchMaxJ = 128;
struct EigBatch {
  int count;
  int Jmax;
  const int* J;
  const double* S;  // Gram matrices
  double* A;        // workspace / Householder vectors
  double* Zt;       // eigenvectors of the tridiagonal matrices
  double* d;
  double* e;
  double* tau;
  double* lam;      // eigenvalues, descending
  double* scal;     // 8 per matrix
  double* U;        // leading eigenvectors, column-major J[m] x R[m]
  int64_t* R;       // ranks
  double* disc;     // discarded energies
  const double* nx2;  // per matrix: threshold multiplier source (||X_m||^2), or null
};
hipError_t launch_eig_truncate_batched(const EigBatch& b, double thr_mul, hipStream_t stream);

// Batched Gram of mode n (J[t] <= 128 for every tensor t).  items: 4 int64
// per work item (tensor, first chunk, end chunk, offset of its partial blocks
// in `part`, in doubles), contiguous per tensor (items ifirst[2t] ..
// ifirst[2t+1] - 1) and ordered so that items [0, nsmall) have J <= 80.  Chunks are 32 columns for
// the reduced forms and 16 for FP64.  S: count x Jmax^2 (matrix t stored
// contiguously, J[t] x J[t]); nx2 (may be null): per-tensor sum of squares.
struct GramBatch {
  int count, N, n, Jmax;
  const void* const* Y;
  const int64_t* cur;
  const int* J;
  const int64_t* items;
  int nitems, nsmall;
  const int* ifirst;
  double* part;
  double* sq;  // per item (needed when nx2 is set)
  double* S;
  double* nx2;
  // recomputation of flagged Grams: only tensors t with flag[t] != 0 are
  // processed (null: all), and the items' chunk ranges are in units of
  // chunk_mul chunks of this arithmetic (a plan made for 32-column chunks
  // run with FP64's 16-column chunks has chunk_mul = 2)
  const int* flag;
  int chunk_mul;
};
template <typename T>
hipError_t launch_gram_batched(const GramBatch& b, int prec, bool unit_l, hipStream_t stream);
// Batched range guard of reduced Grams: for tensor t (J[t], K[t] columns from
// the current sizes), flag[t] = 1 and S_t zeroed under the conditions of
// launch_gram_guard (sq: per-tensor FP64 sums of squares), else 0; status[t]
// accumulates 1 for a non-finite sum of squares and 2 for a flagged Gram.
hipError_t launch_gram_guard_batched(const GramBatch& b, int* flag, int* status, hipStream_t stream);

// Batched mode-n product Z_t = Y_t x_n U_t^T with K = R[t] output rows.
// items: 3 int64 per work item (tensor, first column tile, end column tile),
// tiles of 64 columns.  U: count x Jmax^2 (U_t column-major J[t] x R[t]).
struct TtmBatch {
  int count, N, n, Jmax;
  const void* const* Y;
  void* const* Z;
  const int64_t* cur;
  const int* J;
  const int64_t* R;
  const double* U;
  const int64_t* items;
  int nitems;
};
template <typename TI, typename TO>
hipError_t launch_ttm_batched(const TtmBatch& b, bool fp32_products, bool unit_l, hipStream_t stream);

// ---------------------------------------------------------------- hyperslices (slice.hip)
// Statistics of the J slices of mode n (geometry L, J, Rt): stats[s*J + a]
// for s = mean, std, min, max, 1-norm, 2-norm; the standard deviation (second
// pass) only if both_passes.  work: slice_stats_work_doubles doubles.
int64_t slice_stats_work_doubles(uint64_t L, uint64_t J, uint64_t Rt);
template <typename T>
hipError_t launch_slice_stats(const T* Y, uint64_t L, uint64_t J, uint64_t Rt, bool both_passes, double* work,
                              double* stats, hipStream_t s);
// shift/scale from stats: method 0 standardization, 1 max rescaling (a zero scale becomes 1).
hipError_t launch_scaling_vectors(const double* stats, uint64_t J, int method, double* shift, double* scale,
                                  hipStream_t s);
// pscale[a] = 2^e with max|x| of slice a in [2^(e-1), 2^e) (from the min/max rows of stats).
hipError_t launch_slice_pow2(const double* stats, uint64_t J, double* pscale, hipStream_t s);
// S_ab *= pscale_a * pscale_b (J x J).
hipError_t launch_gram_unscale(double* S, int64_t J, const double* pscale, hipStream_t s);
// Y = (X - shift_a) / scale_a, or fma(X, scale_a, shift_a) if inverse; X == Y allowed.
template <typename TI, typename TO>
hipError_t launch_slice_transform(const TI* X, TO* Y, uint64_t total, uint64_t L, uint64_t J, const double* shift,
                                  const double* scale, bool inverse, hipStream_t s);
// W = C^T diag(scl) U (K x R row-major) for a reconstruction operator (kind as
// tucker_op_kind; Ct the dense K x I operator for kind 5); scl may be null.
hipError_t launch_op_factor(int kind, int64_t begin, int64_t end, int64_t step, const double* Ct, int64_t I, int64_t K,
                            int64_t R, const double* U, const double* scl, double* W, hipStream_t s);
hipError_t launch_fill(double* p, uint64_t n, double v, hipStream_t s);
// coef[e] = prod_{m in [lo,hi)} vec[voff[m] + e_m] over the natural-descending
// multi-index e of sizes K[lo..hi).
// Copy of the leading dst[0..N) part of a tensor of sizes src[0..N) (natural
// descending), e.g. a core whose working extents were padded.
struct CompactGeo {
  int64_t src[16];
  int64_t dst[16];
};
hipError_t launch_compact(const double* src, double* dst, const CompactGeo& g, int N, hipStream_t s);
struct OuterGeo {
  int64_t K[16];
  int64_t voff[16];
};
hipError_t launch_outer_coef(const double* vec, const OuterGeo& g, int lo, int hi, uint64_t count, double* coef,
                             hipStream_t s);
// out[o*inner + i] += co[o] * ci[i].
template <typename TO>
hipError_t launch_add_outer(TO* out, uint64_t inner, uint64_t outer, const double* ci, const double* co,
                            hipStream_t s);

}  // namespace tk
