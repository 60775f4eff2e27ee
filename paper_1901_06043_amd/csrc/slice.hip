// Hyperslice pre/post-processing (paper Sec. 3.5) and the factor side of
// reconstruction through per-mode linear operators (paper Sec. 8).
//
// Geometry: the hyperslices of mode n are the rows a < J of the mode-n
// unfolding; element (l, a, r) of the tensor sits at l + L*a + L*J*r with
// L = prod_{k<n} J_k and r < Rt = prod_{k>n} J_k.  Every kernel here is an
// HBM-bound single pass over the tensor.
//
// Statistics take two passes (sum / extremes / norms, then the squared
// deviations from the mean).  Each pass has two mappings, chosen so that
// global loads are contiguous across a wave:
//  * row mapping (L >= 64, or a period L*J above 1024 elements): a workgroup
//    owns one slice and a range of its columns; threads walk the columns, so
//    a wave reads runs of L contiguous values;
//  * period mapping (L < 64 and L*J <= 1024): the tensor is Rt periods of
//    L*J values; a workgroup owns a range of periods and thread t always reads
//    positions t, t+256, ... of a period (fixed slices per thread), so every
//    load instruction of a wave reads 64 consecutive values.
// Partial results are written per (slice, split) and summed by a second
// kernel in a fixed order, so the statistics do not depend on scheduling.
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace tk {

namespace {

constexpr int kST = 256;
constexpr int kPeriodMax = 4 * kST;  // positions of one period held by a workgroup (4 per thread)

struct Acc {
  double sum, mn, mx, n1, n2;
};

__device__ __forceinline__ void acc_init(Acc& s) {
  s.sum = 0.0;
  s.mn = INFINITY;
  s.mx = -INFINITY;
  s.n1 = 0.0;
  s.n2 = 0.0;
}

template <int PASS>
__device__ __forceinline__ void acc_add(Acc& s, double v, double mean) {
  if constexpr (PASS == 1) {
    s.sum += v;
    s.mn = fmin(s.mn, v);
    s.mx = fmax(s.mx, v);
    s.n1 += fabs(v);
    s.n2 += v * v;
  } else {
    const double d = v - mean;
    s.sum += d * d;
  }
}

__device__ __forceinline__ void acc_merge(Acc& s, const Acc& o) {
  s.sum += o.sum;
  s.mn = fmin(s.mn, o.mn);
  s.mx = fmax(s.mx, o.mx);
  s.n1 += o.n1;
  s.n2 += o.n2;
}

// Values written per partial: 5 in pass 1 (sum, min, max, 1-norm, sum of
// squares), 1 in pass 2 (sum of squared deviations).
template <int PASS>
constexpr int kW = (PASS == 1) ? 5 : 1;

template <int PASS>
__device__ __forceinline__ void acc_store(double* p, const Acc& s) {
  p[0] = s.sum;
  if constexpr (PASS == 1) {
    p[1] = s.mn;
    p[2] = s.mx;
    p[3] = s.n1;
    p[4] = s.n2;
  }
}

// Tree reduction of one Acc per thread over the workgroup (fixed order).
template <int PASS>
__device__ __forceinline__ Acc block_reduce(Acc s, double (*sh)[kST]) {
  const int tid = threadIdx.x;
  sh[0][tid] = s.sum;
  if constexpr (PASS == 1) {
    sh[1][tid] = s.mn;
    sh[2][tid] = s.mx;
    sh[3][tid] = s.n1;
    sh[4][tid] = s.n2;
  }
  __syncthreads();
  for (int w = kST / 2; w > 0; w >>= 1) {
    if (tid < w) {
      sh[0][tid] += sh[0][tid + w];
      if constexpr (PASS == 1) {
        sh[1][tid] = fmin(sh[1][tid], sh[1][tid + w]);
        sh[2][tid] = fmax(sh[2][tid], sh[2][tid + w]);
        sh[3][tid] += sh[3][tid + w];
        sh[4][tid] += sh[4][tid + w];
      }
    }
    __syncthreads();
  }
  Acc r;
  r.sum = sh[0][0];
  if constexpr (PASS == 1) {
    r.mn = sh[1][0];
    r.mx = sh[2][0];
    r.n1 = sh[3][0];
    r.n2 = sh[4][0];
  }
  return r;
}

// Row mapping: workgroup (a, s) reduces columns [s*cper, (s+1)*cper) of
// slice a.  Column c of the unfolding is (r, l) = divmod(c, L).
template <typename T, int PASS>
__global__ __launch_bounds__(kST) void slice_rows_kernel(const T* __restrict__ Y, uint64_t L, uint64_t J,
                                                         uint64_t Rt, int64_t nsplit, uint64_t cper,
                                                         const double* __restrict__ mean,
                                                         double* __restrict__ part) {
  __shared__ double sh[kW<PASS>][kST];
  const uint64_t a = blockIdx.x / nsplit;
  const uint64_t s = blockIdx.x - a * nsplit;
  const uint64_t K = L * Rt;
  const uint64_t c0 = s * cper;
  const uint64_t c1 = (c0 + cper < K) ? c0 + cper : K;
  const double m = (PASS == 2) ? mean[a] : 0.0;
  Acc acc;
  acc_init(acc);
  uint64_t c = c0 + threadIdx.x;
  uint64_t r = c / L, l = c - r * L;
  const uint64_t dr = (L < kST) ? kST / L : 0;
  const uint64_t dl = kST - dr * L;  // < L
  const T* __restrict__ base = Y + L * a;
  const uint64_t rs = L * J;
  for (; c < c1; c += kST) {
    acc_add<PASS>(acc, (double)base[l + rs * r], m);
    l += dl;
    r += dr;
    if (l >= L) {
      l -= L;
      ++r;
    }
  }
  const Acc t = block_reduce<PASS>(acc, sh);
  if (threadIdx.x == 0) acc_store<PASS>(part + (a * nsplit + s) * kW<PASS>, t);
}

// Period mapping: workgroup w reduces periods [w*rper, (w+1)*rper); thread t
// reads positions t + 256k (k < 4) of every period, position p being
// element l = p % L of slice a = p / L.
template <typename T, int PASS>
__global__ __launch_bounds__(kST) void slice_period_kernel(const T* __restrict__ Y, uint64_t L, uint64_t J,
                                                           uint64_t Rt, uint64_t rper,
                                                           const double* __restrict__ mean,
                                                           double* __restrict__ part) {
  __shared__ double sp[kW<PASS>][kPeriodMax];
  const int tid = threadIdx.x;
  const uint64_t P = L * J;
  const uint64_t r0 = (uint64_t)blockIdx.x * rper;
  const uint64_t r1 = (r0 + rper < Rt) ? r0 + rper : Rt;
  Acc acc[4];
  double m[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    acc_init(acc[k]);
    const uint64_t p = tid + kST * k;
    m[k] = (PASS == 2 && p < P) ? mean[p / L] : 0.0;
  }
  for (uint64_t r = r0; r < r1; ++r) {
    const T* __restrict__ row = Y + r * P;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t p = tid + kST * k;
      if (p < P) acc_add<PASS>(acc[k], (double)row[p], m[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint64_t p = tid + kST * k;
    if (p < P) {
      sp[0][p] = acc[k].sum;
      if constexpr (PASS == 1) {
        sp[1][p] = acc[k].mn;
        sp[2][p] = acc[k].mx;
        sp[3][p] = acc[k].n1;
        sp[4][p] = acc[k].n2;
      }
    }
  }
  __syncthreads();
  for (uint64_t a = tid; a < J; a += kST) {
    Acc t;
    acc_init(t);
    for (uint64_t l = 0; l < L; ++l) {
      Acc o;
      acc_init(o);
      const uint64_t p = a * L + l;
      o.sum = sp[0][p];
      if constexpr (PASS == 1) {
        o.mn = sp[1][p];
        o.mx = sp[2][p];
        o.n1 = sp[3][p];
        o.n2 = sp[4][p];
      }
      acc_merge(t, o);
    }
    acc_store<PASS>(part + ((uint64_t)blockIdx.x * J + a) * kW<PASS>, t);
  }
}

// Per slice: sum the partials (stride sa between slices, ss between splits)
// in split order.  Pass 1 writes mean, min, max, 1-norm, 2-norm (and the mean
// for pass 2); pass 2 writes the standard deviation.  stats[s*J + a].
template <int PASS>
__global__ __launch_bounds__(kST) void slice_finalize_kernel(const double* __restrict__ part, uint64_t J,
                                                             int64_t nsplit, uint64_t sa, uint64_t ss, double cnt,
                                                             double* __restrict__ stats) {
  const uint64_t a = (uint64_t)blockIdx.x * kST + threadIdx.x;
  if (a >= J) return;
  Acc t;
  acc_init(t);
  for (int64_t s = 0; s < nsplit; ++s) {
    const double* p = part + a * sa + s * ss;
    Acc o;
    acc_init(o);
    o.sum = p[0];
    if constexpr (PASS == 1) {
      o.mn = p[1];
      o.mx = p[2];
      o.n1 = p[3];
      o.n2 = p[4];
    }
    acc_merge(t, o);
  }
  if constexpr (PASS == 1) {
    stats[0 * J + a] = t.sum / cnt;
    stats[2 * J + a] = t.mn;
    stats[3 * J + a] = t.mx;
    stats[4 * J + a] = t.n1;
    stats[5 * J + a] = sqrt(t.n2);
  } else {
    stats[1 * J + a] = sqrt(t.sum / cnt);
  }
}

__global__ __launch_bounds__(kST) void scaling_vectors_kernel(const double* __restrict__ stats, uint64_t J,
                                                              int method, double* __restrict__ shift,
                                                              double* __restrict__ scale) {
  const uint64_t a = (uint64_t)blockIdx.x * kST + threadIdx.x;
  if (a >= J) return;
  double sh, sc;
  if (method == 0) {  // standardization: shift by the mean, scale by the standard deviation
    sh = stats[0 * J + a];
    sc = stats[1 * J + a];
  } else {  // max rescaling
    sh = 0.0;
    sc = fmax(fabs(stats[2 * J + a]), fabs(stats[3 * J + a]));
  }
  shift[a] = sh;
  scale[a] = (sc == 0.0) ? 1.0 : sc;
}

// Power-of-two divisor per slice for the reduced-precision Gram: pscale[a] =
// 2^e with max|x| of the slice in [2^(e-1), 2^e), so that every scaled value
// x / 2^e has magnitude below 1 and the largest at least 1/2 (1 for an
// all-zero or non-finite slice).  Division by a power of two is exact.
__global__ __launch_bounds__(kST) void slice_pow2_kernel(const double* __restrict__ stats, uint64_t J,
                                                         double* __restrict__ pscale) {
  const uint64_t a = (uint64_t)blockIdx.x * kST + threadIdx.x;
  if (a >= J) return;
  const double mx = fmax(fabs(stats[2 * J + a]), fabs(stats[3 * J + a]));
  int e = 0;
  if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &e);
  pscale[a] = ldexp(1.0, e);
}

// S_ab *= pscale_a pscale_b (exact: powers of two), undoing the per-slice scaling.
__global__ __launch_bounds__(kST) void gram_unscale_kernel(double* __restrict__ S, int64_t J,
                                                           const double* __restrict__ pscale) {
  const int64_t e = (int64_t)blockIdx.x * kST + threadIdx.x;
  if (e >= J * J) return;
  const int64_t a = e / J, b = e - a * J;
  S[e] = S[e] * (pscale[a] * pscale[b]);
}

template <typename TI, typename TO, bool INV>
__device__ __forceinline__ TO affine(TI x, double sh, double sc) {
  const double v = (double)x;
  return (TO)(INV ? fma(v, sc, sh) : (v - sh) / sc);
}

// Y = (X - shift_a) / scale_a (or the inverse fma(X, scale_a, shift_a)) with
// a the slice of each element.  Threads take 4 consecutive elements per
// iteration and carry (l, a) of their first element incrementally.
// X and Y may be the same buffer (in place; each thread reads its elements
// before writing them).
template <typename TI, typename TO, bool INV>
__global__ __launch_bounds__(kST) void slice_transform_kernel(const TI* X, TO* Y,
                                                              uint64_t total, uint64_t L, uint64_t J,
                                                              const double* __restrict__ shift,
                                                              const double* __restrict__ scale) {
  const uint64_t nvec = total / 4;
  const uint64_t stride = (uint64_t)gridDim.x * kST;
  uint64_t v = (uint64_t)blockIdx.x * kST + threadIdx.x;
  uint64_t q = (4 * v) / L;
  uint64_t l = 4 * v - q * L;
  uint64_t a = q % J;
  const uint64_t S = 4 * stride;
  const uint64_t dq = S / L, dl = S - dq * L, da = dq % J;
  for (; v < nvec; v += stride) {
    TI x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = X[4 * v + j];
    uint64_t lc = l, ac = a;
    TO y[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      y[j] = affine<TI, TO, INV>(x[j], shift[ac], scale[ac]);
      if (++lc == L) {
        lc = 0;
        ac = (ac + 1 == J) ? 0 : ac + 1;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) Y[4 * v + j] = y[j];
    l += dl;
    a += da;
    if (l >= L) {
      l -= L;
      ++a;
    }
    while (a >= J) a -= J;
  }
  // the last total % 4 elements
  if (blockIdx.x == 0 && threadIdx.x < total - 4 * nvec) {
    const uint64_t e = 4 * nvec + threadIdx.x;
    const uint64_t ae = (e / L) % J;
    Y[e] = affine<TI, TO, INV>(X[e], shift[ae], scale[ae]);
  }
}

// Factor of one mode of a reconstruction: W = C^T diag(s) U (K x R, row-major,
// element (k, r) at W[k*R + r]) for U the I x R column-major factor and the
// operator kinds of tucker_op_kind; s may be null (no scaling).  One thread
// per (k, r); the sum runs over increasing row index.
__global__ __launch_bounds__(kST) void op_factor_kernel(int kind, int64_t begin, int64_t end, int64_t step,
                                                        const double* __restrict__ Ct, int64_t I, int64_t K,
                                                        int64_t R, const double* __restrict__ U,
                                                        const double* __restrict__ s, double* __restrict__ W) {
  const int64_t idx = (int64_t)blockIdx.x * kST + threadIdx.x;
  if (idx >= K * R) return;
  const int64_t k = idx / R, r = idx - k * R;
  const double* __restrict__ u = U + r * I;
  double acc = 0.0;
  switch (kind) {
    case 0:  // identity
    case 1: {  // strided selection
      const int64_t i = (kind == 0) ? k : begin + k * step;
      acc = u[i] * (s ? s[i] : 1.0);
      break;
    }
    case 2: {  // average of rows [begin + k*step, min(begin + (k+1)*step, end))
      const int64_t lo = begin + k * step;
      const int64_t hi = (lo + step < end) ? lo + step : end;
      for (int64_t i = lo; i < hi; ++i) acc += u[i] * (s ? s[i] : 1.0);
      acc /= (double)(hi - lo);
      break;
    }
    case 3:
    case 4: {  // sum / mean of rows [begin, end)
      for (int64_t i = begin; i < end; ++i) acc += u[i] * (s ? s[i] : 1.0);
      if (kind == 4) acc /= (double)(end - begin);
      break;
    }
    default: {  // dense C^T, K x I row-major
      const double* __restrict__ c = Ct + k * I;
      for (int64_t i = 0; i < I; ++i) acc += c[i] * u[i] * (s ? s[i] : 1.0);
      break;
    }
  }
  W[idx] = acc;
}

__global__ __launch_bounds__(kST) void fill_kernel(double* __restrict__ p, uint64_t n, double v) {
  const uint64_t i = (uint64_t)blockIdx.x * kST + threadIdx.x;
  if (i < n) p[i] = v;
}

// dst (sizes g.dst[0..N)) <- the leading part of src (sizes g.src[k] >=
// g.dst[k]), both natural descending.  One wave per run of dst[0]
// contiguous elements; runs r = 0 .. prod_{k>0} dst[k] - 1.
__global__ __launch_bounds__(kST) void compact_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                      CompactGeo g, int N, int64_t nruns) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kST + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kST) >> 6;
  const int64_t e0 = g.dst[0];
  for (int64_t r = wave; r < nruns; r += nwaves) {
    int64_t rem = r, off = 0, stride = g.src[0];
    for (int k = 1; k < N; ++k) {
      const int64_t i = rem % g.dst[k];
      rem /= g.dst[k];
      off += i * stride;
      stride *= g.src[k];
    }
    for (int64_t i = lane; i < e0; i += 64) dst[r * e0 + i] = src[off + i];
  }
}

// coef[e] = prod_m v_m[e_m] over the multi-index of e in sizes K_lo..K_{hi-1}
// (natural descending); vec holds the vectors one after another.
__global__ __launch_bounds__(kST) void outer_coef_kernel(const double* __restrict__ vec, OuterGeo g, int lo, int hi,
                                                         uint64_t count, double* __restrict__ coef) {
  const uint64_t e = (uint64_t)blockIdx.x * kST + threadIdx.x;
  if (e >= count) return;
  uint64_t rem = e;
  double c = 1.0;
  for (int m = lo; m < hi; ++m) {
    const uint64_t km = rem % (uint64_t)g.K[m];
    rem /= (uint64_t)g.K[m];
    c *= vec[g.voff[m] + km];
  }
  coef[e] = c;
}

// out[o*inner + i] += outer[o] * inner[i], in FP64, rounded once to TO.
template <typename TO>
__global__ __launch_bounds__(kST) void add_outer_kernel(TO* __restrict__ out, uint64_t inner, uint64_t outer,
                                                        const double* __restrict__ ci,
                                                        const double* __restrict__ co) {
  for (uint64_t o = blockIdx.y; o < outer; o += gridDim.y) {
    const double c = co[o];
    TO* __restrict__ row = out + o * inner;
    for (uint64_t i = (uint64_t)blockIdx.x * kST + threadIdx.x; i < inner; i += (uint64_t)gridDim.x * kST)
      row[i] = (TO)((double)row[i] + c * ci[i]);
  }
}

struct StatPlan {
  bool period;
  int64_t nsplit;   // row mapping: splits per slice; period mapping: workgroups
  uint64_t per;     // columns per split / periods per workgroup
};

StatPlan plan_stats(uint64_t L, uint64_t J, uint64_t Rt) {
  StatPlan p{};
  const uint64_t K = L * Rt;
  p.period = (L < 64 && L * J <= (uint64_t)kPeriodMax);
  if (p.period) {
    // at least 16 K elements per workgroup, about 2048 workgroups
    const uint64_t P = L * J;
    uint64_t per = std::max<uint64_t>(ceil_div(Rt, 2048), ceil_div(16384, P));
    p.per = std::max<uint64_t>(1, per);
    p.nsplit = (int64_t)ceil_div(Rt, p.per);
  } else {
    uint64_t ns = std::max<uint64_t>(1, ceil_div(2048, J));
    ns = std::min<uint64_t>(ns, std::max<uint64_t>(1, K / 4096));
    p.per = ceil_div(K, ns);
    p.nsplit = (int64_t)ceil_div(K, p.per);
  }
  return p;
}

template <typename T, int PASS>
void launch_pass(const T* Y, uint64_t L, uint64_t J, uint64_t Rt, const StatPlan& p, const double* mean,
                 double* part, hipStream_t s) {
  if (p.period)
    hipLaunchKernelGGL((slice_period_kernel<T, PASS>), dim3(p.nsplit), dim3(kST), 0, s, Y, L, J, Rt, p.per, mean,
                       part);
  else
    hipLaunchKernelGGL((slice_rows_kernel<T, PASS>), dim3(J * p.nsplit), dim3(kST), 0, s, Y, L, J, Rt, p.nsplit,
                       p.per, mean, part);
}

}  // namespace

int64_t slice_stats_work_doubles(uint64_t L, uint64_t J, uint64_t Rt) {
  const StatPlan p = plan_stats(L, J, Rt);
  return (int64_t)(J * p.nsplit * 5);
}

template <typename T>
hipError_t launch_slice_stats(const T* Y, uint64_t L, uint64_t J, uint64_t Rt, bool both_passes, double* work,
                              double* stats, hipStream_t s) {
  const StatPlan p = plan_stats(L, J, Rt);
  const uint64_t sa1 = p.period ? 5 : (uint64_t)p.nsplit * 5, ss1 = p.period ? J * 5 : 5;
  const uint64_t sa2 = p.period ? 1 : (uint64_t)p.nsplit, ss2 = p.period ? J : 1;
  const double cnt = (double)(L * Rt);
  const dim3 gf((unsigned)ceil_div(J, kST));
  launch_pass<T, 1>(Y, L, J, Rt, p, nullptr, work, s);
  hipLaunchKernelGGL((slice_finalize_kernel<1>), gf, dim3(kST), 0, s, work, J, p.nsplit, sa1, ss1, cnt, stats);
  if (both_passes) {
    launch_pass<T, 2>(Y, L, J, Rt, p, stats /* row 0 = mean */, work, s);
    hipLaunchKernelGGL((slice_finalize_kernel<2>), gf, dim3(kST), 0, s, work, J, p.nsplit, sa2, ss2, cnt, stats);
  }
  return hipGetLastError();
}

hipError_t launch_scaling_vectors(const double* stats, uint64_t J, int method, double* shift, double* scale,
                                  hipStream_t s) {
  hipLaunchKernelGGL(scaling_vectors_kernel, dim3((unsigned)ceil_div(J, kST)), dim3(kST), 0, s, stats, J, method,
                     shift, scale);
  return hipGetLastError();
}

hipError_t launch_slice_pow2(const double* stats, uint64_t J, double* pscale, hipStream_t s) {
  hipLaunchKernelGGL(slice_pow2_kernel, dim3((unsigned)ceil_div(J, kST)), dim3(kST), 0, s, stats, J, pscale);
  return hipGetLastError();
}

hipError_t launch_gram_unscale(double* S, int64_t J, const double* pscale, hipStream_t s) {
  hipLaunchKernelGGL(gram_unscale_kernel, dim3((unsigned)ceil_div(J * J, kST)), dim3(kST), 0, s, S, J, pscale);
  return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t launch_slice_transform(const TI* X, TO* Y, uint64_t total, uint64_t L, uint64_t J, const double* shift,
                                  const double* scale, bool inverse, hipStream_t s) {
  const uint64_t nvec = total / 4;
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(ceil_div((int64_t)nvec, kST), 8192));
  if (inverse)
    hipLaunchKernelGGL((slice_transform_kernel<TI, TO, true>), dim3(grid), dim3(kST), 0, s, X, Y, total, L, J, shift,
                       scale);
  else
    hipLaunchKernelGGL((slice_transform_kernel<TI, TO, false>), dim3(grid), dim3(kST), 0, s, X, Y, total, L, J, shift,
                       scale);
  return hipGetLastError();
}

hipError_t launch_op_factor(int kind, int64_t begin, int64_t end, int64_t step, const double* Ct, int64_t I, int64_t K,
                            int64_t R, const double* U, const double* scl, double* W, hipStream_t s) {
  hipLaunchKernelGGL(op_factor_kernel, dim3((unsigned)ceil_div(K * R, kST)), dim3(kST), 0, s, kind, begin, end, step,
                     Ct, I, K, R, U, scl, W);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, uint64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)ceil_div((int64_t)n, kST)), dim3(kST), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_compact(const double* src, double* dst, const CompactGeo& g, int N, hipStream_t s) {
  int64_t nruns = 1;
  for (int k = 1; k < N; ++k) nruns *= g.dst[k];
  if (nruns <= 0 || g.dst[0] <= 0) return hipSuccess;
  const int64_t grid = std::min<int64_t>(ceil_div(nruns, kST / 64), 8192);
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)grid), dim3(kST), 0, s, src, dst, g, N, nruns);
  return hipGetLastError();
}

hipError_t launch_outer_coef(const double* vec, const OuterGeo& g, int lo, int hi, uint64_t count, double* coef,
                             hipStream_t s) {
  hipLaunchKernelGGL(outer_coef_kernel, dim3((unsigned)ceil_div((int64_t)count, kST)), dim3(kST), 0, s, vec, g, lo, hi,
                     count, coef);
  return hipGetLastError();
}

template <typename TO>
hipError_t launch_add_outer(TO* out, uint64_t inner, uint64_t outer, const double* ci, const double* co,
                            hipStream_t s) {
  const unsigned gx = (unsigned)std::min<int64_t>(ceil_div((int64_t)inner, kST), 64);
  const unsigned gy = (unsigned)std::min<uint64_t>(outer, 65535);
  hipLaunchKernelGGL((add_outer_kernel<TO>), dim3(gx, gy), dim3(kST), 0, s, out, inner, outer, ci, co);
  return hipGetLastError();
}

template hipError_t launch_slice_stats<float>(const float*, uint64_t, uint64_t, uint64_t, bool, double*, double*,
                                              hipStream_t);
template hipError_t launch_slice_stats<double>(const double*, uint64_t, uint64_t, uint64_t, bool, double*, double*,
                                               hipStream_t);
template hipError_t launch_slice_transform<float, float>(const float*, float*, uint64_t, uint64_t, uint64_t,
                                                         const double*, const double*, bool, hipStream_t);
template hipError_t launch_slice_transform<float, double>(const float*, double*, uint64_t, uint64_t, uint64_t,
                                                          const double*, const double*, bool, hipStream_t);
template hipError_t launch_slice_transform<double, float>(const double*, float*, uint64_t, uint64_t, uint64_t,
                                                          const double*, const double*, bool, hipStream_t);
template hipError_t launch_slice_transform<double, double>(const double*, double*, uint64_t, uint64_t, uint64_t,
                                                           const double*, const double*, bool, hipStream_t);
template hipError_t launch_add_outer<float>(float*, uint64_t, uint64_t, const double*, const double*, hipStream_t);
template hipError_t launch_add_outer<double>(double*, uint64_t, uint64_t, const double*, const double*, hipStream_t);

}  // namespace tk
