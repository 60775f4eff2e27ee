// Gram matrix of the strided mode-n unfolding, S = Y_(n) Y_(n)^T
// (paper Alg. 2 / Sec. 5.1), without permuting the tensor: FP64, J <= 240.
//
// The working tensor Y (sizes J_0..J_{N-1}, natural descending, Sec. 4.1) is
// viewed for mode n as Rt row-major blocks of size J x L (Sec. 4.2):
// element (row a, column c) of the unfolding, with c = l + L*r, sits at
//     l + L*a + L*J*r          (L = prod_{k<n} J_k, Rt = prod_{k>n} J_k).
// For n = 0 (L = 1) the unfolding is one column-major J x Rt matrix.
//
// Kernel design (gfx950): one workgroup of 16 waves computes every
// upper-triangle 16x16 block of S (v_mfma_f64_16x16x4f64) for its share of
// the column chunks, so each value of Y is read from HBM exactly once.  The
// K = L*Rt columns are processed in chunks of 16 staged through LDS (all J
// rows of a chunk, double-buffered, one barrier per chunk); global loads walk
// the contiguous axis (rows for L = 1, columns otherwise).  Split-K: split s
// takes chunks s, s + nsplit, s + 2 nsplit, ..., so that at any time the
// workgroups stream neighbouring addresses (spread over all HBM channels)
// rather than one distant range each.  The per-split FP64 partial blocks are
// summed in a fixed order (deterministic), and ||Y||^2 is accumulated in FP64
// from the same loads.  Larger J and the reduced-precision forms use the
// tile-pair kernels of gram_mixed.hip.
#include "common.hpp"
#include "kernels.hpp"

namespace tk {

namespace {

constexpr int kKC = 16;         // unfolding columns per LDS chunk
constexpr int kLds = kKC + 2;   // LDS row stride (doubles)

// ---------------------------------------------------------------- whole triangle per workgroup
// The flattened block list (row-major over bi <= bj) is cut into 16
// contiguous ranges of equal size (+-1), one per wave: four waves per SIMD,
// which hide each other's LDS and barrier waits (with 8 waves and twice the
// blocks each the kernel was 2-3% slower).
constexpr int kTriWaves = 16;
constexpr int kTriRows = 240;  // J_pad limit (kTriMaxJ)

template <typename T, int NBW, bool UNIT_L>
__global__ __launch_bounds__(64 * kTriWaves) void gram_tri_kernel(GramParams g) {
  constexpr int NT = 64 * kTriWaves;
  __shared__ double sY[2][kTriRows * kLds];
  __shared__ double sred[kTriWaves];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t split = blockIdx.x;
  const int J = g.J;
  const int Jp = (J + 15) & ~15;
  const uint32_t L = g.L, K = g.K;
  const int64_t JL = (int64_t)J * L;
  // chunks split, split + nsplit, ...: niter of them
  const int64_t nsplit = g.nsplit;
  const int64_t niter = (g.nchunks - split + nsplit - 1) / nsplit;
  const T* __restrict__ Y = static_cast<const T*>(g.Y);
  const int nb = Jp / 16, nblk = nb * (nb + 1) / 2;

  // this wave's blocks [q0, q0 + nq)
  const int q0 = (int)(((int64_t)nblk * wave) / kTriWaves);
  const int nq = (int)(((int64_t)nblk * (wave + 1)) / kTriWaves) - q0;
  int bI[NBW], bJ[NBW];
  {
    int bi = 0, bj = 0, q = 0;
    while (q < q0) {  // advance to block q0 (row-major over bi <= bj)
      ++q;
      if (++bj == nb) {
        ++bi;
        bj = bi;
      }
    }
    // slots past nq repeat the wave's last block: computed, never stored, so
    // that the MFMA loop below has no per-slot branch
#pragma unroll
    for (int t = 0; t < NBW; ++t) {
      bI[t] = bi;
      bJ[t] = bj;
      if (t + 1 < nq && ++bj == nb) {
        ++bi;
        bj = bi;
      }
    }
  }
  d4 acc[NBW];
#pragma unroll
  for (int t = 0; t < NBW; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  constexpr int E = (kTriRows * kKC + NT - 1) / NT;  // loads per thread per chunk (upper bound)
  const int nel = Jp * kKC;
  double rv[E];
  double sq = 0.0;
  // (row, column-in-chunk) of each element this thread moves (L = 1 layout)
  int erow[E], ek[E];
#pragma unroll
  for (int p = 0; p < E; ++p) {
    const int e = tid + NT * p;
    erow[p] = (e < nel) ? e % Jp : Jp;
    ek[p] = (e < nel) ? e / Jp : 0;
  }
  auto load = [&](int64_t ch) {
    if constexpr (UNIT_L) {
#pragma unroll
      for (int p = 0; p < E; ++p) {
        const int row = erow[p];
        const int64_t c = ch * kKC + ek[p];
        rv[p] = (row < J && c < (int64_t)K) ? to_f64(Y[(int64_t)row + (int64_t)J * c]) : 0.0;
      }
    } else {
      const int k = tid % kKC;
      const int64_t c = ch * kKC + k;
      const bool cv = c < (int64_t)K;
      int64_t base = 0;
      if (cv) {
        const uint32_t cc = (uint32_t)c;
        const uint32_t r = cc / L, l = cc - r * L;
        base = (int64_t)l + JL * r;
      }
#pragma unroll
      for (int p = 0; p < E; ++p) {
        const int row = tid / kKC + (NT / kKC) * p;
        rv[p] = (cv && row < J) ? to_f64(Y[base + (int64_t)L * row]) : 0.0;
      }
    }
  };
  auto store = [&](double* buf) {
    if constexpr (UNIT_L) {
#pragma unroll
      for (int p = 0; p < E; ++p) {
        if (erow[p] < Jp) buf[erow[p] * kLds + ek[p]] = rv[p];
        sq += rv[p] * rv[p];
      }
    } else {
      const int k = tid % kKC;
#pragma unroll
      for (int p = 0; p < E; ++p) {
        const int row = tid / kKC + (NT / kKC) * p;
        if (row < Jp) buf[row * kLds + k] = rv[p];
        sq += rv[p] * rv[p];
      }
    }
  };

  if (niter > 0) load(split);
  for (int64_t it = 0; it < niter; ++it) {
    double* buf = sY[it & 1];
    store(buf);
    lds_barrier();
    if (it + 1 < niter) load(split + (it + 1) * nsplit);
#pragma unroll
    for (int s = 0; s < kKC / 4; ++s) {
#pragma unroll
      for (int t = 0; t < NBW; ++t) {
        const double av = buf[(16 * bI[t] + (lane & 15)) * kLds + 4 * s + (lane >> 4)];
        const double bv = buf[(16 * bJ[t] + (lane & 15)) * kLds + 4 * s + (lane >> 4)];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);  // bound the operand reads in flight (registers)
    }
  }
  // partial blocks out: part[split][q][16 x 16]; f64 MFMA layout D[(l>>4)+4v][l&15]
  double* __restrict__ P = g.part + split * (int64_t)nblk * 256;
#pragma unroll
  for (int t = 0; t < NBW; ++t) {
    if (t < nq) {
#pragma unroll
      for (int v = 0; v < 4; ++v) P[(int64_t)(q0 + t) * 256 + ((lane >> 4) + 4 * v) * 16 + (lane & 15)] = acc[t][v];
    }
  }
  if (g.sq != nullptr) {
    const double w = wave_sum(sq);
    if (lane == 0) sred[wave] = w;
    __syncthreads();
    if (tid == 0) {
      double tot = 0.0;
      for (int w2 = 0; w2 < kTriWaves; ++w2) tot += sred[w2];
      g.sq[split] = tot;
    }
  }
}

// Sum the per-split partial blocks in a fixed order and write both triangles
// of S.  Each entry's nsplit partials are split over kRedQ threads of one
// workgroup (contiguous quarters, each summed with two interleaved
// accumulators), and the quarters are added in order through LDS.
constexpr int kRedQ = 4;

__global__ __launch_bounds__(256 * kRedQ) void gram_tri_reduce_kernel(const double* __restrict__ part, int nb,
                                                                      int64_t nsplit, int J,
                                                                      double* __restrict__ S) {
  __shared__ double sq4[kRedQ][256];
  const int nblk = nb * (nb + 1) / 2;
  const int rem = threadIdx.x & 255, qt = threadIdx.x >> 8;
  const int q = blockIdx.x;  // 16 x 16 block
  const int64_t sp0 = nsplit * qt / kRedQ, sp1 = nsplit * (qt + 1) / kRedQ;
  const double* p = part + (int64_t)q * 256 + rem;
  const int64_t stride = (int64_t)nblk * 256;
  double s0 = 0.0, s1 = 0.0;
  int64_t sp = sp0;
  for (; sp + 1 < sp1; sp += 2) {
    s0 += p[sp * stride];
    s1 += p[(sp + 1) * stride];
  }
  if (sp < sp1) s0 += p[sp * stride];
  sq4[qt][rem] = s0 + s1;
  __syncthreads();
  if (qt != 0) return;
  double s = sq4[0][rem];
#pragma unroll
  for (int t = 1; t < kRedQ; ++t) s += sq4[t][rem];
  int bi = 0, qq = q;
  while (qq >= nb - bi) {
    qq -= nb - bi;
    ++bi;
  }
  const int bj = bi + qq;
  const int r = rem >> 4, c = rem & 15;
  const int a = 16 * bi + r, b = 16 * bj + c;
  if (a >= J || b >= J || (bi == bj && r > c)) return;
  S[(int64_t)a * J + b] = s;
  S[(int64_t)b * J + a] = s;
}

}  // namespace

// Fixed-order sum of n doubles by one workgroup (deterministic).
__global__ __launch_bounds__(256) void sum_fixed_kernel(const double* __restrict__ x, int64_t n,
                                                        double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

GramPlan plan_gram_f64(int J, uint64_t L, uint64_t K) {
  GramPlan p{};
  (void)L;
  p.nchunks = ceil_div((int64_t)K, kKC);
  p.tile = 0;
  p.ntiles = (J + 15) / 16;  // 16-row blocks
  p.npairs = p.ntiles * (p.ntiles + 1) / 2;
  // about one workgroup per CU, at least 8 chunks each
  p.nsplit = std::min<int64_t>(256, std::max<int64_t>(1, p.nchunks / 8));
  p.cps = ceil_div(p.nchunks, p.nsplit);
  p.part_elems = p.nsplit * p.npairs * 256;
  p.sq_elems = p.nsplit;
  return p;
}

template <typename T>
hipError_t launch_gram_f64(const T* Y, int J, uint64_t L, uint64_t K, const GramPlan& p, double* part,
                           double* sq, double* S, double* norm2, hipStream_t stream, hipEvent_t after_main) {
  if (J > kTriMaxJ) return hipErrorInvalidValue;
  GramParams g{};
  g.Y = Y;
  g.J = J;
  g.L = (uint32_t)L;
  g.K = (uint32_t)K;
  g.ntiles = p.ntiles;
  g.npairs = p.npairs;
  g.nchunks = p.nchunks;
  g.cps = p.cps;
  g.nsplit = p.nsplit;
  g.total = p.nsplit;
  g.part = part;
  g.sq = norm2 ? sq : nullptr;
  const bool unit = (L == 1);
  const int nblk = p.npairs;
  const int nbw = (int)ceil_div(nblk, kTriWaves);
#define TRI_GRAM(NBW)                                                                                        \
  do {                                                                                                       \
    if (unit) hipLaunchKernelGGL((gram_tri_kernel<T, NBW, true>), dim3(p.nsplit), dim3(64 * kTriWaves), 0, stream, g); \
    else hipLaunchKernelGGL((gram_tri_kernel<T, NBW, false>), dim3(p.nsplit), dim3(64 * kTriWaves), 0, stream, g);    \
  } while (0)
  if (nbw <= 2) TRI_GRAM(2);
  else if (nbw <= 4) TRI_GRAM(4);
  else if (nbw <= 6) TRI_GRAM(6);
  else TRI_GRAM(8);
#undef TRI_GRAM
  if (after_main) (void)hipEventRecord(after_main, stream);
  hipLaunchKernelGGL(gram_tri_reduce_kernel, dim3(nblk), dim3(256 * kRedQ), 0, stream, part, p.ntiles, p.nsplit,
                     J, S);
  if (norm2) hipLaunchKernelGGL(sum_fixed_kernel, dim3(1), dim3(256), 0, stream, sq, p.sq_elems, norm2);
  return hipGetLastError();
}

template hipError_t launch_gram_f64<float>(const float*, int, uint64_t, uint64_t, const GramPlan&, double*,
                                           double*, double*, double*, hipStream_t, hipEvent_t);
template hipError_t launch_gram_f64<double>(const double*, int, uint64_t, uint64_t, const GramPlan&, double*,
                                            double*, double*, double*, hipStream_t, hipEvent_t);

}  // namespace tk
