// Gram matrix of the strided mode-n unfolding, S = Y_(n) Y_(n)^T
// (paper Alg. 2 / Sec. 5.1), without permuting the tensor.
//
// The working tensor Y (sizes J_0..J_{N-1}, natural descending, Sec. 4.1) is
// viewed for mode n as Rt row-major blocks of size J x L (Sec. 4.2):
// element (row a, column c) of the unfolding, with c = l + L*r, sits at
//     l + L*a + L*J*r          (L = prod_{k<n} J_k, Rt = prod_{k>n} J_k).
// For n = 0 (L = 1) the unfolding is one column-major J x Rt matrix.
//
// Kernel design (gfx950):
//  * The J x J output is cut into TILE x TILE tiles; only tile pairs (ta <= tb)
//    of the upper triangle are computed, and inside a diagonal tile only the
//    16x16 MFMA blocks on or above the diagonal.
//  * The K = L*Rt columns are processed in chunks of 16 staged through LDS
//    (rows x 16 columns, row stride 17 doubles so that both the coalesced
//    global->LDS stores and the MFMA operand reads are bank-conflict free).
//    Global loads walk the contiguous axis: rows for L = 1, columns otherwise.
//  * Split-K: each workgroup takes a contiguous range of chunks and writes its
//    partial tile; gram_reduce sums the partials in a fixed order
//    (deterministic FP64).  Work items of one split land on one XCD so that
//    the tile pairs sharing rows hit the same L2.
//  * FP64 path: v_mfma_f64_16x16x4f64.  The diagonal tile pairs also add up
//    the squares of the values they load (each value is loaded by exactly one
//    diagonal pair), giving ||Y||^2 in FP64 without another pass over HBM.
#include "common.hpp"
#include "kernels.hpp"

namespace tk {

namespace {

constexpr int kKC = 16;         // unfolding columns per LDS chunk
constexpr int kLds = kKC + 1;   // LDS row stride (doubles)

__device__ __forceinline__ void decode_pair(int p, int ntiles, int& ta, int& tb) {
  int t = 0;
  while (p >= ntiles - t) {
    p -= ntiles - t;
    ++t;
  }
  ta = t;
  tb = t + p;
}

template <typename T, int TILE, bool UNIT_L>
__global__ __launch_bounds__(256, 2) void gram_f64_kernel(GramParams g) {
  constexpr int E = TILE * kKC / 256;  // values per thread per tile and chunk
  constexpr int WT = TILE / 2;         // wave tile edge (2 x 2 waves)
  constexpr int NB = WT / 16;          // MFMA blocks per wave tile edge
  __shared__ double sA[TILE * kLds];
  __shared__ double sB[TILE * kLds];
  __shared__ double sred[4];

  const int64_t item = xcd_remap(blockIdx.x, gridDim.x, g.total);
  if (item < 0) return;
  const int pair = (int)(item % g.npairs);
  const int64_t split = item / g.npairs;
  int ta, tb;
  decode_pair(pair, g.ntiles, ta, tb);
  const bool diag = (ta == tb);
  const int a0 = ta * TILE, b0 = tb * TILE;
  const int J = g.J;
  const uint32_t L = g.L;
  const uint32_t K = g.K;
  const int64_t JL = (int64_t)J * L;
  const int64_t ch_begin = split * g.cps;
  const int64_t ch_end = min(ch_begin + g.cps, g.nchunks);
  const T* __restrict__ Y = static_cast<const T*>(g.Y);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  // which 16x16 blocks this wave needs (uniform per wave)
  bool need[NB][NB];
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) {
      const int gi = a0 + wr * WT + 16 * bi, gj = b0 + wc * WT + 16 * bj;
      need[bi][bj] = (gi < J) && (gj < J) && (!diag || gi <= gj);
    }

  d4 acc[NB][NB];
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[E], rb[E];
  double sq = 0.0;

  // Global loads of one chunk into registers (zero outside the tensor).
  auto load = [&](int64_t ch) {
    if constexpr (UNIT_L) {
      constexpr int STEP = 256 / TILE;
      const int row = tid % TILE, kb = tid / TILE;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t c = ch * kKC + kb + STEP * e;
        const bool cv = c < (int64_t)K;
        const int ga = a0 + row, gb = b0 + row;
        ra[e] = (cv && ga < J) ? to_f64(Y[(int64_t)ga + (int64_t)J * c]) : 0.0;
        if (!diag) rb[e] = (cv && gb < J) ? to_f64(Y[(int64_t)gb + (int64_t)J * c]) : 0.0;
      }
    } else {
      const int k = tid % kKC, rbase = tid / kKC;
      const int64_t c = ch * kKC + k;
      const bool cv = c < (int64_t)K;
      int64_t base = 0;
      if (cv) {
        const uint32_t cc = (uint32_t)c;
        const uint32_t r = cc / L, l = cc - r * L;
        base = (int64_t)l + JL * r;
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int row = rbase + 16 * e;
        const int ga = a0 + row, gb = b0 + row;
        ra[e] = (cv && ga < J) ? to_f64(Y[base + (int64_t)L * ga]) : 0.0;
        if (!diag) rb[e] = (cv && gb < J) ? to_f64(Y[base + (int64_t)L * gb]) : 0.0;
      }
    }
  };
  auto store = [&]() {
    if constexpr (UNIT_L) {
      constexpr int STEP = 256 / TILE;
      const int row = tid % TILE, kb = tid / TILE;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        sA[row * kLds + kb + STEP * e] = ra[e];
        if (!diag) sB[row * kLds + kb + STEP * e] = rb[e];
      }
    } else {
      const int k = tid % kKC, rbase = tid / kKC;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        sA[(rbase + 16 * e) * kLds + k] = ra[e];
        if (!diag) sB[(rbase + 16 * e) * kLds + k] = rb[e];
      }
    }
    if (diag) {
#pragma unroll
      for (int e = 0; e < E; ++e) sq += ra[e] * ra[e];
    }
  };

  const double* sBB = diag ? sA : sB;
  if (ch_begin < ch_end) load(ch_begin);
  for (int64_t ch = ch_begin; ch < ch_end; ++ch) {
    store();
    __syncthreads();
    if (ch + 1 < ch_end) load(ch + 1);
#pragma unroll
    for (int s = 0; s < kKC / 4; ++s) {
      double av[NB], bv[NB];
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
        av[bi] = sA[(wr * WT + 16 * bi + (lane & 15)) * kLds + 4 * s + (lane >> 4)];
#pragma unroll
      for (int bj = 0; bj < NB; ++bj)
        bv[bj] = sBB[(wc * WT + 16 * bj + (lane & 15)) * kLds + 4 * s + (lane >> 4)];
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj)
          if (need[bi][bj]) acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], bv[bj], acc[bi][bj], 0, 0, 0);
    }
    __syncthreads();
  }

  // partial tile out; f64 MFMA result layout: lane l, register v holds
  // D[(l >> 4) + 4 v][l & 15]
  double* __restrict__ P = g.part + item * (int64_t)(TILE * TILE);
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = 0; bj < NB; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * WT + 16 * bi + (lane >> 4) + 4 * v;
        const int col = wc * WT + 16 * bj + (lane & 15);
        P[row * TILE + col] = acc[bi][bj][v];
      }

  if (diag && g.sq != nullptr) {
    double w = wave_sum(sq);
    if (lane == 0) sred[wave] = w;
    __syncthreads();
    if (tid == 0) g.sq[split * g.ntiles + ta] = (sred[0] + sred[1]) + (sred[2] + sred[3]);
  }
}

// Sum the split-K partials in split order and write both triangles of S.
template <int TILE>
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ part, int npairs,
                                                          int64_t nsplit, int ntiles, int J,
                                                          double* __restrict__ S) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t per = (int64_t)TILE * TILE;
  if (idx >= per * npairs) return;
  const int pair = (int)(idx / per);
  const int rem = (int)(idx - (int64_t)pair * per);
  const int i = rem / TILE, j = rem - (rem / TILE) * TILE;
  int ta, tb;
  decode_pair(pair, ntiles, ta, tb);
  const int a = ta * TILE + i, b = tb * TILE + j;
  if (a >= J || b >= J || (ta == tb && i > j)) return;
  double s = 0.0;
  for (int64_t sp = 0; sp < nsplit; ++sp) s += part[(sp * npairs + pair) * per + rem];
  S[(int64_t)a * J + b] = s;
  S[(int64_t)b * J + a] = s;
}

// ---------------------------------------------------------------- J <= 256: whole triangle per workgroup
// One workgroup of 8 waves computes every upper-triangle 16x16 block of S for
// a contiguous range of column chunks, so each value of Y is read from HBM
// once.  The flattened block list (row-major over bi <= bj) is cut into 8
// contiguous ranges of equal size (+-1), one per wave.  LDS holds all J rows
// of a 16-column chunk, double-buffered: one barrier per chunk.
constexpr int kTriWaves = 8;
constexpr int kTriRows = 256;  // J_pad limit

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
  const int64_t ch_begin = split * g.cps;
  const int64_t ch_end = min(ch_begin + g.cps, g.nchunks);
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

  if (ch_begin < ch_end) load(ch_begin);
  for (int64_t ch = ch_begin; ch < ch_end; ++ch) {
    double* buf = sY[ch & 1];
    store(buf);
    lds_barrier();
    if (ch + 1 < ch_end) load(ch + 1);
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

// Sum the per-split partial blocks in split order; write both triangles of S.
__global__ __launch_bounds__(256) void gram_tri_reduce_kernel(const double* __restrict__ part, int nb,
                                                              int64_t nsplit, int J, double* __restrict__ S) {
  const int nblk = nb * (nb + 1) / 2;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)nblk * 256) return;
  const int q = (int)(idx >> 8), rem = (int)(idx & 255);
  int bi = 0, qq = q;
  while (qq >= nb - bi) {
    qq -= nb - bi;
    ++bi;
  }
  const int bj = bi + qq;
  const int r = rem >> 4, c = rem & 15;
  const int a = 16 * bi + r, b = 16 * bj + c;
  if (a >= J || b >= J || (bi == bj && r > c)) return;
  double s = 0.0;
  for (int64_t sp = 0; sp < nsplit; ++sp) s += part[(sp * nblk + q) * 256 + rem];
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
  p.nchunks = ceil_div((int64_t)K, kKC);
  if (J <= kTriRows) {
    // whole triangle per workgroup: split K over ~2 workgroups per CU
    p.tile = 0;
    p.ntiles = (J + 15) / 16;  // 16-row blocks
    p.npairs = p.ntiles * (p.ntiles + 1) / 2;
    int64_t nsplit = std::min<int64_t>(256, std::max<int64_t>(1, p.nchunks / 8));
    p.cps = ceil_div(p.nchunks, nsplit);
    p.nsplit = ceil_div(p.nchunks, p.cps);
    p.part_elems = p.nsplit * p.npairs * 256;
    p.sq_elems = p.nsplit;
    (void)L;
    return p;
  }
  p.tile = 128;
  p.ntiles = (int)ceil_div(J, p.tile);
  p.npairs = p.ntiles * (p.ntiles + 1) / 2;
  // enough workgroups to cover 256 CUs a few times, at least 4 chunks each
  const int64_t target = 1024;
  int64_t nsplit = ceil_div(target, p.npairs);
  nsplit = std::min<int64_t>(nsplit, std::max<int64_t>(1, p.nchunks / 4));
  nsplit = std::max<int64_t>(nsplit, 1);
  p.cps = ceil_div(p.nchunks, nsplit);
  p.nsplit = ceil_div(p.nchunks, p.cps);
  p.part_elems = p.nsplit * p.npairs * (int64_t)p.tile * p.tile;
  p.sq_elems = p.nsplit * p.ntiles;
  (void)L;
  return p;
}

template <typename T>
hipError_t launch_gram_f64(const T* Y, int J, uint64_t L, uint64_t K, const GramPlan& p, double* part,
                           double* sq, double* S, double* norm2, hipStream_t stream, hipEvent_t after_main) {
  GramParams g{};
  g.Y = Y;
  g.J = J;
  g.L = (uint32_t)L;
  g.K = (uint32_t)K;
  g.ntiles = p.ntiles;
  g.npairs = p.npairs;
  g.nchunks = p.nchunks;
  g.cps = p.cps;
  g.total = p.nsplit * p.npairs;
  g.part = part;
  g.sq = norm2 ? sq : nullptr;
  const int64_t grid = ceil_div(g.total, kXcds) * kXcds;
  const bool unit = (L == 1);
  if (p.tile == 0) {
    const int nblk = p.npairs;
    const int nbw = (int)ceil_div(nblk, kTriWaves);
#define TRI_GRAM(NBW)                                                                                        \
  do {                                                                                                       \
    if (unit) hipLaunchKernelGGL((gram_tri_kernel<T, NBW, true>), dim3(p.nsplit), dim3(64 * kTriWaves), 0, stream, g); \
    else hipLaunchKernelGGL((gram_tri_kernel<T, NBW, false>), dim3(p.nsplit), dim3(64 * kTriWaves), 0, stream, g);    \
  } while (0)
    if (nbw <= 2) TRI_GRAM(2);
    else if (nbw <= 5) TRI_GRAM(5);
    else if (nbw <= 9) TRI_GRAM(9);
    else if (nbw <= 12) TRI_GRAM(12);
    else TRI_GRAM(17);
#undef TRI_GRAM
    if (after_main) (void)hipEventRecord(after_main, stream);
    hipLaunchKernelGGL(gram_tri_reduce_kernel, dim3(ceil_div((int64_t)nblk * 256, 256)), dim3(256), 0, stream, part,
                       p.ntiles, p.nsplit, J, S);
  } else if (p.tile == 64) {
    if (unit) hipLaunchKernelGGL((gram_f64_kernel<T, 64, true>), dim3(grid), dim3(256), 0, stream, g);
    else hipLaunchKernelGGL((gram_f64_kernel<T, 64, false>), dim3(grid), dim3(256), 0, stream, g);
    if (after_main) (void)hipEventRecord(after_main, stream);
    const int64_t nel = (int64_t)p.npairs * 64 * 64;
    hipLaunchKernelGGL((gram_reduce_kernel<64>), dim3(ceil_div(nel, 256)), dim3(256), 0, stream, part,
                       p.npairs, p.nsplit, p.ntiles, J, S);
  } else {
    if (unit) hipLaunchKernelGGL((gram_f64_kernel<T, 128, true>), dim3(grid), dim3(256), 0, stream, g);
    else hipLaunchKernelGGL((gram_f64_kernel<T, 128, false>), dim3(grid), dim3(256), 0, stream, g);
    if (after_main) (void)hipEventRecord(after_main, stream);
    const int64_t nel = (int64_t)p.npairs * 128 * 128;
    hipLaunchKernelGGL((gram_reduce_kernel<128>), dim3(ceil_div(nel, 256)), dim3(256), 0, stream, part,
                       p.npairs, p.nsplit, p.ntiles, J, S);
  }
  if (norm2) hipLaunchKernelGGL(sum_fixed_kernel, dim3(1), dim3(256), 0, stream, sq, p.sq_elems, norm2);
  return hipGetLastError();
}

template hipError_t launch_gram_f64<float>(const float*, int, uint64_t, uint64_t, const GramPlan&, double*,
                                           double*, double*, double*, hipStream_t, hipEvent_t);
template hipError_t launch_gram_f64<double>(const double*, int, uint64_t, uint64_t, const GramPlan&, double*,
                                            double*, double*, double*, hipStream_t, hipEvent_t);

}  // namespace tk
