// Mode-n product Z = Y x_n M, i.e. Z_(n) = M Y_(n)  (paper Sec. 2.2.3, Alg. 3),
// on the strided unfolding without permuting: with c = l + L*r,
//     Z[l + L*k + L*K*r] = sum_j M(k, j) * Y[l + L*j + L*J*r].
// ST-HOSVD uses M = U_n^T (shrinking, K = R_n <= J); reconstruction uses
// M = rows of U_n (expanding, K >= R_n).
//
// Kernel design (gfx950): each workgroup owns a 64 (k) x 64 (c) output tile;
// J is consumed in chunks of 16 staged through LDS ([c][j] and [k][j] with row
// stride 17 doubles: conflict-free stores and MFMA reads); four waves each own
// 16 columns and up to 4 row blocks of v_mfma_f64_16x16x4f64.  Global loads
// walk the contiguous axis (j for L = 1, c otherwise).  For L = 1 the output
// is staged through LDS so that stores run along k, the contiguous axis of Z.
// Row blocks beyond K are skipped, so small ranks cost proportionally less.
#include "common.hpp"
#include "kernels.hpp"

namespace tk {

namespace {

constexpr int kTC = 64;   // output columns per workgroup
constexpr int kTK = 64;   // output rows per workgroup
constexpr int kJC = 16;   // input rows (j) per chunk
constexpr int kS = kJC + 1;

template <typename T>
__device__ __forceinline__ void store_as(T* p, double v) {
  *p = static_cast<T>(v);
}

template <typename TI, typename TO, bool UNIT_L>
__global__ __launch_bounds__(256, 2) void ttm_kernel(const TI* __restrict__ Y, int J, uint32_t L, uint32_t cols,
                                                     const double* __restrict__ M, int64_t msk, int64_t msj, int K,
                                                     TO* __restrict__ Z, int nrt, int64_t total) {
  __shared__ double sY[kTC * kS];
  __shared__ double sM[kTK * kS];
  __shared__ double sZ[UNIT_L ? kTC * (kTK + 1) : 1];

  const int64_t item = xcd_remap(blockIdx.x, gridDim.x, total);
  if (item < 0) return;
  const int rt = (int)(item % nrt);
  const int64_t ct = item / nrt;
  const int64_t c0 = ct * kTC;
  const int k0 = rt * kTK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t JL = (int64_t)J * L;

  d4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = d4{0.0, 0.0, 0.0, 0.0};
  bool rneed[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) rneed[b] = (k0 + 16 * b) < K;

  // per-thread fixed column for the general (L > 1) loader
  int64_t colbase = 0;
  bool colok = false;
  if constexpr (!UNIT_L) {
    const int64_t c = c0 + (tid % kTC);
    colok = c < (int64_t)cols;
    if (colok) {
      const uint32_t cc = (uint32_t)c;
      const uint32_t r = cc / L, l = cc - r * L;
      colbase = (int64_t)l + JL * r;
    }
  }

  double ry[4], rm[4];
  auto load = [&](int j0) {
    if constexpr (UNIT_L) {
      const int j = tid % kJC, cb = tid / kJC;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t c = c0 + cb + 16 * e;
        ry[e] = (j0 + j < J && c < (int64_t)cols) ? to_f64(Y[(int64_t)(j0 + j) + (int64_t)J * c]) : 0.0;
      }
    } else {
      const int jb = tid / kTC;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = j0 + jb + 4 * e;
        ry[e] = (colok && j < J) ? to_f64(Y[colbase + (int64_t)L * j]) : 0.0;
      }
    }
    {
      const int j = tid % kJC, kb = tid / kJC;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = k0 + kb + 16 * e;
        rm[e] = (k < K && j0 + j < J) ? M[(int64_t)k * msk + (int64_t)(j0 + j) * msj] : 0.0;
      }
    }
  };
  auto store = [&]() {
    if constexpr (UNIT_L) {
      const int j = tid % kJC, cb = tid / kJC;
#pragma unroll
      for (int e = 0; e < 4; ++e) sY[(cb + 16 * e) * kS + j] = ry[e];
    } else {
      const int c = tid % kTC, jb = tid / kTC;
#pragma unroll
      for (int e = 0; e < 4; ++e) sY[c * kS + jb + 4 * e] = ry[e];
    }
    const int j = tid % kJC, kb = tid / kJC;
#pragma unroll
    for (int e = 0; e < 4; ++e) sM[(kb + 16 * e) * kS + j] = rm[e];
  };

  load(0);
  for (int j0 = 0; j0 < J; j0 += kJC) {
    store();
    __syncthreads();
    if (j0 + kJC < J) load(j0 + kJC);
#pragma unroll
    for (int s = 0; s < kJC / 4; ++s) {
      // B[j][c] = Y: lane (c = l & 15, j = l >> 4); A[k][j] = M: lane (k = l & 15, j = l >> 4)
      const double bv = sY[(16 * wave + (lane & 15)) * kS + 4 * s + (lane >> 4)];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (rneed[b]) {
          const double av = sM[(16 * b + (lane & 15)) * kS + 4 * s + (lane >> 4)];
          acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[b], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

  // f64 MFMA result: lane l, register v holds D[(l >> 4) + 4 v][l & 15]
  if constexpr (UNIT_L) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int kk = 16 * b + (lane >> 4) + 4 * v;
        const int cc = 16 * wave + (lane & 15);
        sZ[cc * (kTK + 1) + kk] = acc[b][v];
      }
    __syncthreads();
    const int kk = tid % kTK, cb = tid / kTK;
    if (k0 + kk < K) {
#pragma unroll 4
      for (int e = 0; e < kTC / 4; ++e) {
        const int cc = cb + 4 * e;
        const int64_t c = c0 + cc;
        if (c < (int64_t)cols) store_as(&Z[(int64_t)(k0 + kk) + (int64_t)K * c], sZ[cc * (kTK + 1) + kk]);
      }
    }
  } else {
    const int64_t c = c0 + 16 * wave + (lane & 15);
    if (c < (int64_t)cols) {
      const uint32_t cc = (uint32_t)c;
      const uint32_t r = cc / L, l = cc - r * L;
      const int64_t zb = (int64_t)l + (int64_t)L * K * r;
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = k0 + 16 * b + (lane >> 4) + 4 * v;
          if (k < K) store_as(&Z[zb + (int64_t)L * k], acc[b][v]);
        }
    }
  }
}

}  // namespace

template <typename TI, typename TO>
hipError_t launch_ttm(const TI* Y, int J, uint64_t L, uint64_t cols, const double* M, int64_t msk, int64_t msj,
                      int K, TO* Z, hipStream_t stream) {
  const int nrt = (int)ceil_div(K, kTK);
  const int64_t nct = ceil_div((int64_t)cols, kTC);
  const int64_t total = nct * nrt;
  const int64_t grid = ceil_div(total, kXcds) * kXcds;
  if (L == 1)
    hipLaunchKernelGGL((ttm_kernel<TI, TO, true>), dim3(grid), dim3(256), 0, stream, Y, J, (uint32_t)L,
                       (uint32_t)cols, M, msk, msj, K, Z, nrt, total);
  else
    hipLaunchKernelGGL((ttm_kernel<TI, TO, false>), dim3(grid), dim3(256), 0, stream, Y, J, (uint32_t)L,
                       (uint32_t)cols, M, msk, msj, K, Z, nrt, total);
  return hipGetLastError();
}

template hipError_t launch_ttm<double, double>(const double*, int, uint64_t, uint64_t, const double*, int64_t,
                                               int64_t, int, double*, hipStream_t);
template hipError_t launch_ttm<float, double>(const float*, int, uint64_t, uint64_t, const double*, int64_t,
                                              int64_t, int, double*, hipStream_t);
template hipError_t launch_ttm<double, float>(const double*, int, uint64_t, uint64_t, const double*, int64_t,
                                              int64_t, int, float*, hipStream_t);
template hipError_t launch_ttm<float, float>(const float*, int, uint64_t, uint64_t, const double*, int64_t,
                                             int64_t, int, float*, hipStream_t);

}  // namespace tk
