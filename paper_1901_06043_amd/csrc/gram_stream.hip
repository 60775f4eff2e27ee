// Gram matrix S = Y_(n) Y_(n)^T (Alg. 2) for small mode sizes, J <= 64.
//
// With J <= 64 the Gram has at most 4 x 4 blocks of 16 x 16 and is bound by
// reading Y once (J/b flop per byte), so the kernel streams Y straight into
// MFMA operands without LDS or barriers.  The two operands of a Gram product
// are the same matrix, so a lane's loaded values feed both A and B: lane
// (i, q) holds rows i, 16 + i, ... of its column group, and the MFMA reduction
// index is mapped to columns so that every lane reads contiguous columns:
//   FP64 / FP32 forms (16x16x4): lane (i, q) reads columns 4q .. 4q+3 of a
//     16-column group and feeds column 4q + s to step s;
//   BF16 forms (16x16x32): lane (i, q) reads columns 8q .. 8q+7 of a
//     32-column group, split in registers into bf16 pieces.
// In FP64 arithmetic, a J whose last row block holds only REM (1 or 2) rows
// (J = 33, 50, ...) computes the products with those rows on the VALU: the
// MFMA blocks would be mostly padding (for J = 33, three of six 16 x 16
// blocks for one row), and the kernel then runs at the MFMA rate rather than
// at the rate it reads Y.  Each lane fetches the REM rows' values of its
// columns from the lanes that loaded them (same lane group, lane m) and
// accumulates the dot products of its rows with them.
// Each wave walks column groups g = wave id, wave id + total waves, ..., so
// that all waves stream neighbouring addresses; vector loads are used when the
// lane's columns cannot cross a block of the unfolding (L a multiple of the
// columns per lane and Y 16-byte aligned), column loads for L = 1, scalar
// loads otherwise.  Waves accumulate the upper-triangle blocks (the reduced
// forms in FP32 over 32 columns, 256 for BF16X3, then in FP64), sum them
// through LDS in wave order, and each workgroup writes one FP64 partial per
// block; a second kernel sums the partials in a fixed order.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace tk {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kSW = 4;            // waves per workgroup
constexpr int kSNT = 64 * kSW;

struct StreamParams {
  const void* Y;
  int J;
  uint32_t L;
  uint64_t K;       // columns
  int64_t ngroups;  // column groups of G columns
  int64_t nwaves;   // total waves in the grid
  double* part;     // [workgroup][block][256]
  double* sq;       // [workgroup]
};

__device__ __forceinline__ void split_bf16(float x, __bf16& b0, __bf16& b1, __bf16& b2) {
  b0 = (__bf16)x;
  const float r1 = x - (float)b0;
  b1 = (__bf16)r1;
  b2 = (__bf16)(r1 - (float)b1);
}

// PREC: 0 FP64, 1 FP32, 2 BF16X3, 3 BF16X6.  NB: row blocks (J <= 16 NB).
// VEC: 0 scalar loads, 1 contiguous columns (L % G == 0), 2 L = 1.
// REM: 0, or (FP64 only) the rows of the last block, whose products run on
// the VALU.
template <typename T, int PREC, int NB, int VEC, int REM>
__global__ __launch_bounds__(kSNT) void gram_stream_kernel(StreamParams g) {
  static_assert(REM == 0 || (PREC == 0 && NB >= 2), "VALU rows: FP64 with a full block above");
  constexpr int G = (PREC >= 2) ? 32 : 16;  // columns per group
  constexpr int CPL = G / 4;                // columns per lane (4 or 8)
  constexpr int NBLK = NB * (NB + 1) / 2;
  constexpr int NBM = (REM > 0) ? NB - 1 : NB;  // row blocks of the MFMA products
  __shared__ double sred[NBLK * 256];
  __shared__ double ssq[kSW];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i = lane & 15, q = lane >> 4;
  const int J = g.J;
  const uint32_t L = g.L;
  const uint64_t K = g.K;
  const int64_t JL = (int64_t)J * L;
  const T* __restrict__ Y = static_cast<const T*>(g.Y);
  const int64_t wid = (int64_t)blockIdx.x * kSW + wave;

  d4 acc64[NBLK];
  f4 acc32[NBLK];
#pragma unroll
  for (int b = 0; b < NBLK; ++b) {
    acc64[b] = d4{0.0, 0.0, 0.0, 0.0};
    acc32[b] = f4{0.f, 0.f, 0.f, 0.f};
  }
  // VALU rows: racc[rb][m] = sum over this lane's columns of
  // Y[16 rb + i][c] * Y[16 (NB - 1) + m][c]
  double racc[NB][REM > 0 ? REM : 1];
#pragma unroll
  for (int rb = 0; rb < NB; ++rb)
#pragma unroll
    for (int m = 0; m < (REM > 0 ? REM : 1); ++m) racc[rb][m] = 0.0;
  double sq = 0.0;
  int since_promote = 0;

  // raw[rb][j]: row 16 rb + i, column c0 + j of a group, as loaded; the loads
  // of group grp + nwaves are issued before the products of group grp
  T raw[NB][CPL];
  auto load = [&](int64_t grp) {
    const uint64_t c0 = (uint64_t)grp * G + (uint64_t)(CPL * q);  // this lane's first column
#pragma unroll
    for (int rb = 0; rb < NB; ++rb) {
      const int row = 16 * rb + i;
      const bool rok = row < J;
      if constexpr (VEC == 1) {
        // CPL consecutive columns within one block of the unfolding
        const bool cok = rok && c0 < K;
        if (cok) {
          // 16-byte vector loads: base is a multiple of CPL and Y is 16-byte aligned
          const uint64_t r = c0 / L, l = c0 - r * L;
          const T* src = Y + ((int64_t)l + JL * (int64_t)r + (int64_t)L * row);
          if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int j = 0; j < CPL; j += 4) {
              const float4 f = *reinterpret_cast<const float4*>(src + j);
              raw[rb][j] = f.x;
              raw[rb][j + 1] = f.y;
              raw[rb][j + 2] = f.z;
              raw[rb][j + 3] = f.w;
            }
          } else {
#pragma unroll
            for (int j = 0; j < CPL; j += 2) {
              const double2 d = *reinterpret_cast<const double2*>(src + j);
              raw[rb][j] = d.x;
              raw[rb][j + 1] = d.y;
            }
          }
        } else {
#pragma unroll
          for (int j = 0; j < CPL; ++j) raw[rb][j] = (T)0;
        }
      } else if constexpr (VEC == 2) {
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const uint64_t c = c0 + j;
          raw[rb][j] = (rok && c < K) ? Y[(int64_t)row + (int64_t)J * (int64_t)c] : (T)0;
        }
      } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const uint64_t c = c0 + j;
          T x = (T)0;
          if (rok && c < K) {
            const uint64_t r = c / L, l = c - r * L;
            x = Y[(int64_t)l + JL * (int64_t)r + (int64_t)L * row];
          }
          raw[rb][j] = x;
        }
      }
    }
  };
  if (wid < g.ngroups) load(wid);
  for (int64_t grp = wid; grp < g.ngroups; grp += g.nwaves) {
    // v[rb][j]: row 16 rb + i, column c0 + j
    double v[NB][CPL];
#pragma unroll
    for (int rb = 0; rb < NB; ++rb)
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        v[rb][j] = (double)raw[rb][j];
        sq += v[rb][j] * v[rb][j];
      }
    if (grp + g.nwaves < g.ngroups) load(grp + g.nwaves);  // uniform
    if constexpr (PREC == 0) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        int b = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
          for (int bj = bi; bj < NB; ++bj, ++b)
            if (bj < NBM) acc64[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[bi][s], v[bj][s], acc64[b], 0, 0, 0);
      }
      if constexpr (REM > 0) {
#pragma unroll
        for (int m = 0; m < REM; ++m)
#pragma unroll
          for (int j = 0; j < CPL; ++j) {
            const double xm = __shfl(v[NB - 1][j], (lane & ~15) | m, 64);
#pragma unroll
            for (int rb = 0; rb < NB; ++rb) racc[rb][m] = fma(v[rb][j], xm, racc[rb][m]);
          }
      }
    } else if constexpr (PREC == 1) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        int b = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
          for (int bj = bi; bj < NB; ++bj, ++b)
            acc32[b] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)v[bi][s], (float)v[bj][s], acc32[b], 0, 0, 0);
      }
    } else {
      constexpr int PL = (PREC == 3) ? 3 : 2;
      bf8 P[NB][PL];
#pragma unroll
      for (int rb = 0; rb < NB; ++rb)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 b0, b1, b2;
          split_bf16((float)v[rb][j], b0, b1, b2);
          P[rb][0][j] = b0;
          P[rb][1][j] = b1;
          if constexpr (PL == 3) P[rb][PL - 1][j] = b2;
        }
      int b = 0;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = bi; bj < NB; ++bj, ++b) {
          f4 a = acc32[b];
          if constexpr (PREC == 3) {
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(P[bi][2], P[bj][0], a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(P[bi][0], P[bj][2], a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(P[bi][1], P[bj][1], a, 0, 0, 0);
          }
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(P[bi][1], P[bj][0], a, 0, 0, 0);
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(P[bi][0], P[bj][1], a, 0, 0, 0);
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(P[bi][0], P[bj][0], a, 0, 0, 0);
          acc32[b] = a;
        }
    }
    if constexpr (PREC != 0) {
      // FP32 accumulation over PROMOTE groups, then FP64: 32 columns for FP32
      // and BF16X6, 256 columns for BF16X3 (as in the tiled kernels)
      constexpr int PROMOTE = (PREC == 1) ? 2 : (PREC == 2 ? 8 : 1);
      if (++since_promote == PROMOTE) {
        since_promote = 0;
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[b][r] += (double)acc32[b][r];
          acc32[b] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
  }
  if constexpr (PREC != 0) {
#pragma unroll
    for (int b = 0; b < NBLK; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[b][r] += (double)acc32[b][r];
  }

  // per-wave blocks summed into LDS (16 x 16 row-major) one wave after the
  // other (fixed order).  f64 MFMA result: lane l, register r ->
  // D[(l>>4)+4r][l&15]; f32 MFMA result: lane l, register r -> D[4(l>>4)+r][l&15].
  const double wsq = wave_sum(sq);
  if (lane == 0) ssq[wave] = wsq;
  if constexpr (REM > 0) {
    // the four lane groups' sums of the VALU rows, in a fixed order
#pragma unroll
    for (int rb = 0; rb < NB; ++rb)
#pragma unroll
      for (int m = 0; m < REM; ++m) {
        const double x = racc[rb][m] + __shfl_xor(racc[rb][m], 16, 64);
        racc[rb][m] = x + __shfl_xor(x, 32, 64);
      }
  }
  for (int w = 0; w < kSW; ++w) {
    if (wave == w) {
      int b = 0;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = bi; bj < NB; ++bj, ++b) {
          if (bj < NBM) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = (PREC == 0) ? (q + 4 * r) : (4 * q + r);
              double* d = &sred[b * 256 + row * 16 + i];
              *d = (w == 0) ? acc64[b][r] : *d + acc64[b][r];
            }
          } else if (lane < 16) {
            // block (bi, NB - 1): row i, columns m < REM (the rest is never read)
#pragma unroll
            for (int m = 0; m < (REM > 0 ? REM : 1); ++m) {
              double* d = &sred[b * 256 + i * 16 + m];
              *d = (w == 0) ? racc[bi][m] : *d + racc[bi][m];
            }
          }
        }
    }
    __syncthreads();
  }
  double* __restrict__ P = g.part + (int64_t)blockIdx.x * NBLK * 256;
  for (int e = tid; e < NBLK * 256; e += kSNT) P[e] = sred[e];
  if (tid == 0 && g.sq != nullptr) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kSW; ++w) s += ssq[w];
    g.sq[blockIdx.x] = s;
  }
}

// Sum the workgroup partials in a fixed order and write both triangles.
__global__ __launch_bounds__(256) void gram_stream_reduce_kernel(const double* __restrict__ part, int nb,
                                                                 int64_t nwg, int J, double* __restrict__ S) {
  const int nblk = nb * (nb + 1) / 2;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)nblk * 256) return;
  const int qb = (int)(idx >> 8), rem = (int)(idx & 255);
  int bi = 0, qq = qb;
  while (qq >= nb - bi) {
    qq -= nb - bi;
    ++bi;
  }
  const int bj = bi + qq;
  const int r = rem >> 4, c = rem & 15;
  const int a = 16 * bi + r, b = 16 * bj + c;
  if (a >= J || b >= J || (bi == bj && r > c)) return;
  const double s = sum_strided8(part + (int64_t)qb * 256 + rem, nwg, (int64_t)nblk * 256);
  S[(int64_t)a * J + b] = s;
  S[(int64_t)b * J + a] = s;
}

template <typename T, int PREC, int NB, int REM = 0>
void launch_stream(const StreamParams& g, int vec, int64_t nwg, hipStream_t s) {
  if (vec == 1) hipLaunchKernelGGL((gram_stream_kernel<T, PREC, NB, 1, REM>), dim3(nwg), dim3(kSNT), 0, s, g);
  else if (vec == 2) hipLaunchKernelGGL((gram_stream_kernel<T, PREC, NB, 2, REM>), dim3(nwg), dim3(kSNT), 0, s, g);
  else hipLaunchKernelGGL((gram_stream_kernel<T, PREC, NB, 0, REM>), dim3(nwg), dim3(kSNT), 0, s, g);
}

template <typename T, int PREC>
void launch_stream_nb(const StreamParams& g, int nb, int vec, int64_t nwg, hipStream_t s) {
  switch (nb) {
    case 1: launch_stream<T, PREC, 1>(g, vec, nwg, s); break;
    case 2: launch_stream<T, PREC, 2>(g, vec, nwg, s); break;
    case 3: launch_stream<T, PREC, 3>(g, vec, nwg, s); break;
    default: launch_stream<T, PREC, 4>(g, vec, nwg, s); break;
  }
}

// FP64 with 1 or 2 rows in the last block (J = 17, 18, 33, 34, 49, 50)
template <typename T>
void launch_stream_rem(const StreamParams& g, int nb, int rem, int vec, int64_t nwg, hipStream_t s) {
  if (rem == 1) {
    if (nb == 2) launch_stream<T, 0, 2, 1>(g, vec, nwg, s);
    else if (nb == 3) launch_stream<T, 0, 3, 1>(g, vec, nwg, s);
    else launch_stream<T, 0, 4, 1>(g, vec, nwg, s);
  } else {
    if (nb == 2) launch_stream<T, 0, 2, 2>(g, vec, nwg, s);
    else if (nb == 3) launch_stream<T, 0, 3, 2>(g, vec, nwg, s);
    else launch_stream<T, 0, 4, 2>(g, vec, nwg, s);
  }
}

}  // namespace

GramPlan plan_gram_stream(int J, uint64_t K, int prec) {
  GramPlan p{};
  const int G = (prec >= 2) ? 32 : 16;
  p.tile = -1;
  p.ntiles = (J + 15) / 16;
  p.npairs = p.ntiles * (p.ntiles + 1) / 2;
  p.nchunks = ceil_div((int64_t)K, G);
  // about 8 waves per SIMD, each with at least 8 column groups
  const int64_t want = 2048;
  p.nsplit = std::max<int64_t>(1, std::min<int64_t>(want, ceil_div(p.nchunks, 8 * kSW)));
  p.cps = ceil_div(p.nchunks, p.nsplit * kSW);
  p.part_elems = p.nsplit * p.npairs * 256;
  p.sq_elems = p.nsplit;
  return p;
}

template <typename T>
hipError_t launch_gram_stream(const T* Y, int J, uint64_t L, uint64_t K, int prec, const GramPlan& p, double* part,
                              double* sq, double* S, double* norm2, hipStream_t stream, hipEvent_t after_main) {
  if (J > kStreamMaxJ) return hipErrorInvalidValue;
  const int G = (prec >= 2) ? 32 : 16;
  StreamParams g{};
  g.Y = Y;
  g.J = J;
  g.L = (uint32_t)L;
  g.K = K;
  g.ngroups = p.nchunks;
  g.nwaves = p.nsplit * kSW;
  g.part = part;
  g.sq = norm2 ? sq : nullptr;
  const bool aligned = (reinterpret_cast<uintptr_t>(Y) % 16) == 0;
  const int vec = (L == 1) ? 2 : ((L % (uint64_t)(G / 4) == 0 && aligned) ? 1 : 0);
  const int nb = p.ntiles;
  const int rem = J % 16;
  const bool valu_rows = prec == 0 && J > 16 && (rem == 1 || rem == 2);
  if constexpr (std::is_same<T, double>::value) {
    if (prec != 0) return hipErrorInvalidValue;
    if (valu_rows) launch_stream_rem<T>(g, nb, rem, vec, p.nsplit, stream);
    else launch_stream_nb<T, 0>(g, nb, vec, p.nsplit, stream);
  } else {
    switch (prec) {
      case 0:
        if (valu_rows) launch_stream_rem<T>(g, nb, rem, vec, p.nsplit, stream);
        else launch_stream_nb<T, 0>(g, nb, vec, p.nsplit, stream);
        break;
      case 1: launch_stream_nb<T, 1>(g, nb, vec, p.nsplit, stream); break;
      case 2: launch_stream_nb<T, 2>(g, nb, vec, p.nsplit, stream); break;
      default: launch_stream_nb<T, 3>(g, nb, vec, p.nsplit, stream); break;
    }
  }
  if (after_main) (void)hipEventRecord(after_main, stream);
  hipLaunchKernelGGL(gram_stream_reduce_kernel, dim3(ceil_div((int64_t)p.npairs * 256, 256)), dim3(256), 0, stream,
                     part, nb, p.nsplit, J, S);
  if (norm2) hipLaunchKernelGGL(sum_fixed_kernel, dim3(1), dim3(256), 0, stream, sq, p.nsplit, norm2);
  return hipGetLastError();
}

template hipError_t launch_gram_stream<float>(const float*, int, uint64_t, uint64_t, int, const GramPlan&, double*,
                                              double*, double*, double*, hipStream_t, hipEvent_t);
template hipError_t launch_gram_stream<double>(const double*, int, uint64_t, uint64_t, int, const GramPlan&, double*,
                                               double*, double*, double*, hipStream_t, hipEvent_t);

}  // namespace tk
