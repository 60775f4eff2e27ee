// Mode-n product Z = Y x_n M, i.e. Z_(n) = M Y_(n)  (paper Sec. 2.2.3, Alg. 3),
// on the strided unfolding without permuting: with c = l + L*r,
//     Z[l + L*k + L*K*r] = sum_j M(k, j) * Y[l + L*j + L*J*r].
// ST-HOSVD uses M = U_n^T (shrinking, K = R_n <= J); reconstruction uses
// M = rows of U_n (expanding, K >= R_n).
//
// Kernel design (gfx950): the shrinking TTM is bound by reading Y once from
// HBM, so Y is not staged through LDS.  Each wave owns 16 output columns and
// up to 4 blocks of 16 output rows (v_mfma_f64_16x16x4f64, or
// v_mfma_f32_16x16x4f32 for the reduced-precision path, which has the same
// operand layout) and loads its MFMA B operands straight from global memory.  Since the reduction index of an
// MFMA may be assigned to (step, lane group) in any order, it is chosen so
// that loads run along the contiguous axis:
//   L = 1 (columns contiguous along j): lane group q of step s reads row
//         16 t + 4 q + s, so each lane reads 4 consecutive values of its column;
//   L > 1 (rows contiguous along c):    lane group q of step s reads row
//         16 t + 4 s + q, so the 16 lanes of a group read 16 consecutive columns.
// The A operand (M, small) is staged through LDS in 64 x 64 blocks shared by
// the workgroup's four waves and follows the same assignment.  Four 16-row
// chunks of Y are loaded before they are consumed, keeping enough bytes in
// flight per CU.

#include "common.hpp"
#include "kernels.hpp"

namespace tk {

namespace {

constexpr int kTK = 64;     // output rows per wave (4 MFMA blocks)
constexpr int kWaves = 4;   // waves per workgroup of the batched form; each owns 16 CG columns
// waves per workgroup of the single-tensor tiled kernel: the M block staged in
// LDS (33.8 KB in FP64) then serves 128 columns, which doubles the waves per
// CU that the LDS allows (the kernel waits on memory, so occupancy pays:
// 10-19% faster than 4 waves on the 672x672x33x626 mode products)
constexpr int kTileWaves = 8;
// column groups of 16 per wave in ttm_kernel: two with FP32 products and
// L = 1, else one (FP64 accumulators and operands would halve the occupancy,
// and L > 1 measured slower with two); the batched form uses one
template <typename CT, bool UNIT_L>
constexpr int tile_cg() {
  return (sizeof(CT) == 4 && UNIT_L) ? 2 : 1;
}
constexpr int kJB = 64;     // reduction rows per LDS block of M (4 chunks of 16)
// LDS layout of M blocks (row-major, padded rows).  Lane (i, q) reads the
// A operands of its 4 MFMA steps, reduction rows 16 t + 4 q + s (s < 4), as
// one vector of 4 consecutive values.  The row stride is 4 modulo 64 floats
// (2 modulo 32 doubles), so that the 16 lanes i of a vector read cover 64
// distinct banks.
template <typename CT>
struct MLds {
  static constexpr bool kF32 = sizeof(CT) == 4;
  static constexpr int S = kF32 ? kJB + 4 : kJB + 2;  // tile kernel (kJB columns)
  // resident kernel: jp (a multiple of 16) columns
  static __host__ __device__ __forceinline__ int ld(int jp) {
    return kF32 ? ((jp + 63) & ~63) + 4 : ((jp + 31) & ~31) + 2;
  }
  // the 4 values at p (16-byte aligned)
  static __device__ __forceinline__ void read4(const CT* p, CT (&a)[4]) {
    if constexpr (kF32) {
      const float4 v = *reinterpret_cast<const float4*>(p);
      a[0] = v.x;
      a[1] = v.y;
      a[2] = v.z;
      a[3] = v.w;
    } else {
      const double2 u = *reinterpret_cast<const double2*>(p);
      const double2 w = *reinterpret_cast<const double2*>(p + 2);
      a[0] = u.x;
      a[1] = u.y;
      a[2] = w.x;
      a[3] = w.y;
    }
  }
};

template <typename T>
__device__ __forceinline__ void store_as(T* p, double v) {
  *p = static_cast<T>(v);
}

template <typename CT>
struct Acc;
template <>
struct Acc<double> {
  using type = d4;
  static __device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // result layout: lane l, register v holds D[(l >> 4) + 4 v][l & 15]
  static __device__ __forceinline__ int row(int q, int v) { return q + 4 * v; }
};
template <>
struct Acc<float> {
  using type = f4;
  static __device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // result layout: lane l, register v holds D[4 (l >> 4) + v][l & 15]
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
};

// Raw operand data of one 16-row block for one lane: 4 reduction rows of its
// column.  VW = 4 (L = 1, J % 4 == 0, Y 16-byte aligned): the 4 consecutive
// rows are one 16-byte load (two for doubles); VW = 2 (L = 1, J even): two
// loads of a pair of rows each.
template <typename TI>
struct Raw4 {
  TI v[4];
};

// Issues the loads of block jb without any condition: the row and column are
// clamped into the tensor, and use4() masks what lies outside.  (A load under
// a condition, or converted right after it, would have to complete at once.)
template <typename TI, bool UNIT_L, int VW>
__device__ __forceinline__ void issue4(const TI* __restrict__ Y, int64_t cbase, int J, uint32_t L, int jb, int q,
                                       Raw4<TI>& r) {
  if constexpr (VW == 4) {
    const int j = min(16 * jb + 4 * q, J - 4);
    const TI* src = Y + cbase + j;
    if constexpr (sizeof(TI) == 4) {
      const float4 f = *reinterpret_cast<const float4*>(src);
      r.v[0] = f.x;
      r.v[1] = f.y;
      r.v[2] = f.z;
      r.v[3] = f.w;
    } else {
      const double2 a = *reinterpret_cast<const double2*>(src);
      const double2 b = *reinterpret_cast<const double2*>(src + 2);
      r.v[0] = a.x;
      r.v[1] = a.y;
      r.v[2] = b.x;
      r.v[3] = b.y;
    }
  } else if constexpr (VW == 2) {
    // two pairs of rows, each clamped on its own (J even: a pair never straddles J)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const TI* src = Y + cbase + min(16 * jb + 4 * q + 2 * h, J - 2);
      if constexpr (sizeof(TI) == 4) {
        const float2 f = *reinterpret_cast<const float2*>(src);
        r.v[2 * h] = f.x;
        r.v[2 * h + 1] = f.y;
      } else {
        const double2 f = *reinterpret_cast<const double2*>(src);
        r.v[2 * h] = f.x;
        r.v[2 * h + 1] = f.y;
      }
    }
  } else {
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int j = min(16 * jb + 4 * q + s2, J - 1);
      r.v[s2] = Y[cbase + (UNIT_L ? (int64_t)j : (int64_t)L * j)];
    }
  }
}

// Vector width of the Y loads for L = 1: 4 rows per 16-byte access (two for
// doubles) when J % 4 == 0, pairs of rows when J is even, else single rows;
// Y must be aligned to the access.
template <typename TI>
int y_vector_width(const TI* Y, int J, uint64_t L) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(Y);
  if (L != 1) return 1;
  if (J % 4 == 0 && a % 16 == 0) return 4;
  if (J % 2 == 0 && a % (2 * sizeof(TI)) == 0) return 2;
  return 1;
}

// Converts block jb's raw data to the product type, zero outside the tensor.
template <typename TI, typename CT, bool UNIT_L>
__device__ __forceinline__ void use4(const Raw4<TI>& r, bool cok, int J, int jb, int q, CT (&y)[4]) {
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2) {
    const int j = 16 * jb + 4 * q + s2;
    const CT x = (CT)r.v[s2];
    y[s2] = (cok && j < J) ? x : (CT)0;
  }
}

// CT: arithmetic type of the products (double: FP64 MFMA; float: FP32 MFMA).
// RB: 16-row output blocks per wave (1..4), chosen from K at launch.
// VW: vector width of the Y loads (as in issue4).
// CG: column groups of 16 per wave; the A operand read from LDS serves all
// of them, and the M block staged per workgroup is shared by 64 CG columns.
// NW: waves per workgroup.  One workgroup tile: output rows
// [64 rt, 64 rt + 16 RB) and columns [16 NW CG ct, 16 NW CG (ct + 1)) (16 CG
// per wave); 16-row blocks that lie wholly beyond K are skipped.
// sM: kTK * MLds<CT>::S values of LDS for the M block (64 output rows x 64
// reduction rows).
template <typename TI, typename TO, typename CT, bool UNIT_L, int RB, int VW, int CG, int NW>
__device__ __forceinline__ void ttm_tile_s(const TI* __restrict__ Y, int J, uint32_t L, uint32_t cols,
                                           const double* __restrict__ M, int64_t msk, int64_t msj, int K,
                                           TO* __restrict__ Z, int64_t ct, int rt, CT* sM) {
  using A = Acc<CT>;
  using ML = MLds<CT>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c0 = (ct * NW + wave) * 16 * CG;  // this wave's first column
  const int k0 = rt * kTK;
  const int q = lane >> 4, i = lane & 15;
  const int64_t JL = (int64_t)J * L;

  // the columns this lane reads (B operands: columns c0 + 16 g + i; clamped
  // into the tensor for the addresses, masked where they lie beyond)
  bool cok[CG];
  int64_t cbase[CG];
#pragma unroll
  for (int g = 0; g < CG; ++g) {
    const int64_t c = c0 + 16 * g + i;
    cok[g] = c < (int64_t)cols;
    const int64_t ca = cok[g] ? c : (int64_t)cols - 1;
    if constexpr (UNIT_L) {
      cbase[g] = (int64_t)J * ca;
    } else {
      const uint32_t cc = (uint32_t)ca;
      const uint32_t r = cc / L, l = cc - r * L;
      cbase[g] = (int64_t)l + JL * r;
    }
  }
  typename A::type acc[CG][RB];
#pragma unroll
  for (int g = 0; g < CG; ++g)
#pragma unroll
    for (int b = 0; b < RB; ++b) acc[g][b] = typename A::type{0, 0, 0, 0};

  for (int jb = 0; jb < J; jb += kJB) {
    // Y operands of the four 16-row chunks of this block (row of (chunk t,
    // step s): jb + 16 t + 4 q + s), loaded without condition and masked where
    // they are used (issue4, use4)
    Raw4<TI> raw[CG][4];
#pragma unroll
    for (int g = 0; g < CG; ++g)
#pragma unroll
      for (int t = 0; t < 4; ++t) issue4<TI, UNIT_L, VW>(Y, cbase[g], J, L, jb / 16 + t, q, raw[g][t]);
    // M block into LDS: sM[k][j] = M(k0 + k, jb + j)
    __syncthreads();
    for (int e = tid; e < 16 * RB * kJB; e += 64 * NW) {
      const int kk = e / kJB, jj = e - kk * kJB;
      const int k = k0 + kk, j = jb + jj;
      sM[kk * ML::S + jj] = (k < K && j < J) ? (CT)M[(int64_t)k * msk + (int64_t)j * msj] : (CT)0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      CT y[CG][4];
#pragma unroll
      for (int g = 0; g < CG; ++g) use4<TI, CT, UNIT_L>(raw[g][t], cok[g], J, jb / 16 + t, q, y[g]);
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        if (k0 + 16 * b >= K) break;  // uniform: a block of padding rows
        CT a4[4];
        ML::read4(&sM[(16 * b + i) * ML::S + 16 * t + 4 * q], a4);  // shared by the column groups
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int g = 0; g < CG; ++g) acc[g][b] = A::mfma(a4[s], y[g][s], acc[g][b]);
      }
    }
  }

  // output row k0 + 16 b + A::row(l >> 4, v), output column c0 + 16 g + (l & 15)
#pragma unroll
  for (int g = 0; g < CG; ++g) {
    if (!cok[g]) continue;
    const int64_t c = c0 + 16 * g + i;
    int64_t zb;
    int64_t kstride;
    if constexpr (UNIT_L) {
      zb = (int64_t)K * c;
      kstride = 1;
    } else {
      const uint32_t cc = (uint32_t)c;
      const uint32_t r = cc / L, l = cc - r * L;
      zb = (int64_t)l + (int64_t)L * K * r;
      kstride = L;
    }
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = k0 + 16 * b + A::row(q, v);
        if (k < K) store_as(&Z[zb + kstride * k], (double)acc[g][b][v]);
      }
  }
}

template <typename TI, typename TO, typename CT, bool UNIT_L, int RB, int VW, int CG, int NW>
__device__ __forceinline__ void ttm_tile(const TI* __restrict__ Y, int J, uint32_t L, uint32_t cols,
                                         const double* __restrict__ M, int64_t msk, int64_t msj, int K,
                                         TO* __restrict__ Z, int64_t ct, int rt) {
  __shared__ __align__(16) CT sM[kTK * MLds<CT>::S];
  ttm_tile_s<TI, TO, CT, UNIT_L, RB, VW, CG, NW>(Y, J, L, cols, M, msk, msj, K, Z, ct, rt, sM);
}

template <typename TI, typename TO, typename CT, bool UNIT_L, int RB, int VW>
__global__ __launch_bounds__(64 * kTileWaves) void ttm_kernel(const TI* __restrict__ Y, int J, uint32_t L,
                                                              uint32_t cols, const double* __restrict__ M,
                                                              int64_t msk, int64_t msj, int K, TO* __restrict__ Z,
                                                              int nrt, int64_t total) {
  const int64_t item = xcd_remap(blockIdx.x, gridDim.x, total);
  if (item < 0) return;
  ttm_tile<TI, TO, CT, UNIT_L, RB, VW, tile_cg<CT, UNIT_L>(), kTileWaves>(Y, J, L, cols, M, msk, msj, K, Z,
                                                                         item / nrt, (int)(item % nrt));
}

// Batched item with the factor resident in LDS (K <= 32, J <= kBatchMaxJ):
// the workgroup stages M = U_t^T (32 rows, J padded to 16) once and walks
// the item's column tiles [ct0, ct1) of 16 columns per wave; each lane issues
// the loads of all 16-row blocks of its column before the products.  (The
// generic tile stages a 64 x 64 block of M for every tile, as many values as
// the tile's Y block when J <= 64.)
constexpr int kResBatchRows = 32;
template <typename CT>
constexpr int res_batch_lds() {
  return kResBatchRows * ((sizeof(CT) == 4) ? (((kBatchMaxJ + 63) & ~63) + 4) : (((kBatchMaxJ + 31) & ~31) + 2));
}
template <typename TI, typename TO, typename CT, bool UNIT_L>
__device__ __forceinline__ void ttm_batch_resident(const TI* __restrict__ Y, int J, uint32_t L, uint32_t cols,
                                                   const double* __restrict__ U, int K, TO* __restrict__ Z,
                                                   int64_t ct0, int64_t ct1, CT* sM) {
  using A = Acc<CT>;
  using ML = MLds<CT>;
  constexpr int RB = kResBatchRows / 16, NJ = kBatchMaxJ / 16;
  const int nj = (J + 15) / 16;
  const int jp = 16 * nj;
  const int ldm = ML::ld(jp);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < kResBatchRows * jp; e += 64 * kWaves) {
    const int k = e / jp, j = e - k * jp;
    sM[k * ldm + j] = (k < K && j < J) ? (CT)U[(int64_t)k * J + j] : (CT)0;
  }
  __syncthreads();
  const int q = lane >> 4, i = lane & 15;
  const int64_t JL = (int64_t)J * L;
  for (int64_t ct = ct0; ct < ct1; ++ct) {
    const int64_t c = (ct * kWaves + wave) * 16 + i;  // this lane's column
    const bool cok = c < (int64_t)cols;
    const int64_t ca = cok ? c : (int64_t)cols - 1;  // clamped, for addresses only
    int64_t cbase;
    if constexpr (UNIT_L) {
      cbase = (int64_t)J * ca;
    } else {
      const uint32_t cc = (uint32_t)ca;
      const uint32_t r = cc / L, l = cc - r * L;
      cbase = (int64_t)l + JL * r;
    }
    typename A::type acc[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) acc[b] = typename A::type{0, 0, 0, 0};
    // the blocks in two halves of NJ / 2, all loads of a half issued first
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h * (NJ / 2) >= nj) break;  // uniform
      Raw4<TI> raw[NJ / 2];
#pragma unroll
      for (int u = 0; u < NJ / 2; ++u)
        if (h * (NJ / 2) + u < nj) issue4<TI, UNIT_L, 1>(Y, cbase, J, L, h * (NJ / 2) + u, q, raw[u]);  // uniform
#pragma unroll
      for (int u = 0; u < NJ / 2; ++u) {
        const int jb = h * (NJ / 2) + u;
        if (jb >= nj) break;  // uniform
        CT y[4];
        use4<TI, CT, UNIT_L>(raw[u], cok, J, jb, q, y);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          if (16 * b >= K) break;  // uniform: a block of padding rows
          CT a4[4];
          ML::read4(&sM[(16 * b + i) * ldm + 16 * jb + 4 * q], a4);
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2) acc[b] = A::mfma(a4[s2], y[s2], acc[b]);
        }
      }
    }
    if (!cok) continue;
    int64_t zb, kstride;
    if constexpr (UNIT_L) {
      zb = (int64_t)K * c;
      kstride = 1;
    } else {
      const uint32_t cc = (uint32_t)c;
      const uint32_t r = cc / L, l = cc - r * L;
      zb = (int64_t)l + (int64_t)L * K * r;
      kstride = L;
    }
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = 16 * b + A::row(q, v);
        if (k < K) store_as(&Z[zb + kstride * k], (double)acc[b][v]);
      }
  }
}

// Batched form: item i covers column tiles [ct0, ct1) of tensor t (planned
// from upper bounds of the sizes); the current sizes and the rank R_t come
// from the device, every row tile of R_t is computed, and M = U_t^T.  Ranks
// up to 32 keep M resident (ttm_batch_resident); larger ones take the
// generic tile, which stages M per tile.
template <typename TI, typename TO, typename CT, bool UNIT_L>
__global__ __launch_bounds__(256) void ttm_batch_kernel(TtmBatch b) {
  constexpr int kLds = res_batch_lds<CT>() > kTK * MLds<CT>::S ? res_batch_lds<CT>() : kTK * MLds<CT>::S;
  __shared__ __align__(16) CT sM[kLds];
  const int64_t* d = b.items + 3 * (int64_t)blockIdx.x;
  const int t = (int)d[0];
  const int J = b.J[t];
  const int K = (int)b.R[t];
  uint64_t L = 1, Rt = 1;
  for (int k = 0; k < b.N; ++k) {
    const uint64_t c = (uint64_t)b.cur[(int64_t)t * b.N + k];
    if (k < b.n) L *= c;
    else if (k > b.n) Rt *= c;
  }
  const uint64_t cols = L * Rt;
  const int64_t ct1 = min(d[2], (int64_t)((cols + 16 * kWaves - 1) / (16 * kWaves)));
  const TI* Y = static_cast<const TI*>(b.Y[t]);
  TO* Z = static_cast<TO*>(b.Z[t]);
  const double* U = b.U + (int64_t)t * b.Jmax * b.Jmax;
  if (K <= kResBatchRows && J <= kBatchMaxJ) {
    ttm_batch_resident<TI, TO, CT, UNIT_L>(Y, J, (uint32_t)L, (uint32_t)cols, U, K, Z, d[1], ct1, sM);
    return;
  }
  for (int64_t ct = d[1]; ct < ct1; ++ct)
    for (int rt = 0; rt * kTK < K; ++rt)
      ttm_tile_s<TI, TO, CT, UNIT_L, 4, 1, 1, kWaves>(Y, J, (uint32_t)L, (uint32_t)cols, U, J, 1, K, Z, ct, rt, sM);
}

// Resident-M variant for K <= 64 with M (K_pad x J) small enough for LDS:
// each workgroup (8 waves, 128 columns per tile) stages M once and then walks
// column tiles t = blockIdx.x, blockIdx.x + gridDim.x, ... (all workgroups
// stream neighbouring columns); the Y operands are loaded two blocks of 16
// reduction rows ahead of the MFMAs.  No barrier inside the loop.
constexpr int kResidentLds = 128 * 1024;
constexpr int kResWaves = 8;

// TTM with the whole factor resident in LDS (K <= 64): each wave computes
// 16 output columns at a time, Z[0:K, cols] = M Y[:, cols], with the factor
// rows as the MFMA A operand (from LDS) and the tensor columns as the B
// operand (from HBM, straight into registers).  kDepth blocks of 16 rows are
// in flight per lane; the block loop is unrolled by kDepth so that each
// buffer keeps its registers (no moves that would wait for a load).
constexpr int kDepth = 3;
// ROW1: K = 16 (RB - 1) + 1, so the last row block holds a single output row;
// its products run on the VALU (each lane's four reduction rows of a block
// times that factor row, summed over the four lane groups at the end)
// instead of a 16 x 16 MFMA block that is one sixteenth used.

template <typename TI, typename TO, typename CT, bool UNIT_L, int RB, int VW, bool ROW1 = false>
__global__ __launch_bounds__(64 * kResWaves) void ttm_resident_kernel(const TI* __restrict__ Y, int J, uint32_t L,
                                                                      uint32_t cols, const double* __restrict__ M,
                                                                      int64_t msk, int64_t msj, int K,
                                                                      TO* __restrict__ Z, int64_t nct) {
  using A = Acc<CT>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nj = (J + 15) / 16;
  const int jp = 16 * nj;        // reduction rows padded to whole MFMA blocks (zeros)
  using ML = MLds<CT>;
  const int ldm = ML::ld(jp);
  CT* sM = reinterpret_cast<CT*>(smem);  // [16 RB][ldm]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < 16 * RB * jp; e += 64 * kResWaves) {
    const int k = e / jp, j = e - k * jp;
    sM[k * ldm + j] = (k < K && j < J) ? (CT)M[(int64_t)k * msk + (int64_t)j * msj] : (CT)0;
  }
  __syncthreads();
  const int q = lane >> 4, i = lane & 15;
  const int64_t JL = (int64_t)J * L;
  for (int64_t ct = blockIdx.x; ct < nct; ct += gridDim.x) {
    const int64_t c = (ct * kResWaves + wave) * 16 + i;  // this lane's column
    const bool cok = c < (int64_t)cols;
    const int64_t ca = cok ? c : (int64_t)cols - 1;      // clamped, for addresses only
    int64_t cbase;
    if constexpr (UNIT_L) {
      cbase = (int64_t)J * ca;
    } else {
      const uint32_t cc = (uint32_t)ca;
      const uint32_t r = cc / L, l = cc - r * L;
      cbase = (int64_t)l + JL * r;
    }
    constexpr int RBM = ROW1 ? RB - 1 : RB;  // row blocks on the MFMA
    typename A::type acc[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) acc[b] = typename A::type{0, 0, 0, 0};
    CT racc = (CT)0;  // ROW1: this lane's part of Z[16 (RB - 1)][c]
    // reduction row of (block jb, step s) for this lane: 16 jb + 4 q + s
    Raw4<TI> raw[kDepth];
    auto mma = [&](int jb, const CT (&y)[4]) {
#pragma unroll
      for (int b = 0; b < RBM; ++b) {
        CT a4[4];
        ML::read4(&sM[(16 * b + i) * ldm + 16 * jb + 4 * q], a4);
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) acc[b] = A::mfma(a4[s2], y[s2], acc[b]);
      }
      if constexpr (ROW1) {
        CT a4[4];
        ML::read4(&sM[(16 * (RB - 1)) * ldm + 16 * jb + 4 * q], a4);
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) racc = fma(a4[s2], y[s2], racc);
      }
    };
    if (nj < kDepth) {
      // fewer blocks than buffers: issue them all, then use them
#pragma unroll
      for (int u = 0; u < kDepth - 1; ++u)
        if (u < nj) issue4<TI, UNIT_L, VW>(Y, cbase, J, L, u, q, raw[u]);
#pragma unroll
      for (int u = 0; u < kDepth - 1; ++u)
        if (u < nj) {
          CT y[4];
          use4<TI, CT, UNIT_L>(raw[u], cok, J, u, q, y);
          mma(u, y);
        }
    } else {
#pragma unroll
      for (int u = 0; u < kDepth; ++u) issue4<TI, UNIT_L, VW>(Y, cbase, J, L, u, q, raw[u]);
      // main loop: whole groups of kDepth blocks whose refills all lie inside
      // the tensor; every path issues the same loads in the same order, so each
      // use waits only for its own block
      int jb0 = 0;
      for (; jb0 + 2 * kDepth <= nj; jb0 += kDepth) {
#pragma unroll
        for (int u = 0; u < kDepth; ++u) {
          CT y[4];
          use4<TI, CT, UNIT_L>(raw[u], cok, J, jb0 + u, q, y);
          issue4<TI, UNIT_L, VW>(Y, cbase, J, L, jb0 + u + kDepth, q, raw[u]);
          mma(jb0 + u, y);
        }
      }
      // the last nj - jb0 < 2 kDepth blocks: raw[u] holds block jb0 + u
#pragma unroll
      for (int u = 0; u < kDepth; ++u) {
        if (jb0 + u < nj) {  // uniform
          CT y[4];
          use4<TI, CT, UNIT_L>(raw[u], cok, J, jb0 + u, q, y);
          if (jb0 + u + kDepth < nj) issue4<TI, UNIT_L, VW>(Y, cbase, J, L, jb0 + u + kDepth, q, raw[u]);
          mma(jb0 + u, y);
        }
      }
#pragma unroll
      for (int u = 0; u < kDepth - 1; ++u) {
        if (jb0 + kDepth + u < nj) {  // uniform
          CT y[4];
          use4<TI, CT, UNIT_L>(raw[u], cok, J, jb0 + kDepth + u, q, y);
          mma(jb0 + kDepth + u, y);
        }
      }
    }
    if constexpr (ROW1) {
      // the four lane groups of column i, in a fixed order
      const CT x = racc + __shfl_xor(racc, 16, 64);
      racc = x + __shfl_xor(x, 32, 64);
    }
    if (cok) {
      int64_t zb, kstride;
      if constexpr (UNIT_L) {
        zb = (int64_t)K * c;
        kstride = 1;
      } else {
        const uint32_t cc = (uint32_t)c;
        const uint32_t r = cc / L, l = cc - r * L;
        zb = (int64_t)l + (int64_t)L * K * r;
        kstride = L;
      }
#pragma unroll
      for (int b = 0; b < RBM; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = 16 * b + A::row(q, v);
          if (k < K) store_as(&Z[zb + kstride * k], (double)acc[b][v]);
        }
      if constexpr (ROW1)
        if (q == 0) store_as(&Z[zb + kstride * (16 * (RB - 1))], (double)racc);
    }
  }
}

template <typename TI, typename TO, typename CT>
hipError_t launch_ttm_ct(const TI* Y, int J, uint64_t L, uint64_t cols, const double* M, int64_t msk, int64_t msj,
                         int K, TO* Z, hipStream_t stream) {
  const int rbr = (int)ceil_div(K, 16);
  const size_t lds = sizeof(CT) * (size_t)(16 * rbr) * (size_t)MLds<CT>::ld((int)(16 * ceil_div(J, 16)));
  if (K <= 64 && lds <= (size_t)kResidentLds) {
    const int64_t nct = ceil_div((int64_t)cols, 16 * kResWaves);
    const int64_t grid = std::min<int64_t>(nct, 2 * 256);
#define TR_LAUNCH(U, RBV, V)                                                                                   \
  hipLaunchKernelGGL((ttm_resident_kernel<TI, TO, CT, U, RBV, V>), dim3(grid), dim3(64 * kResWaves), lds,       \
                     stream, Y, J, (uint32_t)L, (uint32_t)cols, M, msk, msj, K, Z, nct)
#define TR_LAUNCH1(U, RBV, V)                                                                                  \
  hipLaunchKernelGGL((ttm_resident_kernel<TI, TO, CT, U, RBV, V, true>), dim3(grid), dim3(64 * kResWaves),     \
                     lds, stream, Y, J, (uint32_t)L, (uint32_t)cols, M, msk, msj, K, Z, nct)
    const int vw = y_vector_width(Y, J, L);
    if constexpr (std::is_same<CT, double>::value) {
      if (K % 16 == 1 && K > 16) {
      // FP64 with a single row in the last row block (K = 17, 33, 49)
      if (vw == 4) {
        if (rbr == 2) TR_LAUNCH1(true, 2, 4);
        else if (rbr == 3) TR_LAUNCH1(true, 3, 4);
        else TR_LAUNCH1(true, 4, 4);
      } else if (vw == 2) {
        if (rbr == 2) TR_LAUNCH1(true, 2, 2);
        else if (rbr == 3) TR_LAUNCH1(true, 3, 2);
        else TR_LAUNCH1(true, 4, 2);
      } else if (L == 1) {
        if (rbr == 2) TR_LAUNCH1(true, 2, 1);
        else if (rbr == 3) TR_LAUNCH1(true, 3, 1);
        else TR_LAUNCH1(true, 4, 1);
      } else {
        if (rbr == 2) TR_LAUNCH1(false, 2, 1);
        else if (rbr == 3) TR_LAUNCH1(false, 3, 1);
        else TR_LAUNCH1(false, 4, 1);
      }
      return hipGetLastError();
      }
    }
    if (vw == 4) {
      if (rbr == 1) TR_LAUNCH(true, 1, 4);
      else if (rbr == 2) TR_LAUNCH(true, 2, 4);
      else if (rbr == 3) TR_LAUNCH(true, 3, 4);
      else TR_LAUNCH(true, 4, 4);
    } else if (vw == 2) {
      if (rbr == 1) TR_LAUNCH(true, 1, 2);
      else if (rbr == 2) TR_LAUNCH(true, 2, 2);
      else if (rbr == 3) TR_LAUNCH(true, 3, 2);
      else TR_LAUNCH(true, 4, 2);
    } else if (L == 1) {
      if (rbr == 1) TR_LAUNCH(true, 1, 1);
      else if (rbr == 2) TR_LAUNCH(true, 2, 1);
      else if (rbr == 3) TR_LAUNCH(true, 3, 1);
      else TR_LAUNCH(true, 4, 1);
    } else {
      if (rbr == 1) TR_LAUNCH(false, 1, 1);
      else if (rbr == 2) TR_LAUNCH(false, 2, 1);
      else if (rbr == 3) TR_LAUNCH(false, 3, 1);
      else TR_LAUNCH(false, 4, 1);
    }
#undef TR_LAUNCH1
#undef TR_LAUNCH
    return hipGetLastError();
  }
  const int nrt = (int)ceil_div(K, kTK);
  const int cg = (L == 1) ? tile_cg<CT, true>() : tile_cg<CT, false>();
  const int64_t nct = ceil_div((int64_t)cols, 16 * kTileWaves * cg);
  const int64_t total = nct * nrt;
  const int64_t grid = ceil_div(total, kXcds) * kXcds;
  const int rb = (K >= kTK) ? 4 : (int)ceil_div(K, 16);
#define TTM_LAUNCH(U, RBV, V)                                                                                  \
  hipLaunchKernelGGL((ttm_kernel<TI, TO, CT, U, RBV, V>), dim3(grid), dim3(64 * kTileWaves), 0, stream, Y, J,   \
                     (uint32_t)L, (uint32_t)cols, M, msk, msj, K, Z, nrt, total)
  const int vw = y_vector_width(Y, J, L);
  if (vw == 4) {
    if (rb == 1) TTM_LAUNCH(true, 1, 4);
    else if (rb == 2) TTM_LAUNCH(true, 2, 4);
    else if (rb == 3) TTM_LAUNCH(true, 3, 4);
    else TTM_LAUNCH(true, 4, 4);
  } else if (vw == 2) {
    if (rb == 1) TTM_LAUNCH(true, 1, 2);
    else if (rb == 2) TTM_LAUNCH(true, 2, 2);
    else if (rb == 3) TTM_LAUNCH(true, 3, 2);
    else TTM_LAUNCH(true, 4, 2);
  } else if (L == 1) {
    if (rb == 1) TTM_LAUNCH(true, 1, 1);
    else if (rb == 2) TTM_LAUNCH(true, 2, 1);
    else if (rb == 3) TTM_LAUNCH(true, 3, 1);
    else TTM_LAUNCH(true, 4, 1);
  } else {
    if (rb == 1) TTM_LAUNCH(false, 1, 1);
    else if (rb == 2) TTM_LAUNCH(false, 2, 1);
    else if (rb == 3) TTM_LAUNCH(false, 3, 1);
    else TTM_LAUNCH(false, 4, 1);
  }
#undef TTM_LAUNCH
  return hipGetLastError();
}

}  // namespace

template <typename TI, typename TO>
hipError_t launch_ttm(const TI* Y, int J, uint64_t L, uint64_t cols, const double* M, int64_t msk, int64_t msj,
                      int K, TO* Z, bool fp32_products, hipStream_t stream) {
  if (fp32_products) return launch_ttm_ct<TI, TO, float>(Y, J, L, cols, M, msk, msj, K, Z, stream);
  // more than 64 output rows with 16-byte aligned operands: the tiled kernel
  // with direct global-to-LDS staging (ttm_dma.hip)
  if (ttm_dma_eligible(J, L, cols, K, msk, msj, (int)sizeof(TI), (int)sizeof(TO), Y, M))
    return launch_ttm_dma(Y, J, L, cols, M, msk, msj, K, Z, stream);
  return launch_ttm_ct<TI, TO, double>(Y, J, L, cols, M, msk, msj, K, Z, stream);
}

template <typename TI, typename TO>
hipError_t launch_ttm_batched(const TtmBatch& b, bool fp32_products, bool unit_l, hipStream_t stream) {
  if (b.nitems <= 0) return hipErrorInvalidValue;
#define TB_LAUNCH(CT, U) \
  hipLaunchKernelGGL((ttm_batch_kernel<TI, TO, CT, U>), dim3(b.nitems), dim3(64 * kWaves), 0, stream, b)
  if (fp32_products) {
    if (unit_l) TB_LAUNCH(float, true);
    else TB_LAUNCH(float, false);
  } else {
    if (unit_l) TB_LAUNCH(double, true);
    else TB_LAUNCH(double, false);
  }
#undef TB_LAUNCH
  return hipGetLastError();
}

template hipError_t launch_ttm_batched<float, float>(const TtmBatch&, bool, bool, hipStream_t);
template hipError_t launch_ttm_batched<float, double>(const TtmBatch&, bool, bool, hipStream_t);
template hipError_t launch_ttm_batched<double, double>(const TtmBatch&, bool, bool, hipStream_t);

template hipError_t launch_ttm<double, double>(const double*, int, uint64_t, uint64_t, const double*, int64_t,
                                               int64_t, int, double*, bool, hipStream_t);
template hipError_t launch_ttm<float, double>(const float*, int, uint64_t, uint64_t, const double*, int64_t,
                                              int64_t, int, double*, bool, hipStream_t);
template hipError_t launch_ttm<double, float>(const double*, int, uint64_t, uint64_t, const double*, int64_t,
                                              int64_t, int, float*, bool, hipStream_t);
template hipError_t launch_ttm<float, float>(const float*, int, uint64_t, uint64_t, const double*, int64_t,
                                             int64_t, int, float*, bool, hipStream_t);

}  // namespace tk
