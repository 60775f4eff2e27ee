// Gram matrix S = Y_(n) Y_(n)^T (Alg. 2; flop count Sec. 7) for mode sizes
// above the whole-triangle kernel's range: FP64 products of float or double
// input, or, for float input, FP32 MFMA products (the FP32 form) or the
// three-piece bf16 split products of the BF16X6 form (b0 = bf16(x),
// b1 = bf16(x - b0), b2 = bf16(x - b0 - b1); b2 c0 + b0 c2 + b1 c1 +
// b1 c0 + b0 c1 + b0 c0 with v_mfma_f32_16x16x32_bf16), each summed in FP32
// over a 32-column chunk and in FP64 across chunks.
//
// Work items: a pair of 128-row tiles (ta <= tb) and a contiguous range of
// column chunks.  Four waves per workgroup; each holds a 64 x 64 part of the
// pair's 128 x 128 output as 4 x 4 blocks of 16 x 16 in FP64 MFMA
// accumulators (v_mfma_f64_16x16x4f64), so a step of four columns reads 8
// operands from LDS for 16 MFMAs.  Diagonal pairs compute the upper triangle
// only (gram_dma.hpp: wave_task), and blocks of rows at or beyond J are
// skipped, so a ragged last tile costs only its rows.  About 8192 items: the
// faster diagonal and ragged items then even out over the run (with two items
// per workgroup slot the run ended on a long tail of slow items).
//
// Staging: the chunk images (gram_dma.hpp) are written straight from global
// memory into LDS (global_load_lds, 64 lanes x 16 bytes per instruction),
// with no registers in between; tensors whose rows or columns are not
// 16-byte aligned use the tile-pair kernels of gram_mixed.hip instead.
// Elements outside the tensor are not loaded: rows >= J feed only rows and
// columns of S that are dropped, and the columns past the end of the
// unfolding (or of a slab of L columns) are zeroed in LDS.  Each workgroup
// double-buffers its chunks (64 or 80 KB), so two workgroups fit on a CU and
// one's barriers overlap the other's MFMAs; the loads of the next chunk run
// during the MFMAs of the current one (chunk_loop).
//
// Output: every item writes its FP64 partial blocks in the layout of the
// tile-pair reduction (gram_mixed.hip), which sums the splits in a fixed
// order.  ||Y||^2 is the trace of S with FP64 products (its diagonal entries
// are FP64 sums of squares of the values as loaded); with FP32 products the
// diagonal items sum the squares of their tile's rows in FP64 from LDS.
#include "common.hpp"
#include "gram_dma.hpp"
#include "kernels.hpp"

namespace tk {

namespace {

using dma::Img;

constexpr int kDW = 4;           // waves per workgroup
constexpr int kDNT = 64 * kDW;   // threads per workgroup

typedef __attribute__((address_space(3))) void lds_void;

struct DmaParams {
  const char* Y;   // the tensor's bytes
  int J;
  int64_t L;       // layout 0: 1
  int64_t K;       // columns of the unfolding
  int64_t CL;      // layout 1: chunks per slab of L columns
  int64_t nchunks, nsplit, total;
  int64_t cps;     // chunks per split
  int ntiles, npairs;
  double* part;
  double* sq;  // PREC 1: one sum of squares per item
};

__device__ __forceinline__ void decode_pair_dma(int p, int ntiles, int& ta, int& tb) {
  int t = 0;
  while (p >= ntiles - t) {
    p -= ntiles - t;
    ++t;
  }
  ta = t;
  tb = t + p;
}

// First column and valid column count of chunk ch (layout 1: and the slab's
// element offset).
template <typename T, int LAY>
__device__ __forceinline__ void chunk_cols(const DmaParams& g, int64_t ch, int64_t& c0, int& ncol, int64_t& base_m) {
  using I = Img<sizeof(T), LAY>;
  if constexpr (LAY == 0) {
    c0 = ch * I::KC;
    ncol = (int)min((int64_t)I::KC, g.K - c0);
    base_m = 0;
  } else {
    const int64_t m = ch / g.CL;
    c0 = (ch - m * g.CL) * I::KC;
    ncol = (int)min((int64_t)I::KC, g.L - c0);
    base_m = m * g.L * g.J;
  }
}

// Issues the loads of chunk ch into one buffer.  Instruction j of the chunk
// covers bytes [1024 jj, 1024 (jj + 1)) of tile image p (jj = j mod IPS);
// wave w issues j = w, w + 4, ...  Lanes whose element lies outside the
// tensor issue nothing: rows >= J only feed rows and columns of S that are
// not kept, and columns past the chunk's end are zeroed by fill_chunk.
// Addresses are split into a part common to the wave (scalar) and a small
// per-lane part, so that an instruction costs a few vector operations.
template <typename T, int LAY>
__device__ __forceinline__ void issue_chunk(const DmaParams& g, int64_t ch, char* buf, int nslots, int r0a, int r0b,
                                            int wave, int lane) {
  using I = Img<sizeof(T), LAY>;
  constexpr int ES = sizeof(T), W = 16;
  constexpr int IPS = I::TB / (64 * W);
  int64_t c0, base_m;
  int ncol;
  chunk_cols<T, LAY>(g, ch, c0, ncol, base_m);
  const int n = nslots * IPS;
  if constexpr (LAY == 1) {
    // instruction jj: rows RPI jj .. RPI jj + RPI - 1 of the tile, LPR lanes per row
    constexpr int LPR = 128 / W, RPI = 64 / LPR;
    const int rl = lane / LPR, wb = (lane % LPR) * W;
    const int64_t lane_row = (int64_t)rl * g.L * ES;  // bytes to the lane's row
    for (int j = wave; j < n; j += kDW) {
      const int p = (j >= IPS) ? 1 : 0;
      const int jj = j - p * IPS;
      const int rt = (p ? r0b : r0a) + RPI * jj;  // the instruction's first row in the tensor
      const int r = RPI * jj + rl;                // the lane's row in the tile
      const int u = (wb >> 4) ^ ((r >> 1) & 7);
      const int c = u * I::E + (wb & 15) / ES;
      if (rt + rl < g.J && c < ncol) {
        const int64_t wave_off = ((c0 + base_m) + g.L * (int64_t)rt) * ES;
        const void* src = static_cast<const void*>(g.Y + wave_off + lane_row + (c * ES + (wb & 15) % ES));
        char* dst = buf + p * I::TB + jj * 64 * W;
        __builtin_amdgcn_global_load_lds(src, (lds_void*)dst, 16, 0, 0);
      }
    }
  } else {
    for (int j = wave; j < n; j += kDW) {
      const int p = (j >= IPS) ? 1 : 0;
      const int jj = j - p * IPS;
      int r, c, b;
      I::inv(jj * 64 * W + lane * W, r, c, b);
      const int rt = p ? r0b : r0a;
      if (rt + r < g.J && c < ncol) {
        const int64_t wave_off = ((int64_t)rt + (int64_t)g.J * c0) * ES;
        const void* src = static_cast<const void*>(g.Y + wave_off + ((r + g.J * c) * ES + b));
        char* dst = buf + p * I::TB + jj * 64 * W;
        __builtin_amdgcn_global_load_lds(src, (lds_void*)dst, 16, 0, 0);
      }
    }
  }
}

// Zeros the positions of chunk ch's columns past its end (the last chunk of
// the unfolding, or of a slab of L columns when KC does not divide L).  Called
// once the wave's own loads have landed, so that no load is in flight; no
// load ever targets these positions.
template <typename T, int LAY>
__device__ __forceinline__ void fill_chunk(const DmaParams& g, int64_t ch, char* buf, int nslots, int wave,
                                           int lane) {
  using I = Img<sizeof(T), LAY>;
  constexpr int W = 16;
  constexpr int IPS = I::TB / (64 * W);
  int64_t c0, base_m;
  int ncol;
  chunk_cols<T, LAY>(g, ch, c0, ncol, base_m);
  if (ncol >= I::KC) return;
  const int n = nslots * IPS;
  for (int j = wave; j < n; j += kDW) {
    const int p = (j >= IPS) ? 1 : 0;
    const int jj = j - p * IPS;
    int r, c, b;
    I::inv(jj * 64 * W + lane * W, r, c, b);
    if (c >= ncol) {
      char* dst = buf + p * I::TB + jj * 64 * W + lane * W;
      *reinterpret_cast<uint4*>(dst) = uint4{0u, 0u, 0u, 0u};
    }
  }
}

template <typename T, int LAY>
struct Ops;

// layout 0: one element per operand and step
template <typename T>
struct Ops<T, 0> {
  using I = Img<sizeof(T), 0>;
  static constexpr int NG = I::KC / 4;  // operand groups (steps) per chunk
  static constexpr int GS = 1;          // steps per group
  T a[4], b[4];
  int d;  // unused
  __device__ __forceinline__ void read(const char* buf, const int (&oa)[4], const int (&ob)[4], int g) {
#pragma unroll
    for (int t = 0; t < 4; ++t) a[t] = *reinterpret_cast<const T*>(buf + oa[t] + g * 4 * I::CB);
#pragma unroll
    for (int t = 0; t < 4; ++t) b[t] = *reinterpret_cast<const T*>(buf + ob[t] + g * 4 * I::CB);
  }
  __device__ __forceinline__ T A(int t, int) const { return a[t]; }
  __device__ __forceinline__ T B(int t, int) const { return b[t]; }
};

// layout 1: one 16-byte unit per operand and group of E steps
template <typename T>
struct Ops<T, 1> {
  using I = Img<sizeof(T), 1>;
  static constexpr int NG = 2;
  static constexpr int GS = I::E;
  typedef T V __attribute__((ext_vector_type(16 / sizeof(T))));
  V a[4], b[4];
  int d;  // byte distance from unit q to unit q | 4 of the lane's rows
  __device__ __forceinline__ void read(const char* buf, const int (&oa)[4], const int (&ob)[4], int g) {
    const int o = g ? d : 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) a[t] = *reinterpret_cast<const V*>(buf + oa[t] + o);
#pragma unroll
    for (int t = 0; t < 4; ++t) b[t] = *reinterpret_cast<const V*>(buf + ob[t] + o);
  }
  __device__ __forceinline__ T A(int t, int s) const { return a[t][s]; }
  __device__ __forceinline__ T B(int t, int s) const { return b[t][s]; }
};

// MK: the compile-time block mask (gram_dma.hpp), or kGeneric for a mask
// known only at run time (ragged last tiles), tested block by block.
constexpr unsigned kGeneric = 0x10000u;

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// The bf16 pieces of eight FP32 values: b0 = bf16(x), b1 = bf16(x - b0)
// (x - b0 is exact in FP32) and b2 = bf16(x - b0 - b1).
__device__ __forceinline__ void split8(const float (&v)[8], bf8 (&p)[3]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float x = v[e];
    const __bf16 b0 = (__bf16)x;
    const float r1 = x - (float)b0;
    const __bf16 b1 = (__bf16)r1;
    p[0][e] = b0;
    p[1][e] = b1;
    p[2][e] = (__bf16)(r1 - (float)b1);
  }
}

// The eight FP32 values of one operand block that lane (i, q) supplies to a
// bf16 MFMA (K = 32, 8 per lane group): slot e holds the column that the FP32
// form reads at its step e (Img::col(e, q)); off is the block's group-0 byte
// offset, d (layout 1) the distance to the lane's second unit.
template <int LAY>
__device__ __forceinline__ void read8(const char* buf, int off, int d, float (&v)[8]) {
  if constexpr (LAY == 0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = *reinterpret_cast<const float*>(buf + off + e * 4 * Img<4, 0>::CB);
  } else {
    const float4 u0 = *reinterpret_cast<const float4*>(buf + off);
    const float4 u1 = *reinterpret_cast<const float4*>(buf + off + d);
    v[0] = u0.x; v[1] = u0.y; v[2] = u0.z; v[3] = u0.w;
    v[4] = u1.x; v[5] = u1.y; v[6] = u1.z; v[7] = u1.w;
  }
}

// BF16X6 products of one chunk (PREC 3).  The slot map of read8 is the same
// for both operands, so slot e of lane group q is the same column in A and B.
// The A blocks are split once per chunk, the B blocks one at a time; each
// block's FP32 chunk sum, smallest terms first, is then added to its FP64
// accumulator.
template <unsigned MK, int LAY>
__device__ __forceinline__ void compute_chunk_bf(const char* buf, const int (&oa)[4], const int (&ob)[4], int d,
                                                 d4 (&acc)[4][4], unsigned mask) {
  auto on = [&](int x, int y) {
    return (MK == kGeneric) ? ((mask >> (4 * x + y)) & 1u) : ((MK >> (4 * x + y)) & 1u);
  };
  bf8 ap[4][3];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    float v[8];
    read8<LAY>(buf, oa[x], d, v);
    split8(v, ap[x]);
  }
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    float v[8];
    read8<LAY>(buf, ob[y], d, v);
    bf8 bp[3];
    split8(v, bp);
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      if (on(x, y)) {
        f4 c = f4{0.f, 0.f, 0.f, 0.f};
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[x][2], bp[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[x][0], bp[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[x][1], bp[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[x][1], bp[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[x][0], bp[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[x][0], bp[0], c, 0, 0, 0);
#pragma unroll
        for (int v2 = 0; v2 < 4; ++v2) acc[x][y][v2] += (double)c[v2];
      }
    }
  }
}

// PREC 0: FP64 products and accumulation.  PREC 1 (float input): FP32 MFMA
// products accumulated in FP32 over the chunk's 32 columns, then added to
// the FP64 accumulators.
template <unsigned MK, typename T, int LAY, int PREC>
__device__ __forceinline__ void compute_chunk(const char* buf, const int (&oa)[4], const int (&ob)[4], int d,
                                              d4 (&acc)[4][4], unsigned mask) {
  if constexpr (PREC == 3) {
    compute_chunk_bf<MK, LAY>(buf, oa, ob, d, acc, mask);
    return;
  }
  using O = Ops<T, LAY>;
  O cur, nxt;
  cur.d = nxt.d = d;
  f4 acc32[4][4];
  if constexpr (PREC == 1) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc32[x][y] = f4{0.f, 0.f, 0.f, 0.f};
  }
  cur.read(buf, oa, ob, 0);
#pragma unroll
  for (int g = 0; g < O::NG; ++g) {
    if (g + 1 < O::NG) nxt.read(buf, oa, ob, g + 1);
#pragma unroll
    for (int s = 0; s < O::GS; ++s) {
#pragma unroll
      for (int x = 0; x < 4; ++x) {
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const bool on = (MK == kGeneric) ? ((mask >> (4 * x + y)) & 1u) : ((MK >> (4 * x + y)) & 1u);
          if (on) {
            if constexpr (PREC == 0)
              acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)cur.A(x, s), (double)cur.B(y, s), acc[x][y],
                                                               0, 0, 0);
            else
              acc32[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur.A(x, s), cur.B(y, s), acc32[x][y], 0, 0, 0);
          }
        }
      }
    }
    if (g + 1 < O::NG) cur = nxt;
  }
  if constexpr (PREC == 1) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const bool on = (MK == kGeneric) ? ((mask >> (4 * x + y)) & 1u) : ((MK >> (4 * x + y)) & 1u);
        if (on) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[x][y][v] += (double)acc32[x][y][v];
        }
      }
  }
}

// FP64 sum of squares of the rows of a diagonal item's tile image (float
// input, PREC 1): rows >= J hold stale data and are skipped, columns past the
// chunk's end were zeroed.
template <int LAY>
__device__ __forceinline__ double chunk_sq(const char* buf, int r0, int J, int tid) {
  using I = Img<4, LAY>;
  double s = 0.0;
  for (int u = tid; u < I::TB / 16; u += kDNT) {
    int r, c, b;
    I::inv(16 * u, r, c, b);
    const float4 v = *reinterpret_cast<const float4*>(buf + 16 * u);
    const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      // layout 1: the unit's elements share row r; layout 0: rows r .. r + 3
      const int row = r0 + r + (LAY == 0 ? h : 0);
      if (row < J) s += (double)e[h] * (double)e[h];
    }
  }
  return s;
}

// The chunks of one item: chunk t sits in buffer t & 1.  The loads of chunk
// t + 1 are issued right after the barrier that makes chunk t available, so
// they run during chunk t's MFMAs; then the wave waits for them, zeros any
// columns past the chunk's end and meets the others at the next barrier,
// after which the buffer of chunk t is free for chunk t + 2.
template <unsigned MK, typename T, int LAY, int PREC>
__device__ __forceinline__ void chunk_loop(const DmaParams& g, int64_t split, int64_t ns, int64_t niter, char* buf0, char* buf1,
                                           int nslots, int r0a, int r0b, int wave, int lane, const int (&oa)[4],
                                           const int (&ob)[4], int d, d4 (&acc)[4][4], unsigned mask, double& sq) {
  // reduced forms: diagonal items also sum the squares of their tile's rows
  const bool dsq = (PREC >= 1) && nslots == 1;
  const int tid = 64 * wave + lane;
  if (niter <= 0) return;
  issue_chunk<T, LAY>(g, split, buf0, nslots, r0a, r0b, wave, lane);
  __builtin_amdgcn_s_waitcnt(0);
  fill_chunk<T, LAY>(g, split, buf0, nslots, wave, lane);
  __syncthreads();
  for (int64_t t = 0;; t += 2) {
    if (t + 1 < niter) issue_chunk<T, LAY>(g, split + (t + 1) * ns, buf1, nslots, r0a, r0b, wave, lane);
    if constexpr (PREC >= 1)
      if (dsq) sq += chunk_sq<LAY>(buf0, r0a, g.J, tid);
    compute_chunk<MK, T, LAY, PREC>(buf0, oa, ob, d, acc, mask);
    if (t + 1 >= niter) break;
    __builtin_amdgcn_s_waitcnt(0);
    fill_chunk<T, LAY>(g, split + (t + 1) * ns, buf1, nslots, wave, lane);
    __syncthreads();
    if (t + 2 < niter) issue_chunk<T, LAY>(g, split + (t + 2) * ns, buf0, nslots, r0a, r0b, wave, lane);
    if constexpr (PREC >= 1)
      if (dsq) sq += chunk_sq<LAY>(buf1, r0a, g.J, tid);
    compute_chunk<MK, T, LAY, PREC>(buf1, oa, ob, d, acc, mask);
    if (t + 2 >= niter) break;
    __builtin_amdgcn_s_waitcnt(0);
    fill_chunk<T, LAY>(g, split + (t + 2) * ns, buf0, nslots, wave, lane);
    __syncthreads();
  }
}

// FP64 products: two workgroups per CU (at most 256 registers per lane).
// The reduced forms keep FP32 chunk sums or bf16 pieces beside the FP64
// accumulators, which does not fit 256 registers: one workgroup (one wave per
// SIMD) per CU.
template <typename T, int LAY, int PREC>
__global__ __launch_bounds__(kDNT, PREC == 0 ? 2 : 1) void gram_dma_kernel(DmaParams g) {
  static_assert(PREC == 0 || sizeof(T) == 4, "the reduced forms read float input");
  using I = Img<sizeof(T), LAY>;
  __shared__ __attribute__((aligned(16))) char buf0[2 * I::TB];
  __shared__ __attribute__((aligned(16))) char buf1[2 * I::TB];
  const int64_t item = xcd_remap(blockIdx.x, gridDim.x, g.total);
  if (item < 0) return;
  const int pair = (int)(item % g.npairs);
  const int64_t split = item / g.npairs;
  int ta, tb;
  decode_pair_dma(pair, g.ntiles, ta, tb);
  const bool diag = (ta == tb);
  const int nslots = diag ? 1 : 2;
  const int r0a = 128 * ta, r0b = 128 * tb;
  // split s takes the contiguous chunks [s cps, (s + 1) cps)
  const int64_t c0 = split * g.cps, cstep = 1, niter = min(g.cps, g.nchunks - c0);

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i = lane & 15, q = lane >> 4;
  int a0, b0, bs;
  unsigned mask;
  dma::wave_task(wave, diag, r0a, r0b, g.J, a0, b0, bs, mask);
  a0 = __builtin_amdgcn_readfirstlane(a0);
  b0 = __builtin_amdgcn_readfirstlane(b0);
  bs = __builtin_amdgcn_readfirstlane(bs);
  mask = __builtin_amdgcn_readfirstlane(mask);
  const int pb = diag ? 0 : I::TB;  // B operand's tile image

  // operand byte offsets (group 0) of this lane's four A and four B blocks
  int oa[4], ob[4], d = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    oa[t] = I::at(16 * (a0 + t) + i, I::col(0, q));
    ob[t] = pb + I::at(16 * (b0 + bs * t) + i, I::col(0, q));
  }
  if constexpr (LAY == 1) d = I::at(i, I::col(I::E, q)) - I::at(i, I::col(0, q));

  d4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};

  // one copy of the loop per mask class, so that the accumulators flow
  // through a single chain of MFMAs; waves without blocks still load and
  // meet the barriers
  double sq = 0.0;
#define DMA_LOOP(MK) \
  chunk_loop<MK, T, LAY, PREC>(g, c0, cstep, niter, buf0, buf1, nslots, r0a, r0b, wave, lane, oa, ob, d, acc, mask, sq)
  if (mask == dma::kMaskFull) DMA_LOOP(dma::kMaskFull);
  else if (mask == dma::kMaskUpper) DMA_LOOP(dma::kMaskUpper);
  else if (mask == dma::kMaskHalf) DMA_LOOP(dma::kMaskHalf);
  else if (mask == dma::kMaskCol1) DMA_LOOP(dma::kMaskCol1);
  else if (mask == 0u) DMA_LOOP(0u);
  else DMA_LOOP(kGeneric);
#undef DMA_LOOP

  if constexpr (PREC >= 1) {
    // the item's sum of squares (zero unless diagonal), in wave order
    __shared__ double sred[kDW];
    const double sw = wave_sum(sq);
    if (lane == 0) sred[wave] = sw;
    __syncthreads();
    if (tid == 0) g.sq[item] = (sred[0] + sred[1]) + (sred[2] + sred[3]);
  }

  // partial blocks.  MFMA result, lane l, register v: FP64 D[(l >> 4) + 4 v][l & 15],
  // FP32 D[4 (l >> 4) + v][l & 15]
  double* __restrict__ P = g.part + item * (int64_t)64 * 256;
#pragma unroll
  for (int x = 0; x < 4; ++x) {
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      if ((mask >> (4 * x + y)) & 1u) {
        const int bi = a0 + x, bj = b0 + bs * y;
        const int qb = diag ? dma::tri_index(bi, bj) : bi * 8 + bj;
#pragma unroll
        for (int v = 0; v < 4; ++v) P[(int64_t)qb * 256 + (PREC == 0 ? q + 4 * v : 4 * q + v) * 16 + i] = acc[x][y][v];
      }
    }
  }
}

// trace(S) in a fixed order: one workgroup.
__global__ __launch_bounds__(256) void gram_trace_kernel(const double* __restrict__ S, int J,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int a = threadIdx.x; a < J; a += 256) s += S[(int64_t)a * J + a];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}


}  // namespace

bool gram_dma_eligible(int J, uint64_t L, int elem_size, const void* Y) {
  const uint64_t KC = 128 / elem_size;
  // 16-byte loads: the base and the stride between consecutive columns (unit
  // stride) or rows (row segments) must be multiples of 16 bytes
  const uint64_t stride_bytes = (L == 1 ? (uint64_t)J : L) * (uint64_t)elem_size;
  return J > 128 && J <= (1 << 20) && (L == 1 || L >= 64 || L % KC == 0) && stride_bytes % 16 == 0 &&
         reinterpret_cast<uintptr_t>(Y) % 16 == 0;
}

GramPlan plan_gram_dma(int J, uint64_t L, uint64_t K, int elem_size, int prec) {
  GramPlan p{};
  const int64_t KC = (L == 1 && elem_size == 8) ? Img<8, 0>::KC : 128 / elem_size;
  p.tile = 128;
  p.nchunks = (L == 1) ? ceil_div((int64_t)K, KC) : (int64_t)(K / L) * ceil_div((int64_t)L, KC);
  p.ntiles = (int)ceil_div(J, 128);
  p.npairs = p.ntiles * (p.ntiles + 1) / 2;
  // about 16 items per workgroup slot (two slots per CU), at least 16 chunks
  // each: items of different speed (diagonal and ragged pairs are faster)
  // then even out over the run; 128 KB of partial blocks per item
  int64_t nsplit = std::max<int64_t>(1, 8192 / p.npairs);
  nsplit = std::min<int64_t>(nsplit, std::max<int64_t>(1, p.nchunks / 16));
  p.cps = ceil_div(p.nchunks, nsplit);
  p.nsplit = ceil_div(p.nchunks, p.cps);
  p.part_elems = p.nsplit * p.npairs * 64 * 256;
  p.sq_elems = (prec >= 1) ? p.nsplit * p.npairs : 0;
  return p;
}

template <typename T>
hipError_t launch_gram_dma(const T* Y, int J, uint64_t L, uint64_t K, int prec, const GramPlan& p, double* part,
                           double* sq, double* S, double* norm2, hipStream_t stream, hipEvent_t after_main) {
  if (!gram_dma_eligible(J, L, (int)sizeof(T), Y)) return hipErrorInvalidValue;
  if (prec != 0 && ((prec != 1 && prec != 3) || sizeof(T) != 4 || sq == nullptr)) return hipErrorInvalidValue;
  DmaParams g{};
  g.Y = reinterpret_cast<const char*>(Y);
  g.J = J;
  g.L = (int64_t)L;
  g.K = (int64_t)K;
  const int64_t KC = 128 / (int64_t)sizeof(T);
  g.CL = ceil_div((int64_t)L, KC);
  g.nchunks = p.nchunks;
  g.nsplit = p.nsplit;
  g.cps = p.cps;
  g.ntiles = p.ntiles;
  g.npairs = p.npairs;
  g.total = p.nsplit * p.npairs;
  g.part = part;
  g.sq = sq;
  const int64_t grid = ceil_div(g.total, kXcds) * kXcds;
  if constexpr (sizeof(T) == 4) {
    // the reduced forms take unit-stride modes only (on row segments the
    // register-staged tile pairs measured faster)
    if (prec != 0 && L != 1) return hipErrorInvalidValue;
    if (prec == 1) hipLaunchKernelGGL((gram_dma_kernel<T, 0, 1>), dim3(grid), dim3(kDNT), 0, stream, g);
    else if (prec == 3) hipLaunchKernelGGL((gram_dma_kernel<T, 0, 3>), dim3(grid), dim3(kDNT), 0, stream, g);
  }
  if (prec == 0) {
    if (L == 1) hipLaunchKernelGGL((gram_dma_kernel<T, 0, 0>), dim3(grid), dim3(kDNT), 0, stream, g);
    else hipLaunchKernelGGL((gram_dma_kernel<T, 1, 0>), dim3(grid), dim3(kDNT), 0, stream, g);
  }
  if (after_main) (void)hipEventRecord(after_main, stream);
  launch_gram_pair_reduce(part, p.ntiles, p.npairs, p.nsplit, J, S, stream);
  if (norm2) {
    // FP64: the trace of S is the FP64 sum of squares; reduced forms: the
    // diagonal items' FP64 sums of squares, in item order
    if (prec == 0) hipLaunchKernelGGL(gram_trace_kernel, dim3(1), dim3(256), 0, stream, S, J, norm2);
    else hipLaunchKernelGGL(sum_fixed_kernel, dim3(1), dim3(256), 0, stream, sq, g.total, norm2);
  }
  return hipGetLastError();
}

template hipError_t launch_gram_dma<float>(const float*, int, uint64_t, uint64_t, int, const GramPlan&, double*,
                                           double*, double*, double*, hipStream_t, hipEvent_t);
template hipError_t launch_gram_dma<double>(const double*, int, uint64_t, uint64_t, int, const GramPlan&, double*,
                                            double*, double*, double*, hipStream_t, hipEvent_t);

}  // namespace tk
