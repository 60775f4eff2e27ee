// Mode-n product Z_(n) = M Y_(n) (Sec. 2.2.3, Alg. 3) with FP64 products, for
// more than 64 output rows, on the strided unfolding (element (j, c = l + L m)
// of Y_(n) at l + L j + L J m, element (k, c) of Z_(n) at l + L k + L K m).
//
// Work items: a tile of 128 output rows k by 128 columns c, over the whole
// reduction J in chunks of 16.  The row tiles of one column tile are
// consecutive items (same XCD), so their reads of the same Y chunks meet in
// L2 and Y comes from HBM about once.  Four waves per workgroup, each holding
// 64 x 64 of the tile as 4 x 4 blocks of 16 x 16 in FP64 MFMA accumulators
// (v_mfma_f64_16x16x4f64): a step of four j reads 8 operands from LDS for 16
// MFMAs.  The MFMA's output rows are k (A = M, B = Y) when L > 1, so that a
// lane group stores 16 consecutive columns, and c (A = Y^T, B = M^T) when
// L = 1, so that it stores 16 consecutive rows k; both are contiguous in Z.
//
// Staging: both operands' chunk images (ttm_dma.hpp) are written straight
// from global memory into LDS (global_load_lds, 16 bytes per lane), double
// buffered; two workgroups fit on a CU.  Rows past K and columns past the end
// are not loaded (their outputs are not stored); indices j >= J of the last
// chunk are zeroed in both images.  Every lane's load addresses are a fixed
// per-lane offset plus a per-instruction offset common to the wave.
#include "common.hpp"
#include "kernels.hpp"
#include "ttm_dma.hpp"

namespace tk {

namespace {

using tdma::kJC;
using tdma::TImg;

constexpr int kTDW = 4;   // waves per workgroup
constexpr int kTDNT = 256;

typedef __attribute__((address_space(3))) void lds_void;

struct TtmDmaParams {
  const char* Y;
  const char* M;
  char* Z;
  int J, K;
  int64_t L, cols;
  int64_t msk, msj;   // M(k, j) at M + k msk + j msj (doubles)
  int64_t nkt, total;
  int64_t Lo;          // L of the output (L unless remapped)
  int64_t Lp, Pp, Rp;  // output remap (TtmOutRemap); Pp == Rp: none
};

// ORI 0 (L > 1): A = M (row form MF = 0, column form MF = 1), B = Y (column
// form).  ORI 1 (L = 1): A = Y (row form), B = M.
// WY: bytes per lane of the Y loads, 16, or 4 where Y's rows or columns are
// only 8-byte aligned (odd L or J); M is always loaded in 16-byte units.
template <typename TY, int ORI, int MF, int WY>
struct Cfg {
  using IM = TImg<MF == 0 ? 0 : 1, 8>;
  using IY = TImg<ORI == 0 ? 1 : 0, sizeof(TY)>;
  static constexpr int MB = IM::BYTES, YB = IY::BYTES;
  static constexpr int BUF = MB + YB;  // one chunk: M image then Y image
  static constexpr int NIM = MB / 1024, NIY = YB / (64 * WY);  // load instructions per image
  static_assert(WY == 16 || sizeof(TY) == 8, "4-byte loads for double input only");
};

// Per-lane state of the loads of one item (tile at output row k0, column
// c0).  The wave issues instructions jj = w, w + 4, ... of each image; a
// lane's load address is a per-lane part fixed for the item plus a
// per-instruction part common to the wave:
//   16-byte loads: in the column form the lane's rows are the same for all of
//     the wave's instructions (the swizzle of j = w + 4 n depends on w only),
//     in the row form they move by 8 rows per instruction;
//   4-byte loads (256 bytes per instruction; Y only): column form, j = n and
//     the lane's rows alternate between two sets with the swizzle of j (bit 1
//     of n); row form, 2 rows per instruction (8 more per n) and the lane's j
//     alternate between two values with the row pair's swizzle (bit 0 of n).
template <typename TY, int ORI, int MF, int WY>
struct Loader {
  const char* mlane;   // M(k0 + mrow0, 0)
  const char* ylane;   // Y(0, c0 + yrow0) (16-byte loads, 4-byte row form)
  const char* ycol0;   // 4-byte column form: Y(0, c0 + yr0) with the lane's byte,
  const char* ycol1;   // and for the other swizzle pattern
  int64_t mjstride;    // M bytes per reduction index j
  int64_t yjstride;    // Y bytes per j
  int64_t c0;
  int k0, mrow0, yrow0;
  int yr0, yr1, yj0, yj1;  // 4-byte loads: rows (column form) or j (row form) per pattern
};

template <typename TY, int ORI, int MF, int WY>
__device__ __forceinline__ void loader_init(Loader<TY, ORI, MF, WY>& ld, const TtmDmaParams& g, int k0, int64_t c0,
                                            int wave, int lane) {
  using C = Cfg<TY, ORI, MF, WY>;
  ld.k0 = k0;
  ld.c0 = c0;
  int r, j;
  C::IM::unit_of(wave, lane, r, j);
  ld.mrow0 = r;
  ld.mlane = g.M + (int64_t)(k0 + r) * g.msk * 8;
  ld.mjstride = g.msj * 8;
  ld.yjstride = (ORI == 0) ? g.L * (int64_t)sizeof(TY) : (int64_t)sizeof(TY);
  // column c of the unfolding sits at l + L J m (clamped into the tensor;
  // lanes past the end issue nothing)
  auto colbase = [&](int rr) {
    const int64_t c = min(c0 + rr, g.cols - 1);
    const int64_t m = c / g.L, l = c - m * g.L;
    return g.Y + (l + g.L * (int64_t)g.J * m) * (int64_t)sizeof(TY);
  };
  if constexpr (WY == 16) {
    C::IY::unit_of(wave, lane, r, j);
    ld.yrow0 = r;
    if constexpr (ORI == 0) ld.ylane = colbase(r);
    else ld.ylane = g.Y + min(c0 + r, g.cols - 1) * g.J * (int64_t)sizeof(TY);
  } else if constexpr (ORI == 0) {
    // column form, 1024 bytes per j: instruction w + 4 n covers quarter w of j = n
    const int u = 16 * wave + (lane >> 2);
    ld.yr0 = 2 * u + ((lane & 3) >> 1);
    ld.yr1 = 2 * (u ^ 8) + ((lane & 3) >> 1);
    ld.ycol0 = colbase(ld.yr0) + (lane & 1) * 4;
    ld.ycol1 = colbase(ld.yr1) + (lane & 1) * 4;
  } else {
    // row form, 2 rows of 128 bytes per instruction: rows 2 w + 8 n + (lane >> 5)
    ld.yrow0 = 2 * wave + (lane >> 5);
    ld.ylane = g.Y + min(c0 + ld.yrow0, g.cols - 1) * g.J * (int64_t)sizeof(TY) + (lane & 1) * 4;
    const int pu = (lane & 31) >> 2;
    ld.yj0 = 2 * (pu ^ wave) + ((lane & 3) >> 1);
    ld.yj1 = 2 * (pu ^ wave ^ 4) + ((lane & 3) >> 1);
  }
}

// Loads chunk t (reduction indices 16 t ..) into buf: M image, then Y image.
template <typename TY, int ORI, int MF, int WY>
__device__ __forceinline__ void issue_chunk(const Loader<TY, ORI, MF, WY>& ld, const TtmDmaParams& g, int t, char* buf,
                                            int wave, int lane) {
  using C = Cfg<TY, ORI, MF, WY>;
  const int j0 = kJC * t;
#pragma unroll
  for (int n = 0; n < C::NIM / kTDW; ++n) {
    const int jj = wave + kTDW * n;
    int r, j;
    C::IM::unit_of(jj, lane, r, j);
    if (ld.k0 + r < g.K && j0 + j < g.J) {
      // rows of later instructions: row form moves 8 rows per instruction,
      // column form keeps the lane's rows
      const int64_t row_off = (MF == 0) ? (int64_t)(r - ld.mrow0) * g.msk * 8 : 0;
      const char* src = ld.mlane + row_off + (int64_t)(j0 + j) * ld.mjstride;
      __builtin_amdgcn_global_load_lds(static_cast<const void*>(src), (lds_void*)(buf + jj * 1024), 16, 0, 0);
    }
  }
  if constexpr (WY == 16) {
#pragma unroll
    for (int n = 0; n < C::NIY / kTDW; ++n) {
      const int jj = wave + kTDW * n;
      int r, j;
      C::IY::unit_of(jj, lane, r, j);
      if (ld.c0 + r < g.cols && j0 + j < g.J) {
        const int64_t row_off = (ORI == 1) ? (int64_t)(r - ld.yrow0) * g.J * (int64_t)sizeof(TY) : 0;
        const char* src = ld.ylane + row_off + (int64_t)(j0 + j) * ld.yjstride;
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(src), (lds_void*)(buf + C::MB + jj * 1024), 16,
                                         0, 0);
      }
    }
  } else {
    // 4-byte loads, 16 instructions per wave, rolled in pairs (the lane
    // pattern is selected per instruction)
#pragma unroll 2
    for (int n = 0; n < C::NIY / kTDW; ++n) {
      const int jj = wave + kTDW * n;
      if constexpr (ORI == 0) {
        const bool p = (n >> 1) & 1;
        if (ld.c0 + (p ? ld.yr1 : ld.yr0) < g.cols && j0 + n < g.J) {
          const char* src = (p ? ld.ycol1 : ld.ycol0) + (int64_t)(j0 + n) * ld.yjstride;
          __builtin_amdgcn_global_load_lds(static_cast<const void*>(src), (lds_void*)(buf + C::MB + jj * 256), 4, 0,
                                           0);
        }
      } else {
        const int yj = (n & 1) ? ld.yj1 : ld.yj0;
        if (ld.c0 + ld.yrow0 + 8 * n < g.cols && j0 + yj < g.J) {
          const char* src = ld.ylane + (int64_t)(8 * n) * g.J * (int64_t)sizeof(TY) + (int64_t)(j0 + yj) * 8;
          __builtin_amdgcn_global_load_lds(static_cast<const void*>(src), (lds_void*)(buf + C::MB + jj * 256), 4, 0,
                                           0);
        }
      }
    }
  }
}

// Zeros the elements of indices j >= J in both images of the last chunk.
// Each wave clears the slots of its own load instructions (loaded or not),
// once its loads have landed, so that no load of another wave can land on a
// cleared element afterwards.
template <typename TY, int ORI, int MF, int WY>
__device__ __forceinline__ void fill_chunk(const Loader<TY, ORI, MF, WY>& ld, const TtmDmaParams& g, int t,
                                           char* buf, int wave, int lane) {
  using C = Cfg<TY, ORI, MF, WY>;
  const int j0 = kJC * t;
  if (j0 + kJC <= g.J) return;
  (void)ld;
  // M: 16-byte units of two doubles; the row form's two elements have j, j + 1
#pragma unroll
  for (int n = 0; n < C::NIM / kTDW; ++n) {
    const int jj = wave + kTDW * n;
    int r, j;
    C::IM::unit_of(jj, lane, r, j);
    double* e = reinterpret_cast<double*>(buf + jj * 1024 + lane * 16);
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (j0 + j + (MF == 0 ? h : 0) >= g.J) e[h] = 0.0;
  }
  constexpr int ES = sizeof(TY);
#pragma unroll
  for (int n = 0; n < C::NIY / kTDW; ++n) {
    const int jj = wave + kTDW * n;
    if constexpr (WY == 16) {
      int r, j;
      C::IY::unit_of(jj, lane, r, j);
      TY* e = reinterpret_cast<TY*>(buf + C::MB + jj * 1024 + lane * 16);
#pragma unroll
      for (int h = 0; h < 16 / ES; ++h)
        if (j0 + j + (ORI == 1 ? h : 0) >= g.J) e[h] = (TY)0;
    } else {
      const int jl = (ORI == 0) ? n : ((n & 1) ? ld.yj1 : ld.yj0);
      if (j0 + jl >= g.J) *reinterpret_cast<uint32_t*>(buf + C::MB + jj * 256 + lane * 4) = 0u;
    }
  }
}

// Operand reads of one lane for its four blocks (16 rows each) of an image,
// one step ahead of the MFMAs.  Row form: one 16-byte unit per block serves
// steps 2 g and 2 g + 1, at o[x] (g = 0) or o[x] + d (g = 1); column form:
// step s at o[x] + (s & 1) CB + 8 (s >> 1) CB.
template <int FORM, typename T>
struct Opnd;

template <typename T>
struct Opnd<0, T> {  // row form (doubles)
  double2 u[4];
  __device__ __forceinline__ void fetch(const char* img, const int (&o)[4], int d, int s) {
    if ((s & 1) == 0) {
#pragma unroll
      for (int x = 0; x < 4; ++x) u[x] = *reinterpret_cast<const double2*>(img + o[x] + (s ? d : 0));
    }
  }
  __device__ __forceinline__ double get(int x, int s) const { return (s & 1) ? u[x].y : u[x].x; }
};

template <typename T>
struct Opnd<1, T> {  // column form
  static constexpr int CB = tdma::kRows * (int)sizeof(T);
  T v[4];
  __device__ __forceinline__ void fetch(const char* img, const int (&o)[4], int, int s) {
#pragma unroll
    for (int x = 0; x < 4; ++x) v[x] = *reinterpret_cast<const T*>(img + o[x] + (s & 1) * CB + (s >> 1) * 8 * CB);
  }
  __device__ __forceinline__ double get(int x, int) const { return (double)v[x]; }
};

// One chunk of MFMAs (four steps of four j).  MK: compile-time block mask.
// `half`: the chunk holds at most 8 valid j (the last chunk of a ragged J),
// which steps 0 and 1 cover (j(s, q) = 2 q + (s & 1) + 8 (s >> 1)), so steps
// 2 and 3 would only multiply zeros.
template <unsigned MK, int FA, typename TA, int FB, typename TB>
__device__ __forceinline__ void compute_chunk(const char* abuf, const char* bbuf, const int (&oa)[4], int da,
                                              const int (&ob)[4], int db, d4 (&acc)[4][4], bool half = false) {
  Opnd<FA, TA> a[2];
  Opnd<FB, TB> b[2];
  a[0].fetch(abuf, oa, da, 0);
  b[0].fetch(bbuf, ob, db, 0);
#pragma unroll
  for (int s = 0; s < kJC / 4; ++s) {
    if (s >= 2 && half) break;  // uniform
    // the row form's unit of step s (odd) is the one fetched for step s - 1
    const int cur = (FA == 0) ? (s >> 1) & 1 : s & 1;
    const int curb = (FB == 0) ? (s >> 1) & 1 : s & 1;
    if (s + 1 < kJC / 4) {
      if (FA == 1 || ((s + 1) & 1) == 0) a[(FA == 0) ? ((s + 1) >> 1) & 1 : (s + 1) & 1].fetch(abuf, oa, da, s + 1);
      if (FB == 1 || ((s + 1) & 1) == 0) b[(FB == 0) ? ((s + 1) >> 1) & 1 : (s + 1) & 1].fetch(bbuf, ob, db, s + 1);
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y)
        if ((MK >> (4 * x + y)) & 1u)
          acc[x][y] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur].get(x, s), b[curb].get(y, s), acc[x][y], 0, 0, 0);
  }
}

template <unsigned MK, typename TY, int ORI, int MF, int WY>
__device__ __forceinline__ void chunk_loop(const Loader<TY, ORI, MF, WY>& ld, const TtmDmaParams& g, char* buf0,
                                           char* buf1, const int (&oa)[4], int da, const int (&ob)[4], int db,
                                           d4 (&acc)[4][4], int wave, int lane, int tid) {
  using C = Cfg<TY, ORI, MF, WY>;
  // A and B operand images: forms, element types and offsets in a buffer
  constexpr int FM = (MF == 0) ? 0 : 1, FY = (ORI == 0) ? 1 : 0;
  constexpr int FA = (ORI == 0) ? FM : FY, FB = (ORI == 0) ? FY : FM;
  using TA = typename std::conditional<ORI == 0, double, TY>::type;
  using TB = typename std::conditional<ORI == 0, TY, double>::type;
  constexpr int AOFF = (ORI == 0) ? 0 : C::MB, BOFF = (ORI == 0) ? C::MB : 0;
  const int nch = (g.J + kJC - 1) / kJC;
  const bool last_half = g.J - kJC * (nch - 1) <= kJC / 2;
  issue_chunk(ld, g, 0, buf0, wave, lane);
  __builtin_amdgcn_s_waitcnt(0);
  fill_chunk(ld, g, 0, buf0, wave, lane);
  __syncthreads();
  for (int t = 0;; t += 2) {
    if (t + 1 < nch) issue_chunk(ld, g, t + 1, buf1, wave, lane);
    compute_chunk<MK, FA, TA, FB, TB>(buf0 + AOFF, buf0 + BOFF, oa, da, ob, db, acc, last_half && t + 1 == nch);
    if (t + 1 >= nch) break;
    __builtin_amdgcn_s_waitcnt(0);
    fill_chunk(ld, g, t + 1, buf1, wave, lane);
    __syncthreads();
    if (t + 2 < nch) issue_chunk(ld, g, t + 2, buf0, wave, lane);
    compute_chunk<MK, FA, TA, FB, TB>(buf1 + AOFF, buf1 + BOFF, oa, da, ob, db, acc, last_half && t + 2 == nch);
    if (t + 2 >= nch) break;
    __builtin_amdgcn_s_waitcnt(0);
    fill_chunk(ld, g, t + 2, buf0, wave, lane);
    __syncthreads();
  }
}

// Stores the wave's blocks of the tile.  MFMA result: lane l, register v ->
// D[(l >> 4) + 4 v][l & 15].
template <unsigned MK, typename TZ, int ORI>
__device__ __forceinline__ void store_tile(const TtmDmaParams& g, const d4 (&acc)[4][4], int k0, int64_t c0l,
                                           int a0, int b0, int i, int q) {
  TZ* __restrict__ Z = reinterpret_cast<TZ*>(g.Z);
  if constexpr (ORI == 0) {
    // D rows k = k0 + 16 (a0 + 2 x) + q + 4 v, columns c = c0 + 16 (b0 + y) + i
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int64_t c = c0l + 16 * (b0 + y) + i;
      if (c >= g.cols) continue;
      const int64_t m = c / g.L, l = c - m * g.L;
      int64_t lo = l;
      bool zpad = false;  // also write the appended zero slice after this one
      if (g.Pp != g.Rp) {  // uniform
        const int64_t t = l / g.Lp, a = l - t * g.Lp;
        const int64_t h = t / g.Pp, ip = t - h * g.Pp;
        if (ip >= g.Rp) continue;  // a zero slice of the padded mode
        lo = a + g.Lp * (ip + g.Rp * h);
        zpad = g.Rp > g.Pp && ip == g.Pp - 1;
      }
      TZ* zc = Z + lo + g.Lo * (int64_t)g.K * m;
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        if (!((MK >> (4 * x + y)) & 1u)) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = k0 + 16 * (a0 + 2 * x) + q + 4 * v;
          if (k < g.K) {
            zc[g.Lo * (int64_t)k] = static_cast<TZ>(acc[x][y][v]);
            if (zpad) zc[g.Lp + g.Lo * (int64_t)k] = static_cast<TZ>(0.0);
          }
        }
      }
    }
  } else {
    // D rows c = c0 + 16 (a0 + x) + q + 4 v, columns k = k0 + 16 (b0 + 2 y) + i
#pragma unroll
    for (int x = 0; x < 4; ++x) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t c = c0l + 16 * (a0 + x) + q + 4 * v;
        if (c >= g.cols) continue;
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          if (!((MK >> (4 * x + y)) & 1u)) continue;
          const int k = k0 + 16 * (b0 + 2 * y) + i;
          if (k < g.K) Z[k + (int64_t)g.K * c] = static_cast<TZ>(acc[x][y][v]);
        }
      }
    }
  }
}

// The whole item for one block mask class: accumulators zeroed, all chunks,
// then the stores (one copy per class, so that no accumulator is merged
// across classes).
template <unsigned MK, typename TY, typename TZ, int ORI, int MF, int WY>
__device__ __forceinline__ void tile_body(const Loader<TY, ORI, MF, WY>& ld, const TtmDmaParams& g, char* buf0,
                                          char* buf1, const int (&oa)[4], int da, const int (&ob)[4], int db,
                                          int wave, int lane, int tid, int k0, int64_t c0l, int a0, int b0) {
  d4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  chunk_loop<MK>(ld, g, buf0, buf1, oa, da, ob, db, acc, wave, lane, tid);
  store_tile<MK, TZ, ORI>(g, acc, k0, c0l, a0, b0, lane & 15, lane >> 4);
}

template <typename TY, typename TZ, int ORI, int MF, int WY>
__global__ __launch_bounds__(kTDNT, 2) void ttm_dma_kernel(TtmDmaParams g) {
  using C = Cfg<TY, ORI, MF, WY>;
  __shared__ __attribute__((aligned(16))) char buf0[C::BUF];
  __shared__ __attribute__((aligned(16))) char buf1[C::BUF];
  const int64_t item = xcd_remap(blockIdx.x, gridDim.x, g.total);
  if (item < 0) return;
  const int64_t ct = item / g.nkt;
  const int k0 = 128 * (int)(item - ct * g.nkt);
  const int64_t c0l = 128 * ct;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i = lane & 15, q = lane >> 4;

  Loader<TY, ORI, MF, WY> ld;
  loader_init(ld, g, k0, c0l, wave, lane);

  // the wave's 64 x 64 part of the tile's 8 x 8 blocks of 16 x 16: along the
  // output rows k the waves take every other block (blocks kw, kw + 2,
  // kw + 4, kw + 6), along the columns four consecutive ones, so that a
  // ragged last row tile (K = 469: six blocks; 448: four) splits evenly
  // between the two waves of a column half instead of leaving one idle.
  // ORI 0: A blocks a0 + 2 x (k), B blocks b0 + y (c); ORI 1: A blocks
  // a0 + x (c), B blocks b0 + 2 y (k).
  const int a0 = (ORI == 0) ? (wave >> 1) : 4 * (wave >> 1);
  const int b0 = (ORI == 0) ? 4 * (wave & 1) : (wave & 1);
  // output rows k beyond K drop this wave's last k blocks: ORI 0 A block
  // rows, ORI 1 B block columns
  const int kw = (ORI == 0) ? a0 : b0;
  const int nbk = min(8, (g.K - k0 + 15) / 16);
  const int nv = max(0, min(4, (nbk - kw + 1) / 2));
  const unsigned mask = (ORI == 0) ? tdma::rows_mask(nv) : tdma::cols_mask(nv);
  // operand offsets of the lane's blocks at step 0 (row form: and the byte
  // distance d to its second unit, whose sign depends on the row's swizzle)
  int oa[4], ob[4], da = 0, db = 0;
  {
    using IA = typename std::conditional<ORI == 0, typename C::IM, typename C::IY>::type;
    using IB = typename std::conditional<ORI == 0, typename C::IY, typename C::IM>::type;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      oa[t] = IA::at(16 * (a0 + (ORI == 0 ? 2 : 1) * t) + i, IA::jstep(0, q));
      ob[t] = IB::at(16 * (b0 + (ORI == 0 ? 1 : 2) * t) + i, IB::jstep(0, q));
    }
    da = IA::at(i, IA::jstep(2, q)) - IA::at(i, IA::jstep(0, q));
    db = IB::at(i, IB::jstep(2, q)) - IB::at(i, IB::jstep(0, q));
  }
#define TDMA_LOOP(MK) \
  tile_body<MK, TY, TZ, ORI, MF, WY>(ld, g, buf0, buf1, oa, da, ob, db, wave, lane, tid, k0, c0l, a0, b0)
  if constexpr (ORI == 0) {
    if (mask == 0xFFFFu) TDMA_LOOP(0xFFFFu);
    else if (mask == 0x0FFFu) TDMA_LOOP(0x0FFFu);
    else if (mask == 0x00FFu) TDMA_LOOP(0x00FFu);
    else if (mask == 0x000Fu) TDMA_LOOP(0x000Fu);
    else TDMA_LOOP(0u);
  } else {
    if (mask == 0xFFFFu) TDMA_LOOP(0xFFFFu);
    else if (mask == 0x7777u) TDMA_LOOP(0x7777u);
    else if (mask == 0x3333u) TDMA_LOOP(0x3333u);
    else if (mask == 0x1111u) TDMA_LOOP(0x1111u);
    else TDMA_LOOP(0u);
  }
#undef TDMA_LOOP
}

}  // namespace

// 16-byte loads of Y need its rows (L = 1: stride J) or slabs (L > 1: the
// element offset L j) 16-byte aligned; otherwise double input takes 4-byte
// loads.
static bool ttm_dma_y16(int J, uint64_t L, int ysize, const void* Y) {
  if (reinterpret_cast<uintptr_t>(Y) % 16) return false;
  if (L == 1) return ((uint64_t)J * ysize) % 16 == 0;
  return L % (16 / ysize) == 0;
}

bool ttm_dma_eligible(int J, uint64_t L, uint64_t cols, int K, int64_t msk, int64_t msj, int ysize, int zsize,
                      const void* Y, const void* M) {
  if (K <= 64 || J < 16 || cols == 0) return false;
  if (reinterpret_cast<uintptr_t>(M) % 16 || reinterpret_cast<uintptr_t>(Y) % ysize) return false;
  // M: rows contiguous (msj = 1, row stride a multiple of 16 bytes) or
  // columns contiguous (msk = 1, column stride likewise)
  const bool mrow = (msj == 1 && msk % 2 == 0), mcol = (msk == 1 && msj % 2 == 0);
  if (!mrow && !mcol) return false;
  if (ysize == 4) {
    // float input: 16-byte loads only, slabs of L > 1, the factor of a
    // compression (rows of M contiguous) and double output
    return L > 1 && ttm_dma_y16(J, L, ysize, Y) && mrow && zsize == 8;
  }
  return true;
}

template <typename TY, typename TZ>
hipError_t launch_ttm_dma(const TY* Y, int J, uint64_t L, uint64_t cols, const double* M, int64_t msk, int64_t msj,
                          int K, TZ* Z, hipStream_t stream, const TtmOutRemap& rm) {
  if (!ttm_dma_eligible(J, L, cols, K, msk, msj, (int)sizeof(TY), (int)sizeof(TZ), Y, M))
    return hipErrorInvalidValue;
  const bool remap = rm.Pp != rm.Rp;
  if (remap && (L == 1 || rm.Lp < 1 || rm.Rp < 1 || rm.Rp > rm.Pp + 1 || (int64_t)L % (rm.Lp * rm.Pp) != 0))
    return hipErrorInvalidValue;
  TtmDmaParams g{};
  g.Y = reinterpret_cast<const char*>(Y);
  g.M = reinterpret_cast<const char*>(M);
  g.Z = reinterpret_cast<char*>(Z);
  g.J = J;
  g.K = K;
  g.L = (int64_t)L;
  g.cols = (int64_t)cols;
  g.msk = msk;
  g.msj = msj;
  g.nkt = ceil_div(K, 128);
  g.total = g.nkt * ceil_div((int64_t)cols, 128);
  g.Lp = remap ? rm.Lp : 1;
  g.Pp = remap ? rm.Pp : 1;
  g.Rp = remap ? rm.Rp : 1;
  g.Lo = remap ? (int64_t)L / rm.Pp * rm.Rp : (int64_t)L;
  const int64_t grid = ceil_div(g.total, kXcds) * kXcds;
  const bool mrow = (msj == 1 && msk % 2 == 0);
  const bool y16 = ttm_dma_y16(J, L, (int)sizeof(TY), Y);
#define TDMA(TYV, ORI, MF, WYV) \
  hipLaunchKernelGGL((ttm_dma_kernel<TYV, TZ, ORI, MF, WYV>), dim3(grid), dim3(kTDNT), 0, stream, g)
#define TDMA_W(ORI, MF)               \
  do {                                \
    if (y16) TDMA(double, ORI, MF, 16); \
    else TDMA(double, ORI, MF, 4);      \
  } while (0)
  if constexpr (std::is_same<TY, float>::value) {
    if constexpr (std::is_same<TZ, double>::value) TDMA(float, 0, 0, 16);
    else return hipErrorInvalidValue;  // excluded by ttm_dma_eligible
  } else {
    if (L == 1) {
      if (mrow) TDMA_W(1, 0);
      else TDMA_W(1, 1);
    } else {
      if (mrow) TDMA_W(0, 0);
      else TDMA_W(0, 1);
    }
  }
#undef TDMA_W
#undef TDMA
  return hipGetLastError();
}

template hipError_t launch_ttm_dma<double, double>(const double*, int, uint64_t, uint64_t, const double*, int64_t,
                                                   int64_t, int, double*, hipStream_t, const TtmOutRemap&);
template hipError_t launch_ttm_dma<float, double>(const float*, int, uint64_t, uint64_t, const double*, int64_t,
                                                  int64_t, int, double*, hipStream_t, const TtmOutRemap&);
template hipError_t launch_ttm_dma<double, float>(const double*, int, uint64_t, uint64_t, const double*, int64_t,
                                                  int64_t, int, float*, hipStream_t, const TtmOutRemap&);
template hipError_t launch_ttm_dma<float, float>(const float*, int, uint64_t, uint64_t, const double*, int64_t,
                                                 int64_t, int, float*, hipStream_t, const TtmOutRemap&);

}  // namespace tk
