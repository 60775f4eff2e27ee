// Index maps of the LDS chunk images used by the FP64 mode-product kernel
// (ttm_dma.hip).  Host and device code: the kernel uses them to place and
// read elements; a host build can replay the same maps.
//
// Z_(n) = M Y_(n) is computed in tiles of 128 output rows k by 128 columns c
// of the unfolding, over chunks of 16 reduction indices j.  Per chunk each
// operand is held in LDS as an image of 128 "rows" (k for M, c for Y) by 16
// j, in 16-byte units (E = 16 / sizeof(T) elements per unit), in one of two
// forms:
//   row form (doubles only): 128 bytes per row; unit u (j = 2u, 2u + 1) of
//     row r stored at unit position u ^ ((r >> 1) & 7);
//   column form: per j, the 128 rows' elements (128 sizeof(T) bytes); unit u
//     (rows E u .. E u + E - 1) of column j stored at u ^ sw(j).
// The reduction index of MFMA step s (of 4) in lane group q is
// j(s, q) = 2 q + (s & 1) + 8 (s >> 1), the same for both operands: in the
// row form a lane then reads one 16-byte unit (unit q, then q | 4) for two
// steps, and in the column form the swizzle sw(j) = ((j >> 1) & 1) << 3
// (doubles) or ((j >> 1) & 3) << 2 (floats) depends on q only, so that the
// four lane groups read distinct banks and a step moves by a fixed offset.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace tk {
namespace tdma {

constexpr int kRows = 128;  // rows of an image (output rows or columns of a tile)
constexpr int kJC = 16;     // reduction indices per chunk

template <int FORM, int ES>
struct TImg {
  static_assert(FORM == 1 || ES == 8, "the row form holds doubles");
  static constexpr int E = 16 / ES;
  static constexpr int BYTES = kRows * kJC * ES;  // 16 KB (doubles) or 8 KB (floats)
  static constexpr int CB = kRows * ES;           // column form: bytes per j

  __host__ __device__ static constexpr int sw(int j) { return ES == 8 ? (((j >> 1) & 1) << 3) : (((j >> 1) & 3) << 2); }

  // Reduction index of MFMA step s in lane group q.
  __host__ __device__ static constexpr int jstep(int s, int q) { return 2 * q + (s & 1) + 8 * (s >> 1); }

  // Byte offset of element (row r, reduction index j).
  __host__ __device__ static int at(int r, int j) {
    if (FORM == 0) return r * 128 + (((j / E) ^ ((r >> 1) & 7)) << 4) + (j % E) * ES;
    return j * CB + (((r / E) ^ sw(j)) << 4) + (r % E) * ES;
  }

  // The first element (row r, index j) of the unit that lane `lane` of
  // instruction jj (covering bytes [1024 jj, 1024 jj + 1024)) loads.
  __host__ __device__ static void unit_of(int jj, int lane, int& r, int& j) {
    const int P = jj * 1024 + lane * 16;
    if (FORM == 0) {
      r = P >> 7;
      j = (((P & 127) >> 4) ^ ((r >> 1) & 7)) * E;
    } else {
      j = P / CB;
      r = ((((P % CB) >> 4) ^ sw(j))) * E;
    }
  }
};

// Block masks of a wave's 4 x 4 grid of 16 x 16 blocks (bit 4 x + y): the
// first nv block rows (x < nv) or block columns (y < nv).
__host__ __device__ inline unsigned rows_mask(int nv) { return nv >= 4 ? 0xFFFFu : ((1u << (4 * nv)) - 1u); }
__host__ __device__ inline unsigned cols_mask(int nv) {
  const unsigned c = nv >= 4 ? 0xFu : ((1u << nv) - 1u);
  return c | (c << 4) | (c << 8) | (c << 12);
}

}  // namespace tdma
}  // namespace tk
