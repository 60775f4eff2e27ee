// Index maps of the LDS chunk images used by the FP64 tile-pair Gram kernel
// (gram_dma.hip).  Host and device code: the kernel uses them to place and
// read elements; a host build can replay the same maps.
//
// A chunk of the mode-n unfolding Y_(n) (Sec. 4.2: element (row a, column
// c = l + L*m) at l + L*a + L*J*m) covers KC columns: 128 / sizeof(T) (128
// bytes of a row), except 20 for doubles with unit stride (five MFMA steps
// per chunk; the column images need no power-of-two count).  For each 128-row
// tile the chunk is held in LDS as an image of TB = 128 KC sizeof(T) bytes in
// 16-byte units (E = 16 / sizeof(T) elements per unit):
//   layout 0 (L = 1, columns contiguous): column-major, 128 * sizeof(T) bytes
//     per column; unit u (rows E u .. E u + E - 1) of column k is stored at
//     unit position u ^ sw(k), with sw(k) = (k & 1) << 3 for doubles and
//     (k & 3) << 2 for floats;
//   layout 1 (L > 1, row segments contiguous): row-major, 128 bytes per row;
//     unit u (columns E u .. E u + E - 1) of row r is stored at u ^ ((r >> 1) & 7).
// The XOR swizzles make the MFMA operand reads of a wave conflict-free:
//   layout 0: lane (i, q) reads row 16 b + i of column 4 s + q, so the four
//     lane groups q read four columns whose swizzles differ;
//   layout 1: lane (i, q) reads unit q (then q | 4) of row 16 b + i, and the
//     16 rows of a block land on 16 distinct 16-byte bank windows.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace tk {
namespace dma {

constexpr int kTileRows = 128;

template <int ES, int LAY>
struct Img {
  static constexpr int E = 16 / ES;                               // elements per unit
  static constexpr int KC = (LAY == 0 && ES == 8) ? 20 : 128 / ES;  // columns per chunk
  static constexpr int CB = 128 * ES;                             // layout 0: bytes per column image
  static constexpr int TB = 128 * KC * ES;                        // bytes per tile image

  __host__ __device__ static constexpr int sw(int k) { return ES == 8 ? ((k & 1) << 3) : ((k & 3) << 2); }

  // Byte offset within the tile image of element (row r, column c).
  __host__ __device__ static int at(int r, int c) {
    if (LAY == 0) return c * CB + (((r / E) ^ sw(c)) << 4) + (r % E) * ES;
    return r * 128 + (((c / E) ^ ((r >> 1) & 7)) << 4) + (c % E) * ES;
  }

  // Inverse: the element (row r, column c) and byte b within it stored at
  // byte P of the tile image.
  __host__ __device__ static void inv(int P, int& r, int& c, int& b) {
    if (LAY == 0) {
      const int k = P / CB, w = P % CB;
      const int u = (w >> 4) ^ sw(k);
      r = u * E + (w & 15) / ES;
      c = k;
      b = (w & 15) % ES;
    } else {
      const int rr = P >> 7, w = P & 127;
      const int u = (w >> 4) ^ ((rr >> 1) & 7);
      r = rr;
      c = u * E + (w & 15) / ES;
      b = (w & 15) % ES;
    }
  }

  // Column read by lane group q at MFMA step s of a chunk (the same map for
  // both operands, so any bijection of (s, q) onto the KC columns is valid):
  //   layout 0: column 4 s + q;
  //   layout 1: element s % E of unit q (s < E) or unit q | 4 (s >= E).
  __host__ __device__ static int col(int s, int q) {
    if (LAY == 0) return 4 * s + q;
    return (s < E ? q : (q | 4)) * E + (s % E);
  }
};

// Triangle index of block (bi, bj), bi <= bj, among the upper-triangle blocks
// of an 8 x 8 block tile enumerated row by row.
__host__ __device__ inline int tri_index(int bi, int bj) { return bi * 8 - bi * (bi - 1) / 2 + (bj - bi); }

// Block masks of a wave's 4 x 4 block grid (bit 4 x + y for block (x, y)).
constexpr unsigned kMaskFull = 0xFFFFu;
constexpr unsigned kMaskUpper = 0x8CEFu;  // x <= y
constexpr unsigned kMaskHalf = 0x3333u;   // y < 2
constexpr unsigned kMaskCol1 = 0x1111u;   // y = 0

// The part of a tile pair's 8 x 8 blocks of 16 x 16 that wave w (of 4)
// computes: blocks (a0 + x, b0 + bs y) of the pair's A and B tiles for the
// bits 4 x + y set in mask.  Off-diagonal pairs: wave w takes the A blocks
// 4 (w >> 1) .. + 3 and every other B block from w & 1 (bs = 2), so that a
// ragged last B tile (J = 672: two blocks) gives each wave the same share
// instead of leaving two waves idle.  Diagonal pairs need the upper triangle
// (36 blocks, bs = 1): waves 0 and 2 take the upper 10 blocks of the diagonal
// 4 x 4 grids, waves 1 and 3 the two 4 x 2 halves of the off-diagonal one.
// Blocks whose rows lie at or beyond J are dropped.
__host__ __device__ inline void wave_task(int w, bool diag, int ra, int rb, int J, int& a0, int& b0, int& bs,
                                          unsigned& mask) {
  if (!diag) {
    a0 = 4 * (w >> 1);
    b0 = w & 1;
    bs = 2;
    mask = kMaskFull;
  } else if (w == 0 || w == 2) {
    a0 = b0 = 2 * w;
    bs = 1;
    mask = kMaskUpper;
  } else {
    a0 = 0;
    b0 = (w == 1) ? 4 : 6;
    bs = 1;
    mask = kMaskHalf;
  }
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; ++y)
      if (ra + 16 * (a0 + x) >= J || rb + 16 * (b0 + bs * y) >= J) mask &= ~(1u << (4 * x + y));
}

}  // namespace dma
}  // namespace tk
