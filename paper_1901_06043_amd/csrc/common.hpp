// Internal helpers shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Number of XCDs on MI355X.  Workgroups are dispatched to XCDs round-robin by
// linear workgroup id, so id w runs on XCD (w % 8).
constexpr int kXcds = 8;

// Remap a linear workgroup id so that work items with consecutive indices land
// on the same XCD (and therefore share its L2).  `total` work items are spread
// over `grid` >= total workgroups, grid a multiple of kXcds; returns -1 for
// workgroups with no work.
__device__ __forceinline__ int64_t xcd_remap(int64_t w, int64_t grid, int64_t total) {
  const int64_t per = grid / kXcds;
  const int64_t item = (w % kXcds) * per + (w / kXcds);
  return item < total ? item : -1;
}

// Workgroup barrier that orders LDS only: unlike __syncthreads() it does not
// wait for the wave's outstanding global-memory stores to complete.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__host__ __device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T>
__device__ __forceinline__ double to_f64(T v) {
  return static_cast<double>(v);
}

// DPP lane permutation of a double (two 32-bit DPP moves).
template <int CTRL>
__device__ __forceinline__ double dpp64(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over each row of 16 lanes with VALU-only DPP steps: quad_perm xor 1,
// quad_perm xor 2, half-row mirror, row mirror.  Every step adds two partial
// sums that are bit-identical in the partner lanes, so all 16 lanes end with
// the same rounded total.
__device__ __forceinline__ double row16_sum(double x) {
  x += dpp64<0xB1>(x);
  x += dpp64<0x4E>(x);
  x += dpp64<0x141>(x);
  x += dpp64<0x140>(x);
  return x;
}

// Wave-wide (64 lanes) sum with butterfly shuffles; every lane gets the sum.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Wave-wide sum without LDS: 16-lane DPP reduction, then the gfx950 permlane
// swaps.  permlane16_swap of a value returns the pair (rows 0,0,2,2 ; rows
// 1,1,3,3) and permlane32_swap the pair (lanes 0-31 twice ; lanes 32-63
// twice), so adding each pair sums rows 0+1 and 2+3, then the two halves.
// Every lane gets the same (bit-identical) total.
__device__ __forceinline__ double swap_add16(double v) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double swap_add32(double v) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double wave_sum_fast(double v) { return swap_add32(swap_add16(row16_sum(v))); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of p[0], p[stride], ..., p[(n - 1) stride] in a fixed order: eight
// running sums (term s goes to sum s % 8), combined pairwise, so that eight
// loads are in flight instead of one.
__device__ __forceinline__ double sum_strided8(const double* __restrict__ p, int64_t n, int64_t stride) {
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t i = 0;
  for (; i + 8 <= n; i += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += p[(i + u) * stride];
  }
#pragma unroll
  for (int u = 0; u < 8; ++u)
    if (i + u < n) s[u] += p[(i + u) * stride];
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

}  // namespace tk
