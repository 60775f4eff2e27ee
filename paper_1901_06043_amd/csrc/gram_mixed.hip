// Gram matrix S = Y_(n) Y_(n)^T (Alg. 2) for the reduced-precision forms and
// for FP64 with large mode sizes.  Arithmetic forms:
//   FP64   : v_mfma_f64_16x16x4f64 with FP64 accumulation;
//   FP32   : v_mfma_f32_16x16x4f32 on FP32 values, FP32 accumulation over
//            one 32-column chunk, the chunk sum promoted to FP64;
//   BF16X3 : every FP32 value x is split into b0 = bf16(x), b1 = bf16(x - b0)
//            and a product x*y is formed as b1 c0 + b0 c1 + b0 c0 with
//            v_mfma_f32_16x16x32_bf16 (the split-product scheme of Henry,
//            Tang and Heinecke, ARITH 2019); FP32 accumulation over groups of
//            8 chunks (256 columns), FP64 across groups;
//   BF16X6 : adds a third piece b2 = bf16(x - b0 - b1) and the products
//            b1 c1, b0 c2, b2 c0, which removes the bias of BF16X3 (the
//            dropped b1 c1 term is a Gram matrix of residuals, hence positive
//            semidefinite); FP32 accumulation per chunk, FP64 across chunks.
// The sum of squares ||Y||^2 is always accumulated in FP64 from the values as
// loaded.
//
// Work decomposition.  Triangle mode (J <= 128): one workgroup covers the
// whole upper triangle of 16 x 16 blocks for its range of column chunks.
// Pair mode (J > 128): rows are cut into 128-row tiles and a work item is a
// tile pair (ta <= tb) with a range of chunks; an off-diagonal pair has 8 x 8
// blocks, wave w taking row w of them so that its A operand is loaded from LDS
// once per step; a diagonal pair has the 36 blocks of an upper triangle.  The
// items of one split are numbered consecutively and placed on one XCD so that
// pairs sharing a tile share its L2.  Eight waves per workgroup; LDS holds the
// current chunk of rows, double-buffered with one barrier per chunk; global
// loads walk the contiguous axis of the unfolding.  Split s takes chunks s,
// s + nsplit, ..., so that the workgroups stream neighbouring addresses.  Every
// item writes its FP64 partial blocks and a second kernel sums the splits in a
// fixed order.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace tk {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kWaves = 8;
constexpr int kNT = 64 * kWaves;

template <int PREC>
struct Cfg;
template <>
struct Cfg<0> {  // FP64
  static constexpr int KC = 16, LR = 18, PLANES = 1, GROUP = 1;
  using elem = double;
};
template <>
struct Cfg<1> {  // FP32: promote every chunk (32 columns)
  static constexpr int KC = 32, LR = 36, PLANES = 1, GROUP = 1;
  using elem = float;
};
template <>
struct Cfg<2> {  // BF16X3 (80-byte rows: conflict-free 16-byte reads); promote every 8 chunks
  static constexpr int KC = 32, LR = 40, PLANES = 2, GROUP = 8;
  using elem = __bf16;
};
template <>
struct Cfg<3> {  // BF16X6: promote every chunk
  static constexpr int KC = 32, LR = 40, PLANES = 3, GROUP = 1;
  using elem = __bf16;
};

struct MPParams {
  const void* Y;
  int J;
  uint32_t L, K;
  int ntiles;  // pair mode: 128-row tiles
  int npairs;  // pair mode: tile pairs; triangle mode: 1
  int nblk;    // partial blocks per item
  int64_t nchunks, nsplit, total;  // split s takes chunks s, s + nsplit, ...
  double* part;
  double* sq;  // one value per item (zero for items that do not own their rows), or null
};

__device__ __forceinline__ void decode_pair(int p, int ntiles, int& ta, int& tb) {
  int t = 0;
  while (p >= ntiles - t) {
    p -= ntiles - t;
    ++t;
  }
  ta = t;
  tb = t + p;
}

template <int PREC>
__device__ __forceinline__ void put(typename Cfg<PREC>::elem* s, int plane_stride, int o, double v) {
  if constexpr (PREC == 0) {
    s[o] = v;
  } else if constexpr (PREC == 1) {
    s[o] = (float)v;
  } else {
    const float x = (float)v;
    const __bf16 b0 = (__bf16)x;
    const float r1 = x - (float)b0;  // exact
    const __bf16 b1 = (__bf16)r1;
    s[o] = b0;
    s[o + plane_stride] = b1;
    if constexpr (PREC == 3) s[o + 2 * plane_stride] = (__bf16)(r1 - (float)b1);
  }
}

// One work item: the blocks of one wave, the chunk loader, the products of a
// chunk and the output.  SHARED_A: all slots of the wave have the same block
// row (off-diagonal pairs), so the A operand is read from LDS once per step.
//
// Pipelining: global loads run two chunks ahead (two register sets), LDS is
// double-buffered with one barrier per chunk, and the MFMA operands of the
// next step (FP64/FP32) or next slot (BF16 forms) are read from LDS while the
// current step's MFMAs run.
// PAIR: rows are the 128-row tiles of a pair (NR = 128 or 256, a power of two),
// so the loader's (row, column) of each value follows from the thread index
// with shifts instead of per-value index registers.
template <typename T, int PREC, int ROWS, int NBW, bool SHARED_A, bool UNIT_L, bool PAIR, bool UNC = false>
struct GramItem {
  using C = Cfg<PREC>;
  using E_t = typename C::elem;
  static constexpr int KC = C::KC, LR = C::LR, PL = C::PLANES;
  static constexpr int PS = ROWS * LR;       // plane stride
  static constexpr int BS = PL * PS;         // buffer stride
  static constexpr int E = ROWS * KC / kNT;  // loaded values per thread and chunk
  static constexpr int NA = SHARED_A ? 1 : NBW;
  using O = typename std::conditional<PREC == 0, double, float>::type;  // FP64 / FP32 operands

  const T* __restrict__ Y;
  int J;
  uint32_t L, K;
  int64_t JL;
  int i, q;
  int bI[NBW], bJ[NBW];
  static constexpr int EA = PAIR ? 1 : E;  // per-value index arrays (triangle mode)
  int eoff[EA], ek[EA], egrow[EA];
  // pair mode: UNIT_L -> one row per thread (lr0, gr0) and columns kb + kstep p;
  // otherwise one column per thread (kb) and rows lr0 + (kNT / KC) p
  int lr0, gr0, kb, kstep, nr, ra, rb;
  bool diag;
  d4 acc64[NBW];
  f4 acc32[NBW];
  double sq;
  int group_left;

  __device__ __forceinline__ int pair_grow(int lr) const {
    return lr < nr ? ((lr < 128 || diag) ? ra + lr : rb + (lr - 128)) : J;
  }

  // Loads chunk ch and returns the mask of the values that lie inside the
  // tensor (none when chv is false); store() zeroes the others.  kUncond: the
  // loads are issued without any condition (row and column clamped into the
  // tensor), since a load under a condition makes the waits before the next
  // loads conservative and undoes the two-chunk lead of the loads.  It is
  // chosen at launch where it measured faster: the FP32 pair kernel (which
  // then also spills far less) and the BF16X3 pair kernel for more than two
  // row tiles; the other kernels keep loads under the bounds condition.
  static constexpr bool kUncond = UNC;
  __device__ __forceinline__ uint32_t load(T (&rv)[E], int64_t ch, bool chv) const {
    uint32_t vm = 0;
#pragma unroll
    for (int p = 0; p < E; ++p) {
      int gr, k;
      if constexpr (PAIR) {
        if constexpr (UNIT_L) {
          k = kb + kstep * p;
          gr = (k < KC) ? gr0 : J;  // diagonal pairs (NR = 128) need half the values
        } else {
          gr = pair_grow(lr0 + (kNT / KC) * p);
          k = kb;
        }
      } else {
        gr = egrow[p];
        k = ek[p];
      }
      const int64_t c = ch * KC + k;
      auto address = [&](int gr_, int64_t c_) {
        if constexpr (UNIT_L) {
          return (int64_t)gr_ + (int64_t)J * c_;
        } else {
          const uint32_t cc = (uint32_t)c_;
          const uint32_t r = cc / L, l = cc - r * L;
          return (int64_t)l + JL * r + (int64_t)L * gr_;
        }
      };
      if constexpr (kUncond) {
        rv[p] = Y[address(min(gr, J - 1), min(c, (int64_t)K - 1))];
        vm |= (uint32_t)(chv && gr < J && c < (int64_t)K) << p;
      } else {
        T v = (T)0;
        if (gr < J && c < (int64_t)K) v = Y[address(gr, c)];
        rv[p] = v;
      }
    }
    return vm;
  }

  __device__ __forceinline__ void store(const T (&rv)[E], uint32_t vm, E_t* s) {
#pragma unroll
    for (int p = 0; p < E; ++p) {
      double v = (double)rv[p];
      if constexpr (kUncond) v = ((vm >> p) & 1u) ? v : 0.0;
      int o;
      if constexpr (PAIR) {
        if constexpr (UNIT_L) {
          const int k = kb + kstep * p;
          o = (lr0 < nr && k < KC) ? lr0 * LR + k : -1;
        } else {
          const int lr = lr0 + (kNT / KC) * p;
          o = (lr < nr) ? lr * LR + kb : -1;
        }
      } else {
        o = eoff[p];
      }
      if (o >= 0) put<PREC>(s, PS, o, v);
      sq += v * v;
    }
  }

  __device__ __forceinline__ void read_ops(const E_t* s, int st, O (&a)[NA], O (&b)[NBW]) const {
#pragma unroll
    for (int t = 0; t < NA; ++t) a[t] = s[(16 * bI[t] + i) * LR + 4 * st + q];
#pragma unroll
    for (int t = 0; t < NBW; ++t) b[t] = s[(16 * bJ[t] + i) * LR + 4 * st + q];
  }

  __device__ __forceinline__ void read_bf(const E_t* s, int blk, bf8 (&v)[PL]) const {
    const int o = (16 * blk + i) * LR + 8 * q;
#pragma unroll
    for (int pl = 0; pl < PL; ++pl) v[pl] = *reinterpret_cast<const bf8*>(s + pl * PS + o);
  }

  __device__ __forceinline__ void compute(const E_t* s, bool last) {
    if constexpr (PREC <= 1) {
      O a[NA], b[NBW];
      read_ops(s, 0, a, b);
#pragma unroll
      for (int st = 0; st < KC / 4; ++st) {
        O an[NA], bn[NBW];
        if (st + 1 < KC / 4) read_ops(s, st + 1, an, bn);
#pragma unroll
        for (int t = 0; t < NBW; ++t) {
          if constexpr (PREC == 0)
            acc64[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[SHARED_A ? 0 : t], b[t], acc64[t], 0, 0, 0);
          else
            acc32[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[SHARED_A ? 0 : t], b[t], acc32[t], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (st + 1 < KC / 4) {
#pragma unroll
          for (int t = 0; t < NA; ++t) a[t] = an[t];
#pragma unroll
          for (int t = 0; t < NBW; ++t) b[t] = bn[t];
        }
      }
    } else {
      // K = 32 per MFMA: lane (i, q) supplies columns 8q .. 8q+7 of its row
      bf8 A[PL], B[PL];
      if constexpr (SHARED_A) read_bf(s, bI[0], A);
      else read_bf(s, bI[0], A);
      read_bf(s, bJ[0], B);
#pragma unroll
      for (int t = 0; t < NBW; ++t) {
        bf8 An[PL], Bn[PL];
        if (t + 1 < NBW) {
          if constexpr (!SHARED_A) read_bf(s, bI[t + 1], An);
          read_bf(s, bJ[t + 1], Bn);
        }
        f4 acc = acc32[t];
        if constexpr (PREC == 3) {
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2], B[0], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[2], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[1], acc, 0, 0, 0);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[0], acc, 0, 0, 0);
        acc32[t] = acc;
        __builtin_amdgcn_sched_barrier(0);
        if (t + 1 < NBW) {
#pragma unroll
          for (int pl = 0; pl < PL; ++pl) {
            if constexpr (!SHARED_A) A[pl] = An[pl];
            B[pl] = Bn[pl];
          }
        }
      }
    }
    if constexpr (PREC != 0) {
      if (--group_left == 0 || last) {  // promote the group sum to FP64
        group_left = C::GROUP;
#pragma unroll
        for (int t = 0; t < NBW; ++t) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc64[t][v] += (double)acc32[t][v];
          acc32[t] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
  }
};

// What one work item reads and writes: the unfolding (Y, J, L, K), the chunks
// ch0, ch0 + chstep, ... (niter of them), its partial blocks P and, if sqo is
// non-null, the sum of squares of the rows it owns.
struct BodyArgs {
  const void* Y;
  int J;
  uint32_t L, K;
  int64_t ch0, chstep, niter;
  double* P;
  double* sqo;
};

template <typename T, int PREC, int ROWS, int NBW, bool SHARED_A, bool UNIT_L, bool PAIR, bool UNC = false>
__device__ __forceinline__ void gram_body(const BodyArgs& g, bool diag, int ra, int rb, int NR, int nbl,
                                          typename Cfg<PREC>::elem* sY, double* sred) {
  using W = GramItem<T, PREC, ROWS, NBW, SHARED_A, UNIT_L, PAIR, UNC>;
  constexpr int E = W::E, KC = W::KC, LR = W::LR;
  W w;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  w.Y = static_cast<const T*>(g.Y);
  w.J = g.J;
  w.L = g.L;
  w.K = g.K;
  w.JL = (int64_t)g.J * g.L;
  const int64_t split = g.ch0, nsplit = g.chstep, niter = g.niter;
  w.i = lane & 15;
  w.q = lane >> 4;
  w.sq = 0.0;
  w.group_left = W::C::GROUP;

  // this wave's block range [q0, q0 + nq) and its blocks (bI, bJ) in local rows
  const int nblk = diag ? nbl * (nbl + 1) / 2 : 64;
  int q0, nq;
  if constexpr (SHARED_A) {
    q0 = 8 * wave;
    nq = 8;
#pragma unroll
    for (int t = 0; t < NBW; ++t) {
      w.bI[t] = wave;
      w.bJ[t] = 8 + t;
    }
  } else {
    q0 = (int)(((int64_t)nblk * wave) / kWaves);
    nq = (int)(((int64_t)nblk * (wave + 1)) / kWaves) - q0;
    int bi = 0, bj = 0;
    for (int qq = 0; qq < q0; ++qq)
      if (++bj == nbl) {
        ++bi;
        bj = bi;
      }
#pragma unroll
    for (int t = 0; t < NBW; ++t) {  // slots past nq repeat the last block and are not stored
      w.bI[t] = bi;
      w.bJ[t] = bj;
      if (t + 1 < nq && ++bj == nbl) {
        ++bi;
        bj = bi;
      }
    }
  }

  // loader: value p of this thread is (local row, chunk column); rows >= NR are padding
  w.nr = NR;
  w.ra = ra;
  w.rb = rb;
  w.diag = diag;
  if constexpr (PAIR) {
    const int sh = (NR == 256) ? 8 : 7;  // log2(NR)
    if constexpr (UNIT_L) {
      w.lr0 = tid & (NR - 1);
      w.kb = tid >> sh;
      w.kstep = kNT >> sh;
    } else {
      w.kb = tid % KC;
      w.lr0 = tid / KC;
      w.kstep = 0;
    }
    w.gr0 = w.pair_grow(w.lr0);
  }
#pragma unroll
  for (int p = 0; p < W::EA; ++p) {
    if constexpr (PAIR) break;
    int lr, k;
    if constexpr (UNIT_L) {
      const int e = tid + kNT * p;
      const bool ok = e < NR * KC;
      lr = ok ? e % NR : NR;
      k = ok ? e / NR : 0;
    } else {
      k = tid % KC;
      lr = tid / KC + (kNT / KC) * p;
      if (lr > NR) lr = NR;
    }
    w.ek[p] = k;
    w.eoff[p] = (lr < NR) ? lr * LR + k : -1;
    int gr = g.J;
    if (lr < NR) gr = (lr < 128 || diag) ? ra + lr : rb + (lr - 128);
    w.egrow[p] = gr;
  }
#pragma unroll
  for (int t = 0; t < NBW; ++t) {
    w.acc64[t] = d4{0.0, 0.0, 0.0, 0.0};
    w.acc32[t] = f4{0.f, 0.f, 0.f, 0.f};
  }

  // chunks split, split + nsplit, ...; chunk j is staged in LDS buffer j & 1
  typename W::E_t* buf0 = sY;
  typename W::E_t* buf1 = sY + W::BS;
  // kUncond: every path issues the same loads (chunks beyond this split's
  // last are replaced by its first, valid memory, and masked); otherwise
  // loads beyond the last chunk are skipped
  T rv0[E], rv1[E];
  uint32_t vm0 = 0, vm1 = 0;
  auto chunk = [&](int64_t j) { return split + (j < niter ? j : 0) * nsplit; };
  if (niter > 0) {
    vm0 = w.load(rv0, chunk(0), true);
    if (W::kUncond || niter > 1) vm1 = w.load(rv1, chunk(1), niter > 1);
    w.store(rv0, vm0, buf0);
    lds_barrier();
  }
  for (int64_t it = 0; it < niter; it += 2) {
    // chunk it in buf0, chunk it + 1 in rv1; rv0 is free
    if (W::kUncond || it + 2 < niter) vm0 = w.load(rv0, chunk(it + 2), it + 2 < niter);
    w.compute(buf0, it + 1 == niter);
    if (W::kUncond || it + 1 < niter) w.store(rv1, vm1, buf1);  // (zero past the last chunk; not read then)
    lds_barrier();
    if (it + 1 >= niter) break;
    // chunk it + 1 in buf1, chunk it + 2 in rv0; rv1 is free
    if (W::kUncond || it + 3 < niter) vm1 = w.load(rv1, chunk(it + 3), it + 3 < niter);
    w.compute(buf1, it + 2 == niter);
    if (W::kUncond || it + 2 < niter) w.store(rv0, vm0, buf0);
    lds_barrier();
  }

  // partial blocks.  f64 MFMA result: lane l, register v -> D[(l>>4)+4v][l&15];
  // f32 MFMA result: lane l, register v -> D[4(l>>4)+v][l&15].
  double* __restrict__ P = g.P;
#pragma unroll
  for (int t = 0; t < NBW; ++t) {
    if (t < nq) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = (PREC == 0) ? (w.q + 4 * v) : (4 * w.q + v);
        P[(int64_t)(q0 + t) * 256 + row * 16 + w.i] = w.acc64[t][v];
      }
    }
  }
  if (g.sqo != nullptr) {
    // padding rows and columns load zeros; rows of an off-diagonal pair are
    // counted by the diagonal pairs
    const double sw = wave_sum(diag ? w.sq : 0.0);
    if (lane == 0) sred[wave] = sw;
    __syncthreads();
    if (tid == 0) {
      double tot = 0.0;
      for (int w2 = 0; w2 < kWaves; ++w2) tot += sred[w2];
      *g.sqo = tot;
    }
  }
}

// Triangle mode: J <= 128, one item per split.
template <typename T, int PREC, int NBW, bool UNIT_L>
__global__ __launch_bounds__(kNT) void gram_mp_tri_kernel(MPParams g) {
  using C = Cfg<PREC>;
  __shared__ typename C::elem sY[2 * C::PLANES * 128 * C::LR];
  __shared__ double sred[kWaves];
  const int NR = (g.J + 15) & ~15;
  const int64_t split = blockIdx.x;
  const BodyArgs a{g.Y, g.J, g.L, g.K, split, g.nsplit, (g.nchunks - split + g.nsplit - 1) / g.nsplit,
                   g.part + split * (int64_t)g.nblk * 256, g.sq ? g.sq + split : nullptr};
  gram_body<T, PREC, 128, NBW, false, UNIT_L, false>(a, true, 0, 0, NR, NR / 16, sY, sred);
}

// Pair mode: J > 128, items (split, tile pair) placed split-major on XCDs.
// UNC: unconditional loads (GramItem::kUncond).
template <typename T, int PREC, bool UNIT_L, bool UNC>
__global__ __launch_bounds__(kNT) void gram_mp_pair_kernel(MPParams g) {
  using C = Cfg<PREC>;
  __shared__ typename C::elem sY[2 * C::PLANES * 256 * C::LR];
  __shared__ double sred[kWaves];
  const int64_t item = xcd_remap(blockIdx.x, gridDim.x, g.total);
  if (item < 0) return;
  const int pair = (int)(item % g.npairs);
  const int64_t split = item / g.npairs;
  int ta, tb;
  decode_pair(pair, g.ntiles, ta, tb);
  const BodyArgs a{g.Y, g.J, g.L, g.K, split, g.nsplit, (g.nchunks - split + g.nsplit - 1) / g.nsplit,
                   g.part + item * (int64_t)g.nblk * 256, g.sq ? g.sq + item : nullptr};
  if (ta == tb)
    gram_body<T, PREC, 256, 5, false, UNIT_L, true, UNC>(a, true, 128 * ta, 128 * ta, 128, 8, sY, sred);
  else
    gram_body<T, PREC, 256, 8, true, UNIT_L, true, UNC>(a, false, 128 * ta, 128 * tb, 256, 8, sY, sred);
}

// Sum the partial blocks of all splits in a fixed order; write both triangles.
__global__ __launch_bounds__(256) void gram_mp_reduce_kernel(const double* __restrict__ part, int tri, int ntiles,
                                                             int npairs, int nblk, int64_t nsplit, int J,
                                                             double* __restrict__ S) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)npairs * nblk * 256) return;
  const int pair = (int)(idx / ((int64_t)nblk * 256));
  const int qrem = (int)(idx - (int64_t)pair * nblk * 256);
  const int qb = qrem >> 8, rem = qrem & 255;
  int ra = 0, rb = 0, nbl;
  bool diag = true;
  if (tri) {
    nbl = ((J + 15) & ~15) / 16;
  } else {
    int ta, tb;
    decode_pair(pair, ntiles, ta, tb);
    ra = 128 * ta;
    rb = 128 * tb;
    diag = (ta == tb);
    nbl = 8;
  }
  int bi, bj;
  if (diag) {
    if (qb >= nbl * (nbl + 1) / 2) return;
    int qq = qb;
    bi = 0;
    while (qq >= nbl - bi) {
      qq -= nbl - bi;
      ++bi;
    }
    bj = bi + qq;
  } else {
    bi = qb / 8;
    bj = 8 + qb % 8;
  }
  const int r = rem >> 4, c = rem & 15;
  const int a = ra + 16 * bi + r;
  const int b = diag ? ra + 16 * bj + c : rb + 16 * (bj - 8) + c;
  if (a >= J || b >= J || (diag && bi == bj && r > c)) return;
  const double s = sum_strided8(part + ((int64_t)pair * nblk + qb) * 256 + rem, nsplit, (int64_t)npairs * nblk * 256);
  S[(int64_t)a * J + b] = s;
  S[(int64_t)b * J + a] = s;
}

// Batched form: work item i (host-planned from upper bounds of the sizes)
// covers chunks [cb, ce) of tensor t; the current sizes are read from the
// device, so items beyond a tensor's actual column count do nothing.
template <typename T, int PREC, int NBW, bool UNIT_L>
__global__ __launch_bounds__(kNT) void gram_batch_kernel(GramBatch b, int item0) {
  using C = Cfg<PREC>;
  __shared__ typename C::elem sY[2 * C::PLANES * 128 * C::LR];
  __shared__ double sred[kWaves];
  const int it = item0 + blockIdx.x;
  const int64_t* d = b.items + 4 * (int64_t)it;
  const int t = (int)d[0];
  if (b.flag != nullptr && b.flag[t] == 0) return;
  const int J = b.J[t];
  uint64_t L = 1, Rt = 1;
  for (int k = 0; k < b.N; ++k) {
    const uint64_t c = (uint64_t)b.cur[(int64_t)t * b.N + k];
    if (k < b.n) L *= c;
    else if (k > b.n) Rt *= c;
  }
  const uint64_t K = L * Rt;
  const int64_t nch = (int64_t)((K + C::KC - 1) / C::KC);
  const int64_t cb = d[1] * b.chunk_mul, ce = min(d[2] * b.chunk_mul, nch);
  const BodyArgs a{b.Y[t], J, (uint32_t)L, (uint32_t)K, cb, 1, ce > cb ? ce - cb : 0, b.part + d[3],
                   b.sq ? b.sq + it : nullptr};
  const int NR = (J + 15) & ~15;
  gram_body<T, PREC, 128, NBW, false, UNIT_L, false>(a, true, 0, 0, NR, NR / 16, sY, sred);
}

// Per tensor: sum its items' partial blocks (in item order) into S_t (J x J,
// both triangles) and, when nx2 is set, its items' sums of squares.
__global__ __launch_bounds__(256) void gram_batch_reduce_kernel(GramBatch b) {
  const int t = blockIdx.x;
  const int J = b.J[t];
  if (J <= 0) return;
  if (b.flag != nullptr && b.flag[t] == 0) return;
  const int nb = (J + 15) / 16, nblk = nb * (nb + 1) / 2;
  const int idx = blockIdx.y * 256 + threadIdx.x;
  const int i0 = b.ifirst[2 * t], i1 = b.ifirst[2 * t + 1];
  if (idx == 0 && b.nx2 != nullptr) {
    double s = 0.0;
    for (int i = i0; i < i1; ++i) s += b.sq[i];
    b.nx2[t] = s;
  }
  if (idx >= nblk * 256) return;
  const int qb = idx >> 8, rem = idx & 255;
  int bi = 0, qq = qb;
  while (qq >= nb - bi) {
    qq -= nb - bi;
    ++bi;
  }
  const int bj = bi + qq;
  const int r = rem >> 4, c = rem & 15;
  const int ra = 16 * bi + r, cb = 16 * bj + c;
  if (ra >= J || cb >= J || (bi == bj && r > c)) return;
  double s = 0.0;
  for (int i = i0; i < i1; ++i) s += b.part[b.items[4 * (int64_t)i + 3] + idx];
  double* S = b.S + (int64_t)t * b.Jmax * b.Jmax;
  S[(int64_t)ra * J + cb] = s;
  S[(int64_t)cb * J + ra] = s;
}

template <typename T, int PREC>
void launch_batch(const GramBatch& b, bool unit, hipStream_t s) {
  // items [0, nsmall) belong to tensors with J <= 80 (at most 16 blocks), the rest to larger ones
  const int nsmall = b.nsmall, nbig = b.nitems - b.nsmall;
  if (nsmall > 0) {
    if (unit) hipLaunchKernelGGL((gram_batch_kernel<T, PREC, 2, true>), dim3(nsmall), dim3(kNT), 0, s, b, 0);
    else hipLaunchKernelGGL((gram_batch_kernel<T, PREC, 2, false>), dim3(nsmall), dim3(kNT), 0, s, b, 0);
  }
  if (nbig > 0) {
    if (unit) hipLaunchKernelGGL((gram_batch_kernel<T, PREC, 5, true>), dim3(nbig), dim3(kNT), 0, s, b, nsmall);
    else hipLaunchKernelGGL((gram_batch_kernel<T, PREC, 5, false>), dim3(nbig), dim3(kNT), 0, s, b, nsmall);
  }
}

template <typename T, int PREC>
void launch_main(const MPParams& g, bool tri, bool unit, int64_t grid, hipStream_t s) {
  if (tri) {
    const int nbw = (int)ceil_div(g.nblk, kWaves);
#define TRI_L(NBW)                                                                                           \
  do {                                                                                                       \
    if (unit) hipLaunchKernelGGL((gram_mp_tri_kernel<T, PREC, NBW, true>), dim3(grid), dim3(kNT), 0, s, g);  \
    else hipLaunchKernelGGL((gram_mp_tri_kernel<T, PREC, NBW, false>), dim3(grid), dim3(kNT), 0, s, g);      \
  } while (0)
    if (nbw <= 2) TRI_L(2);
    else TRI_L(5);
#undef TRI_L
  } else {
#define PAIR_L(UNC)                                                                                              \
  do {                                                                                                           \
    if (unit) hipLaunchKernelGGL((gram_mp_pair_kernel<T, PREC, true, UNC>), dim3(grid), dim3(kNT), 0, s, g);     \
    else hipLaunchKernelGGL((gram_mp_pair_kernel<T, PREC, false, UNC>), dim3(grid), dim3(kNT), 0, s, g);         \
  } while (0)
    // unconditional loads where they measured faster (GramItem::kUncond)
    if constexpr (PREC == 1) {
      PAIR_L(true);
    } else if constexpr (PREC == 2) {
      if (g.ntiles > 2) PAIR_L(true);
      else PAIR_L(false);
    } else {
      PAIR_L(false);
    }
#undef PAIR_L
  }
}

}  // namespace

GramPlan plan_gram_mp(int J, uint64_t K, int prec) {
  GramPlan p{};
  const int KC = (prec == 0) ? 16 : 32;
  p.nchunks = ceil_div((int64_t)K, KC);
  int64_t nblk;
  if (J <= 128) {
    p.tile = 0;
    p.ntiles = 1;
    p.npairs = 1;
    const int nb = (J + 15) / 16;
    nblk = (int64_t)nb * (nb + 1) / 2;
  } else {
    p.tile = 128;
    p.ntiles = (int)ceil_div(J, 128);
    p.npairs = p.ntiles * (p.ntiles + 1) / 2;
    nblk = 64;
  }
  // about two workgroups per CU, at least 8 chunks per item
  int64_t nsplit = std::max<int64_t>(1, 512 / p.npairs);
  nsplit = std::min<int64_t>(nsplit, std::max<int64_t>(1, p.nchunks / 8));
  p.cps = ceil_div(p.nchunks, nsplit);
  p.nsplit = ceil_div(p.nchunks, p.cps);
  p.part_elems = p.nsplit * p.npairs * nblk * 256;
  p.sq_elems = p.nsplit * p.npairs;
  return p;
}

template <typename T>
hipError_t launch_gram_mp(const T* Y, int J, uint64_t L, uint64_t K, int prec, const GramPlan& p, double* part,
                          double* sq, double* S, double* norm2, hipStream_t stream, hipEvent_t after_main) {
  MPParams g{};
  g.Y = Y;
  g.J = J;
  g.L = (uint32_t)L;
  g.K = (uint32_t)K;
  const bool tri = (p.tile == 0);
  g.ntiles = p.ntiles;
  g.npairs = p.npairs;
  const int nb = (J + 15) / 16;
  g.nblk = tri ? nb * (nb + 1) / 2 : 64;
  g.nchunks = p.nchunks;
  g.nsplit = p.nsplit;
  g.total = p.nsplit * p.npairs;
  g.part = part;
  g.sq = norm2 ? sq : nullptr;
  const int64_t grid = tri ? p.nsplit : ceil_div(g.total, kXcds) * kXcds;
  const bool unit = (L == 1);
  if constexpr (std::is_same<T, double>::value) {
    if (prec != 0) return hipErrorInvalidValue;  // the reduced forms read FP32 data
    launch_main<T, 0>(g, tri, unit, grid, stream);
  } else {
    switch (prec) {
      case 0: launch_main<T, 0>(g, tri, unit, grid, stream); break;
      case 1: launch_main<T, 1>(g, tri, unit, grid, stream); break;
      case 2: launch_main<T, 2>(g, tri, unit, grid, stream); break;
      default: launch_main<T, 3>(g, tri, unit, grid, stream); break;
    }
  }
  if (after_main) (void)hipEventRecord(after_main, stream);
  const int64_t nel = (int64_t)p.npairs * g.nblk * 256;
  hipLaunchKernelGGL(gram_mp_reduce_kernel, dim3(ceil_div(nel, 256)), dim3(256), 0, stream, part, tri ? 1 : 0,
                     g.ntiles, g.npairs, g.nblk, p.nsplit, J, S);
  if (norm2) hipLaunchKernelGGL(sum_fixed_kernel, dim3(1), dim3(256), 0, stream, sq, g.total, norm2);
  return hipGetLastError();
}

void launch_gram_pair_reduce(const double* part, int ntiles, int npairs, int64_t nsplit, int J, double* S,
                             hipStream_t stream) {
  const int64_t nel = (int64_t)npairs * 64 * 256;
  hipLaunchKernelGGL(gram_mp_reduce_kernel, dim3(ceil_div(nel, 256)), dim3(256), 0, stream, part, 0, ntiles, npairs,
                     64, nsplit, J, S);
}

template <typename T>
hipError_t launch_gram_batched(const GramBatch& b, int prec, bool unit_l, hipStream_t stream) {
  if (b.Jmax > 128 || b.nitems <= 0) return hipErrorInvalidValue;
  if constexpr (std::is_same<T, double>::value) {
    if (prec != 0) return hipErrorInvalidValue;
    launch_batch<T, 0>(b, unit_l, stream);
  } else {
    switch (prec) {
      case 0: launch_batch<T, 0>(b, unit_l, stream); break;
      case 1: launch_batch<T, 1>(b, unit_l, stream); break;
      case 2: launch_batch<T, 2>(b, unit_l, stream); break;
      default: launch_batch<T, 3>(b, unit_l, stream); break;
    }
  }
  hipLaunchKernelGGL(gram_batch_reduce_kernel, dim3(b.count, 36), dim3(256), 0, stream, b);
  return hipGetLastError();
}

template hipError_t launch_gram_batched<float>(const GramBatch&, int, bool, hipStream_t);
template hipError_t launch_gram_batched<double>(const GramBatch&, int, bool, hipStream_t);

// Range guard of a reduced-precision Gram: flag = 1 and S zeroed if an entry
// is not finite, trace(S) differs from the FP64 sum of squares by more than
// 1e-3 relative, or (K > 0) a diagonal entry's mean square S_aa / K lies
// outside [2^-100, 2^100]; flag = 0 otherwise.  One workgroup.
__global__ __launch_bounds__(256) void gram_guard_kernel(double* __restrict__ S, int J, double K,
                                                         const double* __restrict__ sq, double* __restrict__ flag) {
  __shared__ double str[256];
  __shared__ int sbad[256];
  const int tid = threadIdx.x;
  const int64_t JJ = (int64_t)J * J;
  int bad = 0;
  for (int64_t e = tid; e < JJ; e += 256)
    if (!isfinite(S[e])) bad = 1;
  double tr = 0.0;
  const double lo = (K > 0.0) ? 0x1p-100 * K : 0.0, hi = (K > 0.0) ? 0x1p100 * K : INFINITY;
  for (int a = tid; a < J; a += 256) {
    const double d = S[(int64_t)a * J + a];
    tr += d;
    if (!(d >= lo && d <= hi)) bad = 1;
  }
  str[tid] = tr;
  sbad[tid] = bad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      str[tid] += str[tid + w];
      sbad[tid] |= sbad[tid + w];
    }
    __syncthreads();
  }
  const double ref = *sq;
  const bool fire = sbad[0] != 0 || !(fabs(str[0] - ref) <= 1e-3 * ref);
  if (fire)
    for (int64_t e = tid; e < JJ; e += 256) S[e] = 0.0;
  if (tid == 0) *flag = fire ? 1.0 : 0.0;
}

// One workgroup per tensor of a batch, the checks of gram_guard_kernel.
__global__ __launch_bounds__(256) void gram_guard_batched_kernel(GramBatch b, int* __restrict__ flag,
                                                                 int* __restrict__ status) {
  __shared__ double str[256];
  __shared__ int sbad[256];
  const int t = blockIdx.x;
  const int tid = threadIdx.x;
  const int J = b.J[t];
  if (J <= 0) return;
  double K = 1.0;
  for (int k = 0; k < b.N; ++k)
    if (k != b.n) K *= (double)b.cur[(int64_t)t * b.N + k];
  double* __restrict__ S = b.S + (int64_t)t * b.Jmax * b.Jmax;
  const int64_t JJ = (int64_t)J * J;
  int bad = 0;
  for (int64_t e = tid; e < JJ; e += 256)
    if (!isfinite(S[e])) bad = 1;
  double tr = 0.0;
  const double lo = 0x1p-100 * K, hi = 0x1p100 * K;
  for (int a = tid; a < J; a += 256) {
    const double d = S[(int64_t)a * J + a];
    tr += d;
    if (!(d >= lo && d <= hi)) bad = 1;
  }
  str[tid] = tr;
  sbad[tid] = bad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      str[tid] += str[tid + w];
      sbad[tid] |= sbad[tid + w];
    }
    __syncthreads();
  }
  const double ref = b.nx2[t];
  const bool fire = sbad[0] != 0 || !(fabs(str[0] - ref) <= 1e-3 * ref);
  if (fire)
    for (int64_t e = tid; e < JJ; e += 256) S[e] = 0.0;
  if (tid == 0) {
    flag[t] = fire ? 1 : 0;
    status[t] |= (isfinite(ref) ? 0 : 1) | (fire ? 2 : 0);
  }
}

hipError_t launch_gram_guard_batched(const GramBatch& b, int* flag, int* status, hipStream_t stream) {
  hipLaunchKernelGGL(gram_guard_batched_kernel, dim3(b.count), dim3(256), 0, stream, b, flag, status);
  return hipGetLastError();
}

hipError_t launch_gram_guard(double* S, int J, double K, const double* sq, double* flag, hipStream_t stream) {
  hipLaunchKernelGGL(gram_guard_kernel, dim3(1), dim3(256), 0, stream, S, J, K, sq, flag);
  return hipGetLastError();
}

template hipError_t launch_gram_mp<float>(const float*, int, uint64_t, uint64_t, int, const GramPlan&, double*,
                                          double*, double*, double*, hipStream_t, hipEvent_t);
template hipError_t launch_gram_mp<double>(const double*, int, uint64_t, uint64_t, int, const GramPlan&, double*,
                                           double*, double*, double*, hipStream_t, hipEvent_t);

}  // namespace tk
