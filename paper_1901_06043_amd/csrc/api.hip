// C ABI of the library (include/tucker.h): argument validation, the ST-HOSVD
// mode loop of paper Alg. 1, Multi-TTM reconstruction of Sec. 8, and the
// single-step entry points.  All device work is enqueued on the caller's
// stream.  Device memory comes from a caching allocator: a freed block is kept
// and handed out again only for work on the stream that freed it, so stream
// order makes the reuse safe without synchronisation; hipMalloc is called only
// when no cached block fits.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/tucker.h"
#include "common.hpp"
#include "kernels.hpp"

using tk::ceil_div;

namespace {

thread_local std::string g_err;

tucker_status fail(tucker_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return fail(_e == hipErrorOutOfMemory ? TUCKER_ENOMEM : TUCKER_EHIP, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(_e), __FILE__, __LINE__);                         \
  } while (0)

size_t dtype_size(tucker_dtype t) { return t == TUCKER_F64 ? 8 : 4; }

// Device checks, once per device.
std::mutex g_dev_mu;
bool g_dev_ok[64];
bool g_dev_checked[64];

tucker_status ensure_device() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(TUCKER_EUNSUPPORTED, "no HIP device: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= 64) return fail(TUCKER_EUNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (!g_dev_checked[dev]) {
    g_dev_checked[dev] = true;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    g_dev_ok[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
  }
  if (!g_dev_ok[dev]) return fail(TUCKER_EUNSUPPORTED, "device %d is not gfx950 (MI355X)", dev);
  return TUCKER_OK;
}

// ---------------------------------------------------------------- caching allocator
struct CachedBlock {
  void* p;
  size_t bytes;
  hipStream_t stream;
  int dev;
};
struct LiveBlock {
  void* p;
  size_t bytes;
  bool external;         // from a caller-supplied allocator (returned to it, not cached)
  tucker_allocator ext;  // that allocator
};
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache_free;  // idle blocks
std::vector<LiveBlock> g_cache_live;    // blocks in use
bool g_ext_set = false;                 // tucker_set_allocator
tucker_allocator g_ext{};

size_t round_bytes(size_t b) {
  b = std::max<size_t>(b, 256);
  const size_t g = (b >= (size_t(1) << 20)) ? (size_t(1) << 20) : 512;
  return (b + g - 1) / g * g;
}

hipError_t dev_alloc(void** out, size_t bytes, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  bytes = round_bytes(bytes);
  tucker_allocator ext{};
  bool use_ext = false;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    use_ext = g_ext_set;
    ext = g_ext;
  }
  if (use_ext) {
    void* p = ext.alloc(bytes, ext.ctx, s);
    if (!p) return hipErrorOutOfMemory;
    *out = p;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache_live.push_back({p, bytes, true, ext});
    return hipSuccess;
  }
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int best = -1;
    for (int i = 0; i < (int)g_cache_free.size(); ++i) {
      const CachedBlock& b = g_cache_free[i];
      if (b.dev != dev || b.stream != s || b.bytes < bytes || b.bytes > 2 * bytes + (size_t(4) << 20)) continue;
      if (best < 0 || b.bytes < g_cache_free[best].bytes) best = i;
    }
    if (best >= 0) {
      *out = g_cache_free[best].p;
      g_cache_live.push_back({*out, g_cache_free[best].bytes, false, {}});
      g_cache_free.erase(g_cache_free.begin() + best);
      return hipSuccess;
    }
  }
  // Make room first: when the device has less than the request (plus 1 GiB)
  // free, an idle block of this stream of any larger size is reused, else
  // idle cached blocks of this device go back to HIP, largest first, until the
  // request would fit.  (Failing allocations, and returning every cached
  // block, are much slower than freeing one or two large blocks.)
  {
    size_t fr = 0, tot = 0;
    const size_t want = bytes + (size_t(1) << 30);
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();  // no figure: hipMalloc decides below
    } else if (fr < want) {
      std::vector<void*> drop;
      {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        // a larger idle block of this stream is taken whole rather than freed
        // (fresh device memory is expensive to map)
        int best = -1;
        for (int i = 0; i < (int)g_cache_free.size(); ++i) {
          const CachedBlock& b = g_cache_free[i];
          if (b.dev != dev || b.stream != s || b.bytes < bytes) continue;
          if (best < 0 || b.bytes < g_cache_free[best].bytes) best = i;
        }
        if (best >= 0) {
          *out = g_cache_free[best].p;
          g_cache_live.push_back({*out, g_cache_free[best].bytes, false, {}});
          g_cache_free.erase(g_cache_free.begin() + best);
          return hipSuccess;
        }
        size_t got = 0;
        while (fr + got < want) {
          int big = -1;
          for (int i = 0; i < (int)g_cache_free.size(); ++i)
            if (g_cache_free[i].dev == dev && (big < 0 || g_cache_free[i].bytes > g_cache_free[big].bytes)) big = i;
          if (big < 0) break;
          got += g_cache_free[big].bytes;
          drop.push_back(g_cache_free[big].p);
          g_cache_free.erase(g_cache_free.begin() + big);
        }
      }
      if (!drop.empty()) {
        (void)hipDeviceSynchronize();  // the blocks may still be read by work in flight
        for (void* p : drop) (void)hipFree(p);
      }
    }
  }
  e = hipMalloc(out, bytes);
  if (e == hipErrorOutOfMemory) {
    // give idle cached blocks of this device back and retry once
    (void)hipGetLastError();
    std::vector<void*> drop;
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      for (int i = (int)g_cache_free.size() - 1; i >= 0; --i)
        if (g_cache_free[i].dev == dev) {
          drop.push_back(g_cache_free[i].p);
          g_cache_free.erase(g_cache_free.begin() + i);
        }
    }
    if (!drop.empty()) {
      (void)hipDeviceSynchronize();
      for (void* p : drop) (void)hipFree(p);
      e = hipMalloc(out, bytes);
    }
  }
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache_live.push_back({*out, bytes, false, {}});
  }
  return e;
}

// Bytes the built-in pool can hand out on this device without a failed
// allocation: free device memory plus idle cached blocks.  SIZE_MAX when a
// caller-supplied allocator is set (its capacity is not known here).
size_t dev_available() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  size_t idle = 0;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (g_ext_set) return SIZE_MAX;
    for (const CachedBlock& b : g_cache_free)
      if (b.dev == dev) idle += b.bytes;
  }
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return SIZE_MAX;
  }
  return fr + idle;
}

// Return a block to the cache; it may be reused by later work on stream s.
void dev_free(void* p, hipStream_t s) {
  if (!p) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  tucker_allocator ext{};
  bool external = false;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (size_t i = 0; i < g_cache_live.size(); ++i)
      if (g_cache_live[i].p == p) {
        external = g_cache_live[i].external;
        ext = g_cache_live[i].ext;
        if (!external) g_cache_free.push_back({p, g_cache_live[i].bytes, s, dev});
        g_cache_live[i] = g_cache_live.back();
        g_cache_live.pop_back();
        break;
      }
  }
  if (external) ext.free(p, ext.ctx, s);  // outside the lock: the callback may allocate
}

// Temporary device buffer returned to the cache (stream-ordered) on scope exit.
struct TmpBuf {
  void* p = nullptr;
  hipStream_t s = nullptr;
  TmpBuf() = default;
  TmpBuf(const TmpBuf&) = delete;
  TmpBuf& operator=(const TmpBuf&) = delete;
  ~TmpBuf() { release(); }
  void release() {
    if (p) dev_free(p, s);
    p = nullptr;
  }
  hipError_t alloc(size_t bytes, hipStream_t st) {
    release();
    s = st;
    return dev_alloc(&p, bytes, st);
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Small pinned host staging area for rank read-back (one per thread).
struct Pinned {
  void* p = nullptr;
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};
thread_local Pinned g_pinned;

tucker_status pinned(void** out) {
  if (!g_pinned.p) HIP_TRY(hipHostMalloc(&g_pinned.p, 4096, hipHostMallocDefault));
  *out = g_pinned.p;
  return TUCKER_OK;
}

tucker_status validate_dims(const int64_t* dims, int N) {
  if (!dims) return fail(TUCKER_EINVAL, "dims is NULL");
  if (N < 1 || N > TUCKER_MAX_MODES) return fail(TUCKER_EINVAL, "N=%d outside 1..%d", N, TUCKER_MAX_MODES);
  for (int k = 0; k < N; ++k)
    if (dims[k] < 1) return fail(TUCKER_EINVAL, "dims[%d]=%lld < 1", k, (long long)dims[k]);
  return TUCKER_OK;
}

tucker_status validate_order(const int* order, int N, int* out) {
  if (!order) {
    for (int k = 0; k < N; ++k) out[k] = k;
    return TUCKER_OK;
  }
  bool seen[TUCKER_MAX_MODES] = {false};
  for (int k = 0; k < N; ++k) {
    if (order[k] < 0 || order[k] >= N || seen[order[k]])
      return fail(TUCKER_EINVAL, "mode order is not a permutation of 0..%d", N - 1);
    seen[order[k]] = true;
    out[k] = order[k];
  }
  return TUCKER_OK;
}

void left_right(const int64_t* dims, int N, int n, int64_t& L, int64_t& Rt) {
  L = 1;
  Rt = 1;
  for (int k = 0; k < n; ++k) L *= dims[k];
  for (int k = n + 1; k < N; ++k) Rt *= dims[k];
}

constexpr int64_t kMaxEigJ = tk::kEigMaxJ;

// Products of the direct-load tile-pair Gram for an arithmetic form and the
// stride L of the mode's rows (0 FP64, 1 FP32, 3 BF16X6), or -1 where the
// register-staged tile pairs are used: the reduced forms on row segments and
// BF16X3 (two pieces, FP32 sums over 8 chunks), which measured faster there.
int dma_gram_prec(tucker_gram_prec prec, int64_t L) {
  if (prec == TUCKER_GRAM_FP64) return 0;
  if (prec == TUCKER_GRAM_FP32 && L == 1) return 1;
  if (prec == TUCKER_GRAM_BF16X6 && L == 1) return 3;
  return -1;
}

// Gram of mode n of a tensor in (ptr, dtype) -> S (J x J FP64), optional norm.
tucker_status run_gram(const void* Y, tucker_dtype dt, const int64_t* dims, int N, int n, tucker_gram_prec prec,
                       double* S, double* norm2, hipStream_t s, hipEvent_t after_main = nullptr) {
  int64_t L, Rt;
  left_right(dims, N, n, L, Rt);
  const int64_t J = dims[n];
  const int64_t K = L * Rt;
  if (K >= (int64_t(1) << 32) || J >= (int64_t(1) << 31))
    return fail(TUCKER_EUNSUPPORTED, "unfolding of mode %d has %lld columns (limit 2^32)", n, (long long)K);
  TmpBuf part, sq;
  if (prec != TUCKER_GRAM_FP64 && dt != TUCKER_F32) return fail(TUCKER_EINVAL, "reduced-precision Gram needs FP32 data");
  if (J <= tk::kStreamMaxJ) {
    // small modes: HBM-bound streaming kernel, any arithmetic form
    tk::GramPlan p = tk::plan_gram_stream((int)J, (uint64_t)K, (int)prec);
    HIP_TRY(part.alloc(sizeof(double) * p.part_elems, s));
    HIP_TRY(sq.alloc(sizeof(double) * p.sq_elems, s));
    if (dt == TUCKER_F64)
      HIP_TRY(tk::launch_gram_stream(static_cast<const double*>(Y), (int)J, L, K, (int)prec, p, part.as<double>(),
                                     sq.as<double>(), S, norm2, s, after_main));
    else
      HIP_TRY(tk::launch_gram_stream(static_cast<const float*>(Y), (int)J, L, K, (int)prec, p, part.as<double>(),
                                     sq.as<double>(), S, norm2, s, after_main));
    return TUCKER_OK;
  }
  if (prec == TUCKER_GRAM_FP64 && J <= tk::kTriMaxJ) {
    // whole triangle per workgroup, FP64
    tk::GramPlan p = tk::plan_gram_f64((int)J, (uint64_t)L, (uint64_t)K);
    HIP_TRY(part.alloc(sizeof(double) * p.part_elems, s));
    HIP_TRY(sq.alloc(sizeof(double) * p.sq_elems, s));
    if (dt == TUCKER_F64)
      HIP_TRY(tk::launch_gram_f64(static_cast<const double*>(Y), (int)J, L, K, p, part.as<double>(),
                                  sq.as<double>(), S, norm2, s, after_main));
    else
      HIP_TRY(tk::launch_gram_f64(static_cast<const float*>(Y), (int)J, L, K, p, part.as<double>(),
                                  sq.as<double>(), S, norm2, s, after_main));
    return TUCKER_OK;
  }
  const int es = (dt == TUCKER_F64) ? 8 : 4;
  // reduced forms: the direct-load kernel runs one workgroup per CU (its
  // FP32 chunk sums or bf16 pieces and FP64 accumulators need more than 256
  // registers)
  const int dprec = dma_gram_prec(prec, L);
  if (dprec >= 0 && tk::gram_dma_eligible((int)J, (uint64_t)L, es, Y)) {
    // larger modes, FP64 or FP32 products: tile pairs staged by direct
    // global-to-LDS loads
    tk::GramPlan p = tk::plan_gram_dma((int)J, (uint64_t)L, (uint64_t)K, es, dprec);
    HIP_TRY(part.alloc(sizeof(double) * p.part_elems, s));
    if (p.sq_elems) HIP_TRY(sq.alloc(sizeof(double) * p.sq_elems, s));
    if (dt == TUCKER_F64)
      HIP_TRY(tk::launch_gram_dma(static_cast<const double*>(Y), (int)J, L, K, dprec, p, part.as<double>(),
                                  sq.as<double>(), S, norm2, s, after_main));
    else
      HIP_TRY(tk::launch_gram_dma(static_cast<const float*>(Y), (int)J, L, K, dprec, p, part.as<double>(),
                                  sq.as<double>(), S, norm2, s, after_main));
    return TUCKER_OK;
  }
  tk::GramPlan p = tk::plan_gram_mp((int)J, (uint64_t)K, (int)prec);
  HIP_TRY(part.alloc(sizeof(double) * p.part_elems, s));
  HIP_TRY(sq.alloc(sizeof(double) * p.sq_elems, s));
  if (dt == TUCKER_F64)
    HIP_TRY(tk::launch_gram_mp(static_cast<const double*>(Y), (int)J, L, K, (int)prec, p, part.as<double>(),
                               sq.as<double>(), S, norm2, s, after_main));
  else
    HIP_TRY(tk::launch_gram_mp(static_cast<const float*>(Y), (int)J, L, K, (int)prec, p, part.as<double>(),
                               sq.as<double>(), S, norm2, s, after_main));
  return TUCKER_OK;
}

tucker_status run_ttm(const void* Y, tucker_dtype yd, const int64_t* dims, int N, int n, const double* M,
                      int64_t K, int64_t msk, int64_t msj, void* Z, tucker_dtype zd, bool f32p, hipStream_t s) {
  int64_t L, Rt;
  left_right(dims, N, n, L, Rt);
  const int64_t J = dims[n];
  const int64_t cols = L * Rt;
  if (cols >= (int64_t(1) << 32) || K >= (int64_t(1) << 31) || J >= (int64_t(1) << 31))
    return fail(TUCKER_EUNSUPPORTED, "TTM of mode %d too large for 32-bit column indexing", n);
  if (yd == TUCKER_F64 && zd == TUCKER_F64)
    HIP_TRY(tk::launch_ttm(static_cast<const double*>(Y), (int)J, L, cols, M, msk, msj, (int)K,
                           static_cast<double*>(Z), f32p, s));
  else if (yd == TUCKER_F32 && zd == TUCKER_F64)
    HIP_TRY(tk::launch_ttm(static_cast<const float*>(Y), (int)J, L, cols, M, msk, msj, (int)K,
                           static_cast<double*>(Z), f32p, s));
  else if (yd == TUCKER_F64 && zd == TUCKER_F32)
    HIP_TRY(tk::launch_ttm(static_cast<const double*>(Y), (int)J, L, cols, M, msk, msj, (int)K,
                           static_cast<float*>(Z), f32p, s));
  else
    HIP_TRY(tk::launch_ttm(static_cast<const float*>(Y), (int)J, L, cols, M, msk, msj, (int)K,
                           static_cast<float*>(Z), f32p, s));
  return TUCKER_OK;
}

}  // namespace

struct tucker_t {
  int N = 0;
  int64_t dims[TUCKER_MAX_MODES] = {0};
  int64_t ranks[TUCKER_MAX_MODES] = {0};
  int64_t eigcount[TUCKER_MAX_MODES] = {0};
  int order[TUCKER_MAX_MODES] = {0};
  double disc[TUCKER_MAX_MODES] = {0};
  double ms[4 * TUCKER_MAX_MODES] = {0};
  double norm2 = 0.0;
  tucker_dtype core_dtype = TUCKER_F64;
  tucker_gram_prec prec_used[TUCKER_MAX_MODES] = {TUCKER_GRAM_FP64};
  int scaled[TUCKER_MAX_MODES] = {0};  // per mode: 1 if its Gram ran with per-slice scaling
  void* core = nullptr;
  double* U[TUCKER_MAX_MODES] = {nullptr};
  double* lam[TUCKER_MAX_MODES] = {nullptr};
  // [0] ||X||^2; [2, 2+16) discarded energy per mode; [18, 34) sum of squares of
  // the working tensor per step; [34, 50) range-guard flag per step
  double* scalars = nullptr;
  int64_t* dranks = nullptr;
  hipStream_t stream = nullptr;
  std::vector<void*> owned;
  // post-processing of one mode (tucker_set_postprocess): shift may be null
  int post_mode = -1;
  double* post_shift = nullptr;  // post_shift_buf while a shift is attached
  double* post_shift_buf = nullptr;
  double* post_scale = nullptr;
  // events recorded on other streams after work that reads the handle
  // (reconstructions); tucker_free orders the release after them
  mutable std::mutex foreign_mu;
  mutable std::vector<hipEvent_t> foreign;

  hipError_t alloc(void** p, size_t bytes);
  void release();
};

hipError_t tucker_t::alloc(void** p, size_t bytes) {
  hipError_t e = dev_alloc(p, bytes, stream);
  if (e == hipSuccess) owned.push_back(*p);
  return e;
}

void tucker_t::release() {
  {
    // blocks go back to the cache of `stream`; work on other streams that
    // still reads them must finish first
    std::lock_guard<std::mutex> lk(foreign_mu);
    for (hipEvent_t e : foreign) {
      (void)hipStreamWaitEvent(stream, e, 0);
      (void)hipEventDestroy(e);
    }
    foreign.clear();
  }
  for (void* p : owned) dev_free(p, stream);
  owned.clear();
}

namespace {

struct HandleGuard {
  tucker_t* t;
  explicit HandleGuard(tucker_t* h) : t(h) {}
  ~HandleGuard() {
    if (t) {
      t->release();
      delete t;
    }
  }
  tucker_t* take() {
    tucker_t* h = t;
    t = nullptr;
    return h;
  }
};

struct Events {
  hipEvent_t ev[7 * TUCKER_MAX_MODES] = {nullptr};
  int n = 0;
  ~Events() {
    for (int i = 0; i < n; ++i) (void)hipEventDestroy(ev[i]);
  }
  hipError_t create(int count) {
    for (; n < count; ++n) {
      hipError_t e = hipEventCreate(&ev[n]);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
};

}  // namespace

extern "C" {

const char* tucker_last_error(void) { return g_err.c_str(); }
const char* tucker_version(void) { return "tuckerhip 0.1 (gfx950)"; }

tucker_status tucker_reconstruct_order(int N, const int64_t* ranks, const int64_t* out_sizes, int* order_out) {
  if (!ranks || !out_sizes || !order_out) return fail(TUCKER_EINVAL, "NULL argument");
  if (N < 1 || N > TUCKER_MAX_MODES) return fail(TUCKER_EINVAL, "N=%d outside 1..%d", N, TUCKER_MAX_MODES);
  for (int k = 0; k < N; ++k)
    if (ranks[k] < 1 || out_sizes[k] < 1) return fail(TUCKER_EINVAL, "sizes must be >= 1");
  std::vector<int> ord(N);
  std::iota(ord.begin(), ord.end(), 0);
  // i before j iff K_i R_i R_j + K_i R_j K_j < R_i R_j K_j + R_i K_i K_j  (exact, 128-bit)
  std::stable_sort(ord.begin(), ord.end(), [&](int i, int j) {
    const __int128 Ri = ranks[i], Rj = ranks[j], Ki = out_sizes[i], Kj = out_sizes[j];
    return Ki * Ri * Rj + Ki * Rj * Kj < Ri * Rj * Kj + Ri * Ki * Kj;
  });
  for (int k = 0; k < N; ++k) order_out[k] = ord[k];
  return TUCKER_OK;
}

}  // extern "C"

namespace {

// Predicted unit roundoff-level error of a reduced Gram, relative to ||Y||^2
// (the selection rule of TUCKER_GRAM_AUTO): FP32 and BF16X6 carry the FP32
// rounding of the working tensor and of the accumulation, 2^-23; BF16X3 its
// systematic under-estimate, 2^-16 / 3 of the trace (the dropped product).
constexpr double kAutoErrFp32 = 0x1p-23;
constexpr double kAutoErrBf16x3 = 0x1p-16 / 3.0;

tucker_gram_prec resolve_auto(tucker_dtype dtype, int N, double eps, bool fixed) {
  if (dtype != TUCKER_F32 || fixed) return TUCKER_GRAM_FP64;
  // slack of the 1.05 eps target in the truncation rule, relative to ||X||^2
  const double slack = (1.05 * 1.05 - 1.0) * eps * eps / N;
  if (kAutoErrBf16x3 <= 0.01 * slack) return TUCKER_GRAM_BF16X3;
  if (kAutoErrFp32 <= 0.01 * slack) return TUCKER_GRAM_FP32;
  return TUCKER_GRAM_FP64;
}

// Scratch of one Gram of mode n (split-K partials and sums of squares).
int64_t gram_scratch_doubles(const int64_t* dims, int N, int n, tucker_gram_prec prec) {
  int64_t L, Rt;
  left_right(dims, N, n, L, Rt);
  const int64_t J = dims[n], K = L * Rt;
  tk::GramPlan p;
  if (J <= tk::kStreamMaxJ) p = tk::plan_gram_stream((int)J, (uint64_t)K, (int)prec);
  else if (prec == TUCKER_GRAM_FP64 && J <= tk::kTriMaxJ) p = tk::plan_gram_f64((int)J, (uint64_t)L, (uint64_t)K);
  else p = tk::plan_gram_mp((int)J, (uint64_t)K, (int)prec);
  int64_t need = p.part_elems + p.sq_elems;
  const int dprec = dma_gram_prec(prec, L);
  if (dprec >= 0 && J > (dprec == 0 ? tk::kTriMaxJ : tk::kStreamMaxJ)) {
    // the tile-pair kernel with direct LDS loads (FP64: either input type;
    // reduced forms: float input)
    for (int es : {4, 8}) {
      if (dprec >= 1 && es == 8) continue;
      if (tk::gram_dma_eligible((int)J, (uint64_t)L, es, nullptr)) {
        const tk::GramPlan d = tk::plan_gram_dma((int)J, (uint64_t)L, (uint64_t)K, es, dprec);
        need = std::max(need, d.part_elems + d.sq_elems);
      }
    }
  }
  return need;
}

// Working extent of mode n after its truncation to rank R at `step`: R, or
// R + 1 (a zero slice, from a zero column appended to U_n) when R is odd and
// the FP64 path would otherwise meet an odd L = prod_{k<m} J_k at a later
// mode m > n, whose rows of the unfolding would then not be 16-byte aligned
// for the direct-load Gram and mode-product kernels.  The zero slice adds
// nothing to any later Gram or product; the core is compacted at the end.
int64_t working_rank(const int64_t* cur, int N, const int* order, int step, int64_t R, bool reduced) {
  const int n = order[step];
  if (reduced || R % 2 == 0 || R >= cur[n]) return R;
  for (int s = step + 1; s < N; ++s) {
    const int m = order[s];
    if (m <= n) continue;
    int64_t L = 1;
    for (int k = 0; k < m; ++k) L *= (k == n) ? R : cur[k];
    if (L > 1 && L % 2 == 1) return R + 1;
  }
  return R;
}

// Device memory of one compression (the input excluded), following the
// allocations of sthosvd_impl: the handle's factors, eigenvalues and
// scalars, the Gram and eigensolver workspaces, and per step the current and
// next working tensors plus that step's Gram scratch (and, for the reduced
// forms, what the per-slice scaled pass needs).  `ranks` = NULL takes R_n =
// J_n at every step (an upper bound when the ranks are not known).
size_t predict_bytes(tucker_dtype dtype, const int64_t* dims, int N, const int64_t* ranks, const int* order,
                     tucker_gram_prec prec) {
  const bool reduced = (prec != TUCKER_GRAM_FP64);
  const size_t wsz = reduced ? 4 : 8;
  int64_t maxJ = 0;
  for (int k = 0; k < N; ++k) maxJ = std::max(maxJ, dims[k]);
  size_t fixed = round_bytes(sizeof(double) * (2 + 3 * TUCKER_MAX_MODES)) + round_bytes(8 * TUCKER_MAX_MODES) +
                 round_bytes(sizeof(double) * maxJ * maxJ) +
                 round_bytes(sizeof(double) * tk::eig_work_doubles(maxJ));
  for (int k = 0; k < N; ++k)
    fixed += round_bytes(sizeof(double) * dims[k] * dims[k]) + round_bytes(sizeof(double) * dims[k]);
  int64_t cur[TUCKER_MAX_MODES];
  std::memcpy(cur, dims, sizeof(int64_t) * N);
  size_t peak = 0;
  bool padded = false;
  for (int s = 0; s < N; ++s) {
    const int n = order[s];
    int64_t total = 1;
    for (int k = 0; k < N; ++k) total *= cur[k];
    const int64_t J = cur[n];
    const int64_t R0 = ranks ? std::min<int64_t>(ranks[n], J) : J;
    const int64_t R = working_rank(cur, N, order, s, R0, reduced);
    padded = padded || (R != R0);
    const size_t ycur = (s == 0) ? 0 : round_bytes(wsz * total);
    const size_t ynext = round_bytes(wsz * (total / J * R));
    size_t gram = round_bytes(sizeof(double) * gram_scratch_doubles(cur, N, n, prec));
    if (reduced) {
      int64_t L, Rt;
      left_right(cur, N, n, L, Rt);
      gram += round_bytes(4 * total) + round_bytes(sizeof(double) * tk::slice_stats_work_doubles(L, J, Rt)) +
              3 * round_bytes(sizeof(double) * TUCKER_NSTATS * J);
    }
    // the Gram scratch is released before the next working tensor is allocated
    peak = std::max(peak, ycur + std::max(gram, ynext));
    cur[n] = R;
  }
  if (padded && ranks) {
    // the padded core and its compacted copy
    int64_t tp = 1, tc = 1;
    for (int k = 0; k < N; ++k) {
      tp *= cur[k];
      tc *= std::min<int64_t>(ranks[k], dims[k]);
    }
    peak = std::max(peak, round_bytes(wsz * tp) + round_bytes(wsz * tc));
  }
  (void)dtype;
  return fixed + peak;
}

tucker_status fits(size_t bytes, const char* what) {
  const size_t avail = dev_available();
  if (bytes > avail)
    return fail(TUCKER_ENOMEM, "%s needs %.3f GB of device memory; %.3f GB are available", what, bytes / 1e9,
                avail / 1e9);
  return TUCKER_OK;
}

// ST-HOSVD (Alg. 1) with the eq. Un rank rule, or with given ranks.
tucker_status sthosvd_impl(const void* data, tucker_dtype dtype, const int64_t* dims, int N, double eps,
                           const int64_t* fixed_ranks, const int* mode_order, tucker_gram_prec prec,
                           hipStream_t stream, tucker_t** out) {
  if (!out) return fail(TUCKER_EINVAL, "out is NULL");
  *out = nullptr;
  if (!data) return fail(TUCKER_EINVAL, "data is NULL");
  if (dtype != TUCKER_F32 && dtype != TUCKER_F64) return fail(TUCKER_EINVAL, "bad dtype");
  if (prec < TUCKER_GRAM_FP64 || prec > TUCKER_GRAM_AUTO) return fail(TUCKER_EINVAL, "bad Gram precision");
  if (prec != TUCKER_GRAM_FP64 && prec != TUCKER_GRAM_AUTO && dtype != TUCKER_F32)
    return fail(TUCKER_EINVAL, "reduced-precision Gram needs FP32 data");
  if (!fixed_ranks && (!(eps >= 0.0) || !std::isfinite(eps)))
    return fail(TUCKER_EINVAL, "eps must be finite and >= 0");
  tucker_status st = validate_dims(dims, N);
  if (st) return st;
  if (fixed_ranks)
    for (int k = 0; k < N; ++k)
      if (fixed_ranks[k] < 1) return fail(TUCKER_EINVAL, "ranks[%d]=%lld < 1", k, (long long)fixed_ranks[k]);
  int order[TUCKER_MAX_MODES];
  if ((st = validate_order(mode_order, N, order))) return st;
  for (int k = 0; k < N; ++k)
    if (dims[k] > kMaxEigJ)
      return fail(TUCKER_EUNSUPPORTED, "mode %d has size %lld; the eigensolver supports up to %lld", k,
                  (long long)dims[k], (long long)kMaxEigJ);
  if (prec == TUCKER_GRAM_AUTO) prec = resolve_auto(dtype, N, eps, fixed_ranks != nullptr);
  if ((st = ensure_device())) return st;
  // memory: the whole run when the ranks are given, else what the first step needs
  {
    int64_t first[TUCKER_MAX_MODES];
    for (int k = 0; k < N; ++k) first[k] = (k == order[0]) ? dims[k] : 1;
    const size_t need = fixed_ranks ? predict_bytes(dtype, dims, N, fixed_ranks, order, prec)
                                    : predict_bytes(dtype, dims, N, first, order, prec);
    if ((st = fits(need, "the compression"))) return st;
  }

  HandleGuard g(new tucker_t);
  tucker_t* t = g.t;
  t->N = N;
  t->stream = stream;
  std::memcpy(t->dims, dims, sizeof(int64_t) * N);
  std::memcpy(t->order, order, sizeof(int) * N);
  const tucker_dtype wdt = (prec == TUCKER_GRAM_FP64) ? TUCKER_F64 : TUCKER_F32;
  t->core_dtype = wdt;
  HIP_TRY(t->alloc((void**)&t->scalars, sizeof(double) * (2 + 3 * TUCKER_MAX_MODES)));
  HIP_TRY(t->alloc((void**)&t->dranks, sizeof(int64_t) * TUCKER_MAX_MODES));
  double* d_nx2 = t->scalars;
  double* d_disc = t->scalars + 2;
  double* d_sq = t->scalars + 2 + TUCKER_MAX_MODES;
  double* d_flag = t->scalars + 2 + 2 * TUCKER_MAX_MODES;
  const bool reduced = (prec != TUCKER_GRAM_FP64);
  // with given ranks in FP64 nothing depends on a read-back: one synchronisation at the end
  const bool async = fixed_ranks && !reduced;

  void* hp = nullptr;
  if ((st = pinned(&hp))) return st;
  int64_t* h_R = static_cast<int64_t*>(hp);
  double* h_flag = reinterpret_cast<double*>(static_cast<char*>(hp) + 8);
  double* h_nx2 = reinterpret_cast<double*>(static_cast<char*>(hp) + 16);

  Events evs;
  HIP_TRY(evs.create(7 * N));  // 5 per step, then 2 per deferred product
  hipEvent_t rank_ready = nullptr;
  HIP_TRY(hipEventCreateWithFlags(&rank_ready, hipEventDisableTiming));
  struct EventGuard {
    hipEvent_t e;
    ~EventGuard() { (void)hipEventDestroy(e); }
  } rank_ready_guard{rank_ready};

  int64_t cur[TUCKER_MAX_MODES];
  std::memcpy(cur, dims, sizeof(int64_t) * N);
  const void* Y = data;
  tucker_dtype ydt = dtype;
  TmpBuf ybuf;  // owns Y after the first TTM (unless it became the core)
  int64_t maxJ = 0;
  for (int k = 0; k < N; ++k) maxJ = std::max(maxJ, dims[k]);
  TmpBuf Sbuf, ewbuf;
  HIP_TRY(Sbuf.alloc(sizeof(double) * maxJ * maxJ, stream));
  HIP_TRY(ewbuf.alloc(sizeof(double) * tk::eig_work_doubles(maxJ), stream));
  const double thr_mul = fixed_ranks ? 0.0 : eps * eps / N;
  bool padded = false;  // some working extent exceeds its rank (working_rank)
  int ndef = 0, defm[TUCKER_MAX_MODES];  // modes whose product is deferred to the end

  for (int step = 0; step < N; ++step) {
    const int n = order[step];
    const int64_t J = cur[n];
    const int fixed = fixed_ranks ? (int)std::min<int64_t>(fixed_ranks[n], J) : 0;
    hipEvent_t* ev = evs.ev + 5 * step;
    HIP_TRY(t->alloc((void**)&t->U[n], sizeof(double) * J * J));
    HIP_TRY(t->alloc((void**)&t->lam[n], sizeof(double) * J));
    t->eigcount[n] = J;
    tk::EigWork w;
    tk::eig_work_carve(ewbuf.as<double>(), J, w);
    t->prec_used[n] = prec;
    int64_t L, Rt;
    left_right(cur, N, n, L, Rt);
    double* sqp = (step == 0) ? d_nx2 : (reduced ? d_sq + step : nullptr);
    // Gram (+ range guard) and eigensolve.  Reduced forms: if the guard fires,
    // a second pass with per-slice power-of-two scaling, and FP64 if that
    // fires too.
    for (int pass = 0; pass < 3; ++pass) {
      if (pass > 0 && !reduced) break;
      const tucker_gram_prec pp = (pass < 2) ? prec : TUCKER_GRAM_FP64;
      HIP_TRY(hipEventRecord(ev[0], stream));
      TmpBuf stats, pscale, zero, scaled;
      if (pass == 1) {
        // each slice of mode n divided by a power of two near its largest
        // magnitude (exact), the Gram of that copy, S multiplied back
        HIP_TRY(stats.alloc(sizeof(double) * TUCKER_NSTATS * J, stream));
        HIP_TRY(pscale.alloc(sizeof(double) * J, stream));
        HIP_TRY(zero.alloc(sizeof(double) * J, stream));
        TmpBuf work;
        HIP_TRY(work.alloc(sizeof(double) * tk::slice_stats_work_doubles(L, J, Rt), stream));
        if (ydt == TUCKER_F64)
          HIP_TRY(tk::launch_slice_stats(static_cast<const double*>(Y), L, J, Rt, false, work.as<double>(),
                                         stats.as<double>(), stream));
        else
          HIP_TRY(tk::launch_slice_stats(static_cast<const float*>(Y), L, J, Rt, false, work.as<double>(),
                                         stats.as<double>(), stream));
        HIP_TRY(tk::launch_slice_pow2(stats.as<double>(), J, pscale.as<double>(), stream));
        HIP_TRY(tk::launch_fill(zero.as<double>(), J, 0.0, stream));
        const uint64_t total = (uint64_t)(L * J * Rt);
        HIP_TRY(scaled.alloc(sizeof(float) * total, stream));
        if (ydt == TUCKER_F64)
          HIP_TRY(tk::launch_slice_transform(static_cast<const double*>(Y), scaled.as<float>(), total, L, J,
                                             zero.as<double>(), pscale.as<double>(), false, stream));
        else
          HIP_TRY(tk::launch_slice_transform(static_cast<const float*>(Y), scaled.as<float>(), total, L, J,
                                             zero.as<double>(), pscale.as<double>(), false, stream));
        // the FP64 sum of squares of the unscaled tensor is already known (pass 0)
        if ((st = run_gram(scaled.p, TUCKER_F32, cur, N, n, pp, Sbuf.as<double>(), nullptr, stream, ev[4]))) return st;
        HIP_TRY(tk::launch_gram_unscale(Sbuf.as<double>(), J, pscale.as<double>(), stream));
      } else {
        if ((st = run_gram(Y, ydt, cur, N, n, pp, Sbuf.as<double>(), sqp, stream, ev[4]))) return st;
      }
      if (pp != TUCKER_GRAM_FP64)
        HIP_TRY(tk::launch_gram_guard(Sbuf.as<double>(), (int)J, pass == 1 ? 0.0 : (double)(L * Rt),
                                      sqp ? sqp : d_sq + step, d_flag + step, stream));
      HIP_TRY(hipEventRecord(ev[1], stream));
      HIP_TRY(tk::launch_eig_values(Sbuf.as<double>(), (int)J, thr_mul, fixed_ranks ? nullptr : d_nx2, fixed, w,
                                    t->lam[n], t->dranks + n, d_disc + n, stream));
      if (!async) {
        // the rank (and flag, norm) go to the host while the eigenvectors are
        // formed, so that the next launches are enqueued before the GPU runs
        // out of work
        HIP_TRY(hipMemcpyAsync(h_R, t->dranks + n, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        if (pp != TUCKER_GRAM_FP64)
          HIP_TRY(hipMemcpyAsync(h_flag, d_flag + step, sizeof(double), hipMemcpyDeviceToHost, stream));
        if (step == 0) HIP_TRY(hipMemcpyAsync(h_nx2, d_nx2, sizeof(double), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipEventRecord(rank_ready, stream));
      }
      HIP_TRY(tk::launch_eig_vectors((int)J, w, t->lam[n], t->dranks + n, t->U[n], stream));
      HIP_TRY(hipEventRecord(ev[2], stream));
      if (async) break;
      HIP_TRY(hipEventSynchronize(rank_ready));
      if (pp == TUCKER_GRAM_FP64 || h_flag[0] == 0.0) break;
      if (pass == 0) t->scaled[n] = 1;
      else t->prec_used[n] = TUCKER_GRAM_FP64;
    }
    const int64_t R = async ? fixed : h_R[0];
    if (R < 1 || R > J) return fail(TUCKER_ENOCONV, "eigensolver returned rank %lld for J=%lld", (long long)R, (long long)J);
    if (step == 0 && !async) {
      // non-finite data shows up as a non-finite norm
      const double nx2 = h_nx2[0];  // read back with the rank
      if (!std::isfinite(nx2)) return fail(TUCKER_EINVAL, "data contains non-finite values (||X||^2 = %g)", nx2);
      t->norm2 = nx2;
    }
    t->ranks[n] = R;
    // A mode kept at full rank (R = J) is an orthogonal change of basis, under
    // which the Gram Y_(m) Y_(m)^T of every other mode m is invariant (and so
    // is ||Y||, which the range guards compare with): its product commutes
    // with the later ones and changes none of their Grams, so it is applied
    // last, to the core-sized tensor (never the last step itself).
    if (R == J && step < N - 1) {
      defm[ndef++] = n;
      HIP_TRY(hipEventRecord(ev[3], stream));
      continue;
    }
    // working extent (R, or R + 1 with a zero column R of U_n)
    const int64_t Rw = working_rank(cur, N, order, step, R, reduced);
    if (Rw != R) {
      HIP_TRY(tk::launch_fill(t->U[n] + R * J, (uint64_t)J, 0.0, stream));
      padded = true;
    }
    // Y <- Y x_n U_n^T: M(k, j) = U[j + k*J]
    int64_t total = 1;
    for (int k = 0; k < N; ++k) total *= cur[k];
    int64_t next_elems = total / J * Rw;
    // the last product writes the compact core itself when one earlier mode
    // p < n carries a zero slice and the direct-load kernel takes the product
    int pad = -1, npad = 0;
    if (padded && step == N - 1)
      for (int k = 0; k < N; ++k)
        if (k != n && cur[k] != t->ranks[k]) {
          pad = k;
          ++npad;
        }
    tk::TtmOutRemap rm;
    bool fused = false;
    if (npad == 1 && pad < n && Rw == R && ydt == TUCKER_F64 && wdt == TUCKER_F64) {
      int64_t L, Rt;
      left_right(cur, N, n, L, Rt);
      if (L > 1 && L * Rt < (int64_t(1) << 32) &&
          tk::ttm_dma_eligible((int)J, (uint64_t)L, (uint64_t)(L * Rt), (int)Rw, J, 1, 8, 8, Y, t->U[n])) {
        rm.Lp = 1;
        for (int k = 0; k < pad; ++k) rm.Lp *= cur[k];
        rm.Pp = cur[pad];
        rm.Rp = t->ranks[pad];
        fused = true;
        next_elems = next_elems / rm.Pp * rm.Rp;
      }
    }
    if (!async && (st = fits(round_bytes(dtype_size(wdt) * next_elems), "the next working tensor"))) return st;
    TmpBuf nbuf;
    HIP_TRY(nbuf.alloc(dtype_size(wdt) * next_elems, stream));
    if (fused) {
      int64_t L, Rt;
      left_right(cur, N, n, L, Rt);
      HIP_TRY(tk::launch_ttm_dma(static_cast<const double*>(Y), (int)J, (uint64_t)L, (uint64_t)(L * Rt), t->U[n], J,
                                 1, (int)Rw, static_cast<double*>(nbuf.p), stream, rm));
      cur[pad] = t->ranks[pad];
      padded = false;
    } else if ((st = run_ttm(Y, ydt, cur, N, n, t->U[n], Rw, J, 1, nbuf.p, wdt, reduced, stream))) {
      return st;
    }
    HIP_TRY(hipEventRecord(ev[3], stream));
    ybuf.release();  // stream-ordered: after the TTM that read it
    ybuf.p = nbuf.p;
    ybuf.s = stream;
    nbuf.p = nullptr;
    Y = ybuf.p;
    ydt = wdt;
    cur[n] = Rw;
  }
  if (padded) {
    // the core without the zero slices of padded modes
    tk::CompactGeo geo{};
    int64_t ctotal = 1;
    for (int k = 0; k < N; ++k) {
      geo.src[k] = cur[k];
      geo.dst[k] = t->ranks[k];
      ctotal *= t->ranks[k];
    }
    if (!async && (st = fits(round_bytes(sizeof(double) * ctotal), "the core"))) return st;
    TmpBuf cbuf;
    HIP_TRY(cbuf.alloc(sizeof(double) * ctotal, stream));
    HIP_TRY(tk::launch_compact(ybuf.as<double>(), cbuf.as<double>(), geo, N, stream));
    ybuf.release();
    ybuf.p = cbuf.p;
    ybuf.s = stream;
    cbuf.p = nullptr;
  }
  // the deferred full-rank products (Y <- Y x_m U_m^T), on the compact core
  // (ybuf holds it, of sizes R_0 .. R_{N-1} in the working type: the last
  // step always runs its product)
  Y = ybuf.p;
  ydt = wdt;
  std::memcpy(cur, t->ranks, sizeof(int64_t) * N);
  for (int i = 0; i < ndef; ++i) {
    const int m = defm[i];
    int64_t total = 1;
    for (int k = 0; k < N; ++k) total *= cur[k];
    if (!async && (st = fits(round_bytes(dtype_size(wdt) * total), "the core"))) return st;
    TmpBuf nbuf;
    HIP_TRY(nbuf.alloc(dtype_size(wdt) * total, stream));
    HIP_TRY(hipEventRecord(evs.ev[5 * N + 2 * i], stream));
    if ((st = run_ttm(Y, ydt, cur, N, m, t->U[m], cur[m], cur[m], 1, nbuf.p, wdt, reduced, stream))) return st;
    HIP_TRY(hipEventRecord(evs.ev[5 * N + 2 * i + 1], stream));
    ybuf.release();
    ybuf.p = nbuf.p;
    ybuf.s = stream;
    nbuf.p = nullptr;
    Y = ybuf.p;
  }
  // the last Y is the core; hand ownership to the handle
  t->core = ybuf.p;
  t->owned.push_back(ybuf.p);
  ybuf.p = nullptr;
  HIP_TRY(hipMemcpyAsync(t->disc, d_disc, sizeof(double) * N, hipMemcpyDeviceToHost, stream));
  if (async) HIP_TRY(hipMemcpyAsync(h_nx2, d_nx2, sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (async) {
    const double nx2 = h_nx2[0];
    if (!std::isfinite(nx2)) return fail(TUCKER_EINVAL, "data contains non-finite values (||X||^2 = %g)", nx2);
    t->norm2 = nx2;
  }
  for (int step = 0; step < N; ++step) {
    const int n = order[step];
    float a = 0, b = 0, c = 0, k = 0;
    hipEvent_t* ev = evs.ev + 5 * step;
    HIP_TRY(hipEventElapsedTime(&a, ev[0], ev[1]));
    HIP_TRY(hipEventElapsedTime(&b, ev[1], ev[2]));
    HIP_TRY(hipEventElapsedTime(&c, ev[2], ev[3]));
    HIP_TRY(hipEventElapsedTime(&k, ev[0], ev[4]));
    t->ms[4 * n + 0] = a;
    t->ms[4 * n + 1] = b;
    t->ms[4 * n + 2] = c;
    t->ms[4 * n + 3] = k;
  }
  for (int i = 0; i < ndef; ++i) {
    float c = 0;
    HIP_TRY(hipEventElapsedTime(&c, evs.ev[5 * N + 2 * i], evs.ev[5 * N + 2 * i + 1]));
    t->ms[4 * defm[i] + 2] = c;
  }
  *out = g.take();
  return TUCKER_OK;
}

}  // namespace

extern "C" {

tucker_status tucker_sthosvd(const void* data, tucker_dtype dtype, const int64_t* dims, int N, double eps,
                             const int* mode_order, tucker_gram_prec prec, hipStream_t stream, tucker_t** out) {
  return sthosvd_impl(data, dtype, dims, N, eps, nullptr, mode_order, prec, stream, out);
}

tucker_status tucker_sthosvd_ranks(const void* data, tucker_dtype dtype, const int64_t* dims, int N,
                                   const int64_t* ranks, const int* mode_order, tucker_gram_prec prec,
                                   hipStream_t stream, tucker_t** out) {
  if (!ranks) {
    if (out) *out = nullptr;
    return fail(TUCKER_EINVAL, "ranks is NULL");
  }
  return sthosvd_impl(data, dtype, dims, N, 0.0, ranks, mode_order, prec, stream, out);
}

tucker_status tucker_sthosvd_memory(tucker_dtype dtype, const int64_t* dims, int N, const int64_t* ranks,
                                    const int* mode_order, tucker_gram_prec prec, size_t* bytes) {
  if (!bytes) return fail(TUCKER_EINVAL, "bytes is NULL");
  if (dtype != TUCKER_F32 && dtype != TUCKER_F64) return fail(TUCKER_EINVAL, "bad dtype");
  if (prec < TUCKER_GRAM_FP64 || prec > TUCKER_GRAM_BF16X6) return fail(TUCKER_EINVAL, "bad Gram precision");
  tucker_status st = validate_dims(dims, N);
  if (st) return st;
  if (ranks)
    for (int k = 0; k < N; ++k)
      if (ranks[k] < 1) return fail(TUCKER_EINVAL, "ranks[%d] < 1", k);
  int order[TUCKER_MAX_MODES];
  if ((st = validate_order(mode_order, N, order))) return st;
  *bytes = predict_bytes(dtype, dims, N, ranks, order, prec);
  return TUCKER_OK;
}

tucker_status tucker_set_allocator(const tucker_allocator* a) {
  if (a && (!a->alloc || !a->free)) return fail(TUCKER_EINVAL, "allocator needs alloc and free");
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_ext_set = (a != nullptr);
  g_ext = a ? *a : tucker_allocator{};
  return TUCKER_OK;
}

tucker_status tucker_sthosvd_order(int N, const int64_t* dims, const int64_t* ranks, int* order_out,
                                   double* flops_out) {
  if (!dims || !order_out) return fail(TUCKER_EINVAL, "NULL argument");
  tucker_status st = validate_dims(dims, N);
  if (st) return st;
  if (ranks)
    for (int k = 0; k < N; ++k)
      if (ranks[k] < 1) return fail(TUCKER_EINVAL, "ranks[%d] < 1", k);
  if (!ranks) {
    // unknown ranks: increasing size (ties: lower mode first)
    std::vector<int> ord(N);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int i, int j) { return dims[i] < dims[j]; });
    for (int k = 0; k < N; ++k) order_out[k] = ord[k];
    if (flops_out) *flops_out = 0.0;
    return TUCKER_OK;
  }
  // exact minimum over orders of the flop model, by dynamic programming over
  // the set of processed modes: processing mode n after the set P costs
  // (J_n^2 + 2 R_n J_n) K with J_n = I_n and K = prod_{m in P} R_m prod_{m not in P, m != n} I_m
  // (the eigensolve, (10/3) I_n^3, does not depend on the order)
  const int64_t nset = int64_t(1) << N;
  std::vector<double> best(nset, INFINITY);
  std::vector<int8_t> last(nset, -1);
  best[0] = 0.0;
  double R[TUCKER_MAX_MODES];
  for (int k = 0; k < N; ++k) R[k] = (double)std::min(ranks[k], dims[k]);
  for (int64_t P = 0; P < nset; ++P) {
    if (!std::isfinite(best[P])) continue;
    double prodP = 1.0, prodQ = 1.0;  // over processed (ranks) and unprocessed (sizes) modes
    for (int m = 0; m < N; ++m) {
      if (P >> m & 1) prodP *= R[m];
      else prodQ *= (double)dims[m];
    }
    for (int n = 0; n < N; ++n) {
      if (P >> n & 1) continue;
      const double I = (double)dims[n];
      const double K = prodP * (prodQ / I);
      const double c = best[P] + (I * I + 2.0 * R[n] * I) * K;
      const int64_t Q = P | (int64_t(1) << n);
      if (c < best[Q]) {
        best[Q] = c;
        last[Q] = (int8_t)n;
      }
    }
  }
  int64_t P = nset - 1;
  for (int k = N - 1; k >= 0; --k) {
    const int n = last[P];
    order_out[k] = n;
    P &= ~(int64_t(1) << n);
  }
  if (flops_out) *flops_out = best[nset - 1];
  return TUCKER_OK;
}

tucker_status tucker_empty_cache(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TUCKER_EHIP, "no HIP device");
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (int i = (int)g_cache_free.size() - 1; i >= 0; --i)
      if (g_cache_free[i].dev == dev) {
        drop.push_back(g_cache_free[i].p);
        g_cache_free.erase(g_cache_free.begin() + i);
      }
  }
  if (!drop.empty()) {
    HIP_TRY(hipDeviceSynchronize());  // idle blocks may still be read by work in flight
    for (void* p : drop) HIP_TRY(hipFree(p));
  }
  return TUCKER_OK;
}

tucker_status tucker_gram_scaled(const tucker_t* t, int* o) {
  if (!t || !o) return fail(TUCKER_EINVAL, "NULL argument");
  std::memcpy(o, t->scaled, sizeof(int) * t->N);
  return TUCKER_OK;
}

tucker_status tucker_create(const void* core, tucker_dtype core_dtype, const int64_t* dims, const int64_t* ranks,
                            int N, const double* const* factors, hipStream_t stream, tucker_t** out) {
  if (!out) return fail(TUCKER_EINVAL, "out is NULL");
  *out = nullptr;
  if (!core || !ranks || !factors) return fail(TUCKER_EINVAL, "NULL argument");
  if (core_dtype != TUCKER_F32 && core_dtype != TUCKER_F64) return fail(TUCKER_EINVAL, "bad dtype");
  tucker_status st = validate_dims(dims, N);
  if (st) return st;
  for (int k = 0; k < N; ++k) {
    if (ranks[k] < 1 || ranks[k] > dims[k])
      return fail(TUCKER_EINVAL, "rank %lld of mode %d outside 1..%lld", (long long)ranks[k], k, (long long)dims[k]);
    if (!factors[k]) return fail(TUCKER_EINVAL, "factor %d is NULL", k);
  }
  if ((st = ensure_device())) return st;
  HandleGuard g(new tucker_t);
  tucker_t* t = g.t;
  t->N = N;
  t->stream = stream;
  t->core_dtype = core_dtype;
  int64_t ce = 1;
  for (int k = 0; k < N; ++k) {
    t->dims[k] = dims[k];
    t->ranks[k] = ranks[k];
    t->order[k] = k;
    t->prec_used[k] = TUCKER_GRAM_FP64;
    ce *= ranks[k];
    HIP_TRY(t->alloc((void**)&t->U[k], sizeof(double) * dims[k] * ranks[k]));
    HIP_TRY(hipMemcpyAsync(t->U[k], factors[k], sizeof(double) * dims[k] * ranks[k], hipMemcpyDeviceToDevice,
                           stream));
  }
  HIP_TRY(t->alloc(&t->core, dtype_size(core_dtype) * ce));
  HIP_TRY(hipMemcpyAsync(t->core, core, dtype_size(core_dtype) * ce, hipMemcpyDeviceToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  *out = g.take();
  return TUCKER_OK;
}

int tucker_ndims(const tucker_t* t) { return t ? t->N : 0; }

tucker_status tucker_dims(const tucker_t* t, int64_t* o) {
  if (!t || !o) return fail(TUCKER_EINVAL, "NULL argument");
  std::memcpy(o, t->dims, sizeof(int64_t) * t->N);
  return TUCKER_OK;
}

tucker_status tucker_ranks(const tucker_t* t, int64_t* o) {
  if (!t || !o) return fail(TUCKER_EINVAL, "NULL argument");
  std::memcpy(o, t->ranks, sizeof(int64_t) * t->N);
  return TUCKER_OK;
}

tucker_status tucker_mode_order(const tucker_t* t, int* o) {
  if (!t || !o) return fail(TUCKER_EINVAL, "NULL argument");
  std::memcpy(o, t->order, sizeof(int) * t->N);
  return TUCKER_OK;
}

const void* tucker_core(const tucker_t* t, tucker_dtype* dt) {
  if (!t) return nullptr;
  if (dt) *dt = t->core_dtype;
  return t->core;
}

const double* tucker_factor(const tucker_t* t, int n) {
  if (!t || n < 0 || n >= t->N) return nullptr;
  return t->U[n];
}

const double* tucker_eigenvalues(const tucker_t* t, int n, int64_t* count) {
  if (!t || n < 0 || n >= t->N) return nullptr;
  if (count) *count = t->eigcount[n];
  return t->lam[n];
}

double tucker_norm2(const tucker_t* t) { return t ? t->norm2 : 0.0; }

tucker_status tucker_discarded(const tucker_t* t, double* o) {
  if (!t || !o) return fail(TUCKER_EINVAL, "NULL argument");
  std::memcpy(o, t->disc, sizeof(double) * t->N);
  return TUCKER_OK;
}

tucker_status tucker_timings(const tucker_t* t, double* o) {
  if (!t || !o) return fail(TUCKER_EINVAL, "NULL argument");
  std::memcpy(o, t->ms, sizeof(double) * 4 * t->N);
  return TUCKER_OK;
}

tucker_status tucker_gram_precision(const tucker_t* t, tucker_gram_prec* o) {
  if (!t || !o) return fail(TUCKER_EINVAL, "NULL argument");
  std::memcpy(o, t->prec_used, sizeof(tucker_gram_prec) * t->N);
  return TUCKER_OK;
}

void tucker_free(tucker_t* t) {
  if (!t) return;
  t->release();
  delete t;
}

tucker_status tucker_op_size(const tucker_op* op, int64_t I, int64_t* K) {
  if (!op || !K) return fail(TUCKER_EINVAL, "NULL argument");
  if (I < 1) return fail(TUCKER_EINVAL, "mode size %lld < 1", (long long)I);
  const bool ranged = op->kind >= TUCKER_OP_RANGE && op->kind <= TUCKER_OP_MEAN;
  if (ranged && !(op->begin >= 0 && op->begin < op->end && op->end <= I))
    return fail(TUCKER_EINVAL, "operator range [%lld, %lld) invalid for size %lld", (long long)op->begin,
                (long long)op->end, (long long)I);
  switch (op->kind) {
    case TUCKER_OP_IDENTITY: *K = I; return TUCKER_OK;
    case TUCKER_OP_RANGE:
    case TUCKER_OP_AVERAGE:
      if (op->step < 1) return fail(TUCKER_EINVAL, "operator step %lld < 1", (long long)op->step);
      *K = (op->end - op->begin + op->step - 1) / op->step;
      return TUCKER_OK;
    case TUCKER_OP_SUM:
    case TUCKER_OP_MEAN: *K = 1; return TUCKER_OK;
    case TUCKER_OP_MATRIX:
      if (op->rows < 1 || !op->matrix) return fail(TUCKER_EINVAL, "matrix operator needs rows >= 1 and a matrix");
      *K = op->rows;
      return TUCKER_OK;
    default: return fail(TUCKER_EINVAL, "unknown operator kind %d", op->kind);
  }
}

tucker_status tucker_reconstruct_order_rule(int N, const int64_t* ranks, const int64_t* out_sizes,
                                            tucker_order_rule rule, int* order_out) {
  if (rule == TUCKER_ORDER_FLOPS) return tucker_reconstruct_order(N, ranks, out_sizes, order_out);
  if (rule != TUCKER_ORDER_MEMORY) return fail(TUCKER_EINVAL, "unknown order rule %d", (int)rule);
  if (!ranks || !out_sizes || !order_out) return fail(TUCKER_EINVAL, "NULL argument");
  if (N < 1 || N > TUCKER_MAX_MODES) return fail(TUCKER_EINVAL, "N=%d outside 1..%d", N, TUCKER_MAX_MODES);
  for (int k = 0; k < N; ++k)
    if (ranks[k] < 1 || out_sizes[k] < 1) return fail(TUCKER_EINVAL, "sizes must be >= 1");
  std::vector<int> ord(N);
  std::iota(ord.begin(), ord.end(), 0);
  // i before j iff K_i / R_i < K_j / R_j, i.e. K_i R_j < K_j R_i (exact, 128-bit)
  std::stable_sort(ord.begin(), ord.end(), [&](int i, int j) {
    return (__int128)out_sizes[i] * ranks[j] < (__int128)out_sizes[j] * ranks[i];
  });
  for (int k = 0; k < N; ++k) order_out[k] = ord[k];
  return TUCKER_OK;
}

}  // extern "C"

namespace {

// Shared by tucker_reconstruct and tucker_reconstruct_ops: the mode products
// G x_n W_n with W_n = C_n^T diag(s) U_n (s: the post-processing scale of its
// mode), then the separable shift term of the post-processing.
tucker_status reconstruct_impl(const tucker_t* t, const tucker_op* ops, const int* order, tucker_order_rule rule,
                               void* out, tucker_dtype out_dtype, hipStream_t stream) {
  if (!t) return fail(TUCKER_EINVAL, "handle is NULL");
  if (!out) return fail(TUCKER_EINVAL, "out is NULL");
  if (out_dtype != TUCKER_F32 && out_dtype != TUCKER_F64) return fail(TUCKER_EINVAL, "bad dtype");
  const int N = t->N;
  tucker_op op[TUCKER_MAX_MODES];
  int64_t K[TUCKER_MAX_MODES];
  tucker_status st;
  for (int k = 0; k < N; ++k) {
    op[k] = ops ? ops[k] : tucker_op{TUCKER_OP_IDENTITY, 0, 0, 1, 0, nullptr};
    if ((st = tucker_op_size(&op[k], t->dims[k], &K[k]))) return fail(st, "mode %d: %s", k, g_err.c_str());
  }
  int ord[TUCKER_MAX_MODES];
  if (order) {
    if ((st = validate_order(order, N, ord))) return st;
  } else if ((st = tucker_reconstruct_order_rule(N, t->ranks, K, rule, ord))) {
    return st;
  }
  if ((st = ensure_device())) return st;
  // factors: a row slice of U_n read in place where possible, else W_n formed on the device
  const double* M[TUCKER_MAX_MODES];
  int64_t msk[TUCKER_MAX_MODES], msj[TUCKER_MAX_MODES];
  TmpBuf wbuf[TUCKER_MAX_MODES];
  for (int k = 0; k < N; ++k) {
    const bool post = (k == t->post_mode);
    const bool slice =
        !post && (op[k].kind == TUCKER_OP_IDENTITY || (op[k].kind == TUCKER_OP_RANGE && op[k].step == 1));
    if (slice) {
      M[k] = t->U[k] + (op[k].kind == TUCKER_OP_RANGE ? op[k].begin : 0);
      msk[k] = 1;
      msj[k] = t->dims[k];
      continue;
    }
    HIP_TRY(wbuf[k].alloc(sizeof(double) * K[k] * t->ranks[k], stream));
    HIP_TRY(tk::launch_op_factor(op[k].kind, op[k].begin, op[k].end, op[k].step, op[k].matrix, t->dims[k], K[k],
                                 t->ranks[k], t->U[k], post ? t->post_scale : nullptr, wbuf[k].as<double>(), stream));
    M[k] = wbuf[k].as<double>();
    msk[k] = t->ranks[k];
    msj[k] = 1;
  }
  int64_t cur[TUCKER_MAX_MODES];
  std::memcpy(cur, t->ranks, sizeof(int64_t) * N);
  const void* Y = t->core;
  tucker_dtype ydt = t->core_dtype;
  const bool f32p = (t->core_dtype == TUCKER_F32 && out_dtype == TUCKER_F32);
  // A mode-0 product over an odd extent R_0 reads the columns of its
  // unfolding (R_0 consecutive doubles, 8-byte aligned) in 4-byte pieces.
  // When the FP64 product just before it takes the direct-load kernel, that
  // product appends a zero slice to mode 0 (extent R_0 + 1, the output remap)
  // and the mode-0 product multiplies by [W_0 0] with 16-byte loads.
  int zpad_step = -1;
  TmpBuf wpad;
  for (int s = 1; s < N; ++s)
    if (ord[s] == 0 && cur[0] % 2 == 1 && cur[0] > 1 && !f32p && t->core_dtype == TUCKER_F64 && msk[0] == 1) {
      const int n = ord[s - 1];
      int64_t pc[TUCKER_MAX_MODES];  // sizes before step s - 1
      std::memcpy(pc, t->ranks, sizeof(int64_t) * N);
      for (int q = 0; q < s - 1; ++q) pc[ord[q]] = K[ord[q]];
      int64_t L, Rt;
      left_right(pc, N, n, L, Rt);
      // (the core and every intermediate are 16-byte aligned allocations)
      if (L * Rt < (int64_t(1) << 32) && K[0] % 2 == 0 &&
          tk::ttm_dma_eligible((int)pc[n], (uint64_t)L, (uint64_t)(L * Rt), (int)K[n], msk[n], msj[n], 8, 8, t->core,
                               M[n])) {
        zpad_step = s - 1;
        const int64_t J0 = cur[0];
        HIP_TRY(wpad.alloc(sizeof(double) * K[0] * (J0 + 1), stream));
        HIP_TRY(hipMemcpy2DAsync(wpad.p, sizeof(double) * K[0], M[0], sizeof(double) * msj[0], sizeof(double) * K[0],
                                 J0, hipMemcpyDeviceToDevice, stream));
        HIP_TRY(tk::launch_fill(wpad.as<double>() + K[0] * J0, (uint64_t)K[0], 0.0, stream));
      }
    }
  TmpBuf a;
  for (int step = 0; step < N; ++step) {
    const int n = ord[step];
    int64_t total = 1;
    for (int k = 0; k < N; ++k) total *= cur[k];
    int64_t next = total / cur[n] * K[n];
    if (step == zpad_step) next = next / cur[0] * (cur[0] + 1);
    const bool last = (step == N - 1);
    void* Z = out;
    tucker_dtype zdt = out_dtype;
    TmpBuf nb;
    if (!last) {
      zdt = f32p ? TUCKER_F32 : TUCKER_F64;  // intermediates at the precision of the products
      HIP_TRY(nb.alloc(dtype_size(zdt) * next, stream));
      Z = nb.p;
    }
    if (step == zpad_step) {
      int64_t L, Rt;
      left_right(cur, N, n, L, Rt);
      tk::TtmOutRemap rm;
      rm.Lp = 1;
      rm.Pp = cur[0];
      rm.Rp = cur[0] + 1;
      HIP_TRY(tk::launch_ttm_dma(static_cast<const double*>(Y), (int)cur[n], (uint64_t)L, (uint64_t)(L * Rt), M[n],
                                 msk[n], msj[n], (int)K[n], static_cast<double*>(Z), stream, rm));
      cur[0] += 1;
    } else if (n == 0 && zpad_step >= 0) {
      if ((st = run_ttm(Y, ydt, cur, N, n, wpad.as<double>(), K[0], 1, K[0], Z, zdt, f32p, stream))) return st;
    } else if ((st = run_ttm(Y, ydt, cur, N, n, M[n], K[n], msk[n], msj[n], Z, zdt, f32p, stream))) {
      return st;
    }
    a.release();
    if (!last) {
      a.p = nb.p;
      a.s = stream;
      nb.p = nullptr;
      Y = a.p;
      ydt = zdt;
    }
    cur[n] = K[n];
  }
  if (t->post_mode >= 0 && t->post_shift) {
    // + (C_p^T shift) x prod_{m != p} (C_m^T 1): one vector per mode, then a
    // two-factor broadcast over the output (modes below q / from q on)
    int64_t Imax = 1, voff[TUCKER_MAX_MODES], vtot = 0;
    for (int k = 0; k < N; ++k) {
      Imax = std::max(Imax, t->dims[k]);
      voff[k] = vtot;
      vtot += K[k];
    }
    TmpBuf ones, vec;
    HIP_TRY(ones.alloc(sizeof(double) * Imax, stream));
    HIP_TRY(vec.alloc(sizeof(double) * vtot, stream));
    HIP_TRY(tk::launch_fill(ones.as<double>(), (uint64_t)Imax, 1.0, stream));
    for (int k = 0; k < N; ++k) {
      const double* src = (k == t->post_mode) ? t->post_shift : ones.as<double>();
      HIP_TRY(tk::launch_op_factor(op[k].kind, op[k].begin, op[k].end, op[k].step, op[k].matrix, t->dims[k], K[k], 1,
                                   src, nullptr, vec.as<double>() + voff[k], stream));
    }
    tk::OuterGeo g{};
    for (int k = 0; k < N; ++k) {
      g.K[k] = K[k];
      g.voff[k] = voff[k];
    }
    int q = 0;
    uint64_t inner = 1;
    while (q < N && inner < 256) inner *= (uint64_t)K[q++];
    uint64_t outer = 1;
    for (int k = q; k < N; ++k) outer *= (uint64_t)K[k];
    TmpBuf ci, co;
    HIP_TRY(ci.alloc(sizeof(double) * inner, stream));
    HIP_TRY(co.alloc(sizeof(double) * outer, stream));
    HIP_TRY(tk::launch_outer_coef(vec.as<double>(), g, 0, q, inner, ci.as<double>(), stream));
    HIP_TRY(tk::launch_outer_coef(vec.as<double>(), g, q, N, outer, co.as<double>(), stream));
    if (out_dtype == TUCKER_F64)
      HIP_TRY(tk::launch_add_outer(static_cast<double*>(out), inner, outer, ci.as<double>(), co.as<double>(), stream));
    else
      HIP_TRY(tk::launch_add_outer(static_cast<float*>(out), inner, outer, ci.as<double>(), co.as<double>(), stream));
  }
  if (stream != t->stream) {
    // the handle's memory is read on a stream other than its own: tucker_free
    // makes the owning stream wait for this point before reusing it
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(e, stream));
    std::lock_guard<std::mutex> lk(t->foreign_mu);
    t->foreign.push_back(e);
  }
  return TUCKER_OK;
}

}  // namespace

extern "C" {

tucker_status tucker_reconstruct(const tucker_t* t, const int64_t* begin, const int64_t* end, const int* order,
                                 void* out, tucker_dtype out_dtype, hipStream_t stream) {
  if (!t) return fail(TUCKER_EINVAL, "handle is NULL");
  tucker_op op[TUCKER_MAX_MODES];
  for (int k = 0; k < t->N; ++k) {
    const int64_t b = begin ? begin[k] : 0, e = end ? end[k] : t->dims[k];
    if (b < 0 || e > t->dims[k] || b >= e)
      return fail(TUCKER_EINVAL, "mode %d range [%lld, %lld) invalid for size %lld", k, (long long)b, (long long)e,
                  (long long)t->dims[k]);
    op[k] = tucker_op{TUCKER_OP_RANGE, b, e, 1, 0, nullptr};
  }
  return reconstruct_impl(t, op, order, TUCKER_ORDER_FLOPS, out, out_dtype, stream);
}

tucker_status tucker_reconstruct_ops(const tucker_t* t, const tucker_op* ops, const int* order,
                                     tucker_order_rule rule, void* out, tucker_dtype out_dtype, hipStream_t stream) {
  if (rule != TUCKER_ORDER_FLOPS && rule != TUCKER_ORDER_MEMORY)
    return fail(TUCKER_EINVAL, "unknown order rule %d", (int)rule);
  return reconstruct_impl(t, ops, order, rule, out, out_dtype, stream);
}

// ---------------------------------------------------------------- pre/post-processing
tucker_status tucker_slice_stats(const void* X, tucker_dtype dtype, const int64_t* dims, int N, int n, double* stats,
                                 hipStream_t stream) {
  if (!X || !stats) return fail(TUCKER_EINVAL, "NULL pointer");
  if (dtype != TUCKER_F32 && dtype != TUCKER_F64) return fail(TUCKER_EINVAL, "bad dtype");
  tucker_status st = validate_dims(dims, N);
  if (st) return st;
  if (n < 0 || n >= N) return fail(TUCKER_EINVAL, "mode %d outside 0..%d", n, N - 1);
  if ((st = ensure_device())) return st;
  int64_t L, Rt;
  left_right(dims, N, n, L, Rt);
  TmpBuf work;
  HIP_TRY(work.alloc(sizeof(double) * tk::slice_stats_work_doubles(L, dims[n], Rt), stream));
  if (dtype == TUCKER_F64)
    HIP_TRY(tk::launch_slice_stats(static_cast<const double*>(X), L, dims[n], Rt, true, work.as<double>(), stats,
                                   stream));
  else
    HIP_TRY(tk::launch_slice_stats(static_cast<const float*>(X), L, dims[n], Rt, true, work.as<double>(), stats,
                                   stream));
  return TUCKER_OK;
}

tucker_status tucker_scaling_vectors(const double* stats, int64_t J, tucker_scale_method method, double* shift,
                                     double* scale, hipStream_t stream) {
  if (!stats || !shift || !scale) return fail(TUCKER_EINVAL, "NULL pointer");
  if (J < 1) return fail(TUCKER_EINVAL, "J=%lld < 1", (long long)J);
  if (method != TUCKER_SCALE_STANDARDIZE && method != TUCKER_SCALE_MAX)
    return fail(TUCKER_EINVAL, "unknown scaling method %d", (int)method);
  tucker_status st;
  if ((st = ensure_device())) return st;
  HIP_TRY(tk::launch_scaling_vectors(stats, (uint64_t)J, (int)method, shift, scale, stream));
  return TUCKER_OK;
}

tucker_status tucker_slice_transform(const void* X, tucker_dtype xdtype, const int64_t* dims, int N, int n,
                                     const double* shift, const double* scale, int inverse, void* Y,
                                     tucker_dtype ydtype, hipStream_t stream) {
  if (!X || !Y || !shift || !scale) return fail(TUCKER_EINVAL, "NULL pointer");
  if ((xdtype != TUCKER_F32 && xdtype != TUCKER_F64) || (ydtype != TUCKER_F32 && ydtype != TUCKER_F64))
    return fail(TUCKER_EINVAL, "bad dtype");
  tucker_status st = validate_dims(dims, N);
  if (st) return st;
  if (n < 0 || n >= N) return fail(TUCKER_EINVAL, "mode %d outside 0..%d", n, N - 1);
  if (X == Y && xdtype != ydtype) return fail(TUCKER_EINVAL, "in-place transform needs equal dtypes");
  if ((st = ensure_device())) return st;
  int64_t L, Rt;
  left_right(dims, N, n, L, Rt);
  const uint64_t total = (uint64_t)(L * dims[n] * Rt);
  const bool inv = inverse != 0;
  if (xdtype == TUCKER_F32 && ydtype == TUCKER_F32)
    HIP_TRY(tk::launch_slice_transform(static_cast<const float*>(X), static_cast<float*>(Y), total, L, dims[n], shift,
                                       scale, inv, stream));
  else if (xdtype == TUCKER_F32)
    HIP_TRY(tk::launch_slice_transform(static_cast<const float*>(X), static_cast<double*>(Y), total, L, dims[n], shift,
                                       scale, inv, stream));
  else if (ydtype == TUCKER_F32)
    HIP_TRY(tk::launch_slice_transform(static_cast<const double*>(X), static_cast<float*>(Y), total, L, dims[n],
                                       shift, scale, inv, stream));
  else
    HIP_TRY(tk::launch_slice_transform(static_cast<const double*>(X), static_cast<double*>(Y), total, L, dims[n],
                                       shift, scale, inv, stream));
  return TUCKER_OK;
}

tucker_status tucker_preprocess(const void* X, tucker_dtype xdtype, const int64_t* dims, int N, int n,
                                tucker_scale_method method, void* Y, tucker_dtype ydtype, double* shift,
                                double* scale, hipStream_t stream) {
  if (!shift || !scale) return fail(TUCKER_EINVAL, "NULL pointer");
  tucker_status st = validate_dims(dims, N);
  if (st) return st;
  if (n < 0 || n >= N) return fail(TUCKER_EINVAL, "mode %d outside 0..%d", n, N - 1);
  if ((st = ensure_device())) return st;
  TmpBuf stats;
  HIP_TRY(stats.alloc(sizeof(double) * TUCKER_NSTATS * dims[n], stream));
  if ((st = tucker_slice_stats(X, xdtype, dims, N, n, stats.as<double>(), stream))) return st;
  if ((st = tucker_scaling_vectors(stats.as<double>(), dims[n], method, shift, scale, stream))) return st;
  return tucker_slice_transform(X, xdtype, dims, N, n, shift, scale, 0, Y, ydtype, stream);
}

tucker_status tucker_set_postprocess(tucker_t* t, int n, const double* shift, const double* scale,
                                     hipStream_t stream) {
  if (!t || !scale) return fail(TUCKER_EINVAL, "NULL argument");
  if (n < 0 || n >= t->N) return fail(TUCKER_EINVAL, "mode %d outside 0..%d", n, t->N - 1);
  tucker_status st;
  if ((st = ensure_device())) return st;
  if (t->post_mode >= 0 && t->post_mode != n)
    return fail(TUCKER_EINVAL, "post-processing is already attached to mode %d", t->post_mode);
  const size_t bytes = sizeof(double) * t->dims[n];
  // the vectors may still be being written on `stream`
  HIP_TRY(hipStreamSynchronize(stream));
  if (!t->post_scale) HIP_TRY(t->alloc((void**)&t->post_scale, bytes));
  if (shift && !t->post_shift_buf) HIP_TRY(t->alloc((void**)&t->post_shift_buf, bytes));
  HIP_TRY(hipMemcpyAsync(t->post_scale, scale, bytes, hipMemcpyDeviceToDevice, t->stream));
  if (shift) HIP_TRY(hipMemcpyAsync(t->post_shift_buf, shift, bytes, hipMemcpyDeviceToDevice, t->stream));
  HIP_TRY(hipStreamSynchronize(t->stream));
  t->post_shift = shift ? t->post_shift_buf : nullptr;
  t->post_mode = n;
  return TUCKER_OK;
}

tucker_status tucker_gram(const void* Y, tucker_dtype dtype, const int64_t* dims, int N, int n,
                          tucker_gram_prec prec, double* S, double* norm2, hipStream_t stream) {
  if (!Y || !S) return fail(TUCKER_EINVAL, "NULL pointer");
  if (dtype != TUCKER_F32 && dtype != TUCKER_F64) return fail(TUCKER_EINVAL, "bad dtype");
  tucker_status st = validate_dims(dims, N);
  if (st) return st;
  if (n < 0 || n >= N) return fail(TUCKER_EINVAL, "mode %d outside 0..%d", n, N - 1);
  if (prec < TUCKER_GRAM_FP64 || prec > TUCKER_GRAM_BF16X6) return fail(TUCKER_EINVAL, "bad Gram precision");
  if (prec != TUCKER_GRAM_FP64 && dtype != TUCKER_F32)
    return fail(TUCKER_EINVAL, "reduced-precision Gram needs FP32 data");
  if ((st = ensure_device())) return st;
  return run_gram(Y, dtype, dims, N, n, prec, S, norm2, stream);
}

}  // extern "C"

namespace {

// Workspace of tucker_eig_truncate_noalloc: the eigensolver's workspace for
// J up to 1024 (2 J^2 + 3 J + 8 doubles, 16.8 MB; the allocating entry point
// goes further), one copy per device for the life of the process.  Host code
// never uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr int64_t kNoAllocMaxJ = 1024;
constexpr int64_t kNoAllocDoubles = 2 * kNoAllocMaxJ * kNoAllocMaxJ + 3 * kNoAllocMaxJ + 8;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[64];

tucker_status scratch_address(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(TUCKER_EUNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(TUCKER_EHIP, "hipGetSymbolAddress returned no address for the static workspace");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return TUCKER_OK;
}

}  // namespace

extern "C" {

tucker_status tucker_eig_truncate_noalloc(const double* S, int64_t J, double thr, double* lam, double* U,
                                          int64_t* R, double* disc, hipStream_t stream) {
  if (!S || !lam || !U || !R || !disc) return fail(TUCKER_EINVAL, "NULL pointer");
  if (J < 1 || J > kNoAllocMaxJ)
    return fail(TUCKER_EINVAL, "J=%lld outside 1..%lld (the static workspace holds the eigensolver of J <= %lld)",
                (long long)J, (long long)kNoAllocMaxJ, (long long)kNoAllocMaxJ);
  if (!(thr >= 0.0) || !std::isfinite(thr)) return fail(TUCKER_EINVAL, "thr must be finite and >= 0");
  tucker_status st;
  if ((st = ensure_device())) return st;
  double* ws = nullptr;
  if ((st = scratch_address(&ws))) return st;
  tk::EigWork w;
  tk::eig_work_carve(ws, J, w);
  HIP_TRY(tk::launch_eig_truncate(S, (int)J, thr, nullptr, 0, w, lam, U, R, disc, stream));
  return TUCKER_OK;
}

tucker_status tucker_eig_truncate(const double* S, int64_t J, double thr, double* lam, double* U, int64_t* R,
                                  double* disc, hipStream_t stream) {
  if (!S || !lam || !U || !R || !disc) return fail(TUCKER_EINVAL, "NULL pointer");
  if (J < 1 || J > kMaxEigJ) return fail(TUCKER_EINVAL, "J=%lld outside 1..%lld", (long long)J, (long long)kMaxEigJ);
  if (!(thr >= 0.0) || !std::isfinite(thr)) return fail(TUCKER_EINVAL, "thr must be finite and >= 0");
  tucker_status st;
  if ((st = ensure_device())) return st;
  TmpBuf wb;
  HIP_TRY(wb.alloc(sizeof(double) * tk::eig_work_doubles(J), stream));
  tk::EigWork w;
  tk::eig_work_carve(wb.as<double>(), J, w);
  HIP_TRY(tk::launch_eig_truncate(S, (int)J, thr, nullptr, 0, w, lam, U, R, disc, stream));
  return TUCKER_OK;
}

tucker_status tucker_ttm(const void* Y, tucker_dtype ydtype, const int64_t* dims, int N, int n, const double* M,
                         int64_t K, int64_t msk, int64_t msj, void* Z, tucker_dtype zdtype, int fp32_products,
                         hipStream_t stream) {
  if (!Y || !M || !Z) return fail(TUCKER_EINVAL, "NULL pointer");
  if ((ydtype != TUCKER_F32 && ydtype != TUCKER_F64) || (zdtype != TUCKER_F32 && zdtype != TUCKER_F64))
    return fail(TUCKER_EINVAL, "bad dtype");
  tucker_status st = validate_dims(dims, N);
  if (st) return st;
  if (n < 0 || n >= N) return fail(TUCKER_EINVAL, "mode %d outside 0..%d", n, N - 1);
  if (K < 1) return fail(TUCKER_EINVAL, "K=%lld < 1", (long long)K);
  if ((st = ensure_device())) return st;
  return run_ttm(Y, ydtype, dims, N, n, M, K, msk, msj, Z, zdtype, fp32_products != 0, stream);
}

}  // extern "C"

// ======================================================================
// Batching form: many independent tensors, device-side sizes, no host
// synchronisation between steps (tucker_batch_run only enqueues kernels).
// ======================================================================
namespace {

__global__ void batch_reset_cur_kernel(const int64_t* __restrict__ dims0, int64_t* __restrict__ cur, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cur[i] = dims0[i];
}

__global__ void batch_zero_int_kernel(int* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void batch_set_rank_kernel(const int64_t* __restrict__ R, int count, int N, int n,
                                      int64_t* __restrict__ cur) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) cur[(int64_t)t * N + n] = R[t];
}

// Tile choices of the batched kernels, picked by timing candidates on the
// first plan of a given shape class and remembered for the process.
struct BatchTiles {
  int gram_chunks;  // Gram chunks per work item
  int ttm_tiles;    // TTM column tiles (64 columns) per work item
};
std::mutex g_tune_mu;
std::vector<std::pair<std::string, BatchTiles>> g_tuned;

}  // namespace

struct tucker_batch {
  int count = 0, N = 0;
  int order[TUCKER_MAX_MODES] = {0};
  tucker_gram_prec prec = TUCKER_GRAM_FP64;
  tucker_dtype in_dt = TUCKER_F64, wdt = TUCKER_F64;
  double eps = 0.0;
  hipStream_t alloc_stream = nullptr, run_stream = nullptr;
  bool ran = false;
  BatchTiles tiles{64, 8};
  std::vector<int64_t> dims;      // host, count x N
  std::vector<int64_t> off;       // element offset of tensor t in the work buffers
  int Jmax[TUCKER_MAX_MODES] = {0};
  std::vector<void*> owned;
  // device
  int64_t *dims0 = nullptr, *cur = nullptr;
  void* buf[2] = {nullptr, nullptr};
  const void** ptrY[TUCKER_MAX_MODES] = {nullptr};
  void** ptrZ[TUCKER_MAX_MODES] = {nullptr};
  int* Jd[TUCKER_MAX_MODES] = {nullptr};
  int64_t* gitems[TUCKER_MAX_MODES] = {nullptr};
  int* gfirst[TUCKER_MAX_MODES] = {nullptr};
  int gn[TUCKER_MAX_MODES] = {0}, gsmall[TUCKER_MAX_MODES] = {0};
  int64_t* titems[TUCKER_MAX_MODES] = {nullptr};
  int tn[TUCKER_MAX_MODES] = {0};
  double *part = nullptr, *sq = nullptr, *S = nullptr, *A = nullptr, *Zt = nullptr, *dd = nullptr, *ee = nullptr,
         *tau = nullptr, *scal = nullptr, *nx2 = nullptr;
  double* sqs = nullptr;  // per step s >= 1 and tensor: FP64 sum of squares of the working tensor
  int* gflag = nullptr;   // per tensor: the last reduced Gram was flagged by the range guard
  int* status = nullptr;  // per tensor: 1 non-finite data, 2 a Gram recomputed in FP64
  double* U[TUCKER_MAX_MODES] = {nullptr};
  double* lam[TUCKER_MAX_MODES] = {nullptr};
  int64_t* R[TUCKER_MAX_MODES] = {nullptr};
  double* disc[TUCKER_MAX_MODES] = {nullptr};
  // host copies, refreshed by every result query
  std::vector<int64_t> hR;     // count x N
  std::vector<double> hnorm2;  // count
  std::vector<double> hdisc;   // count x N
  std::vector<int> hstatus;    // count

  hipError_t alloc(void** p, size_t bytes) {
    hipError_t e = dev_alloc(p, bytes, alloc_stream);
    if (e == hipSuccess) owned.push_back(*p);
    return e;
  }
  template <typename T>
  hipError_t upload(T** dst, const std::vector<T>& v) {
    hipError_t e = alloc((void**)dst, sizeof(T) * std::max<size_t>(1, v.size()));
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    // the host vector is temporary: wait for the copy
    e = hipMemcpyAsync(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, alloc_stream);
    return e == hipSuccess ? hipStreamSynchronize(alloc_stream) : e;
  }
  void release() {
    if (run_stream) (void)hipStreamSynchronize(run_stream);
    for (void* p : owned) dev_free(p, alloc_stream);
    owned.clear();
  }
};

namespace {

size_t wsize(tucker_dtype t) { return t == TUCKER_F64 ? 8 : 4; }

// Host plan of the work items of step s (sizes bounded by the original ones).
void plan_step_items(const tucker_batch* b, int s, const BatchTiles& tiles, std::vector<int64_t>& gitems,
                     std::vector<int>& gfirst, int& nsmall, std::vector<int64_t>& titems, int64_t& part_elems) {
  const int N = b->N, n = b->order[s];
  const int KC = (b->prec == TUCKER_GRAM_FP64) ? 16 : 32;
  gitems.clear();
  titems.clear();
  gfirst.assign(2 * (size_t)b->count, 0);
  part_elems = 0;
  nsmall = 0;
  for (int pass = 0; pass < 2; ++pass) {  // tensors with J <= 80 first
    for (int t = 0; t < b->count; ++t) {
      const int64_t* d = &b->dims[(size_t)t * N];
      const int64_t J = d[n];
      if ((J <= 80) != (pass == 0)) continue;
      int64_t K = 1;
      for (int k = 0; k < N; ++k)
        if (k != n) K *= d[k];
      const int64_t nch = ceil_div(K, KC);
      const int64_t nb = (J + 15) / 16, nblk = nb * (nb + 1) / 2;
      gfirst[2 * t] = (int)(gitems.size() / 4);
      for (int64_t c0 = 0; c0 < nch; c0 += tiles.gram_chunks) {
        gitems.push_back(t);
        gitems.push_back(c0);
        gitems.push_back(std::min<int64_t>(nch, c0 + tiles.gram_chunks));
        gitems.push_back(part_elems);
        part_elems += nblk * 256;
      }
      gfirst[2 * t + 1] = (int)(gitems.size() / 4);
      const int64_t nct = ceil_div(K, 64);
      for (int64_t c0 = 0; c0 < nct; c0 += tiles.ttm_tiles) {
        titems.push_back(t);
        titems.push_back(c0);
        titems.push_back(std::min<int64_t>(nct, c0 + tiles.ttm_tiles));
      }
    }
    if (pass == 0) nsmall = (int)(gitems.size() / 4);
  }
}

tucker_status batch_enqueue_gram(tucker_batch* b, int s, hipStream_t stream) {
  const int n = b->order[s];
  tk::GramBatch g{};
  g.count = b->count;
  g.N = b->N;
  g.n = n;
  g.Jmax = b->Jmax[s];
  g.Y = b->ptrY[s];
  g.cur = b->cur;
  g.J = b->Jd[s];
  g.items = b->gitems[s];
  g.nitems = b->gn[s];
  g.nsmall = b->gsmall[s];
  g.ifirst = b->gfirst[s];
  g.part = b->part;
  g.sq = b->sq;
  g.S = b->S;
  // per-tensor FP64 sums of squares: ||X_t||^2 at the first step, the working
  // tensor's later (the range guard compares the trace with them)
  g.nx2 = (s == 0) ? b->nx2 : b->sqs + (size_t)s * b->count;
  g.flag = nullptr;
  g.chunk_mul = 1;
  const tucker_dtype ydt = (s == 0) ? b->in_dt : b->wdt;
  if (ydt == TUCKER_F64) HIP_TRY(tk::launch_gram_batched<double>(g, (int)b->prec, n == 0, stream));
  else HIP_TRY(tk::launch_gram_batched<float>(g, (int)b->prec, n == 0, stream));
  if (b->prec != TUCKER_GRAM_FP64) {
    // range guard per tensor, then the flagged tensors' Grams again in FP64
    // (launched unconditionally; items of other tensors return at once, so a
    // captured run stays valid whatever the data)
    HIP_TRY(tk::launch_gram_guard_batched(g, b->gflag, b->status, stream));
    tk::GramBatch g2 = g;
    g2.flag = b->gflag;
    g2.chunk_mul = 2;  // the plan's 32-column chunks in FP64's 16-column chunks
    g2.nx2 = nullptr;
    g2.sq = nullptr;
    HIP_TRY(tk::launch_gram_batched<float>(g2, (int)TUCKER_GRAM_FP64, n == 0, stream));
  }
  return TUCKER_OK;
}

tucker_status batch_enqueue_ttm(tucker_batch* b, int s, hipStream_t stream) {
  const int n = b->order[s];
  tk::TtmBatch m{};
  m.count = b->count;
  m.N = b->N;
  m.n = n;
  m.Jmax = b->Jmax[s];
  m.Y = b->ptrY[s];
  m.Z = b->ptrZ[s];
  m.cur = b->cur;
  m.J = b->Jd[s];
  m.R = b->R[n];
  m.U = b->U[n];
  m.items = b->titems[s];
  m.nitems = b->tn[s];
  const bool f32p = (b->prec != TUCKER_GRAM_FP64);
  const tucker_dtype ydt = (s == 0) ? b->in_dt : b->wdt;
  if (ydt == TUCKER_F32 && b->wdt == TUCKER_F32) HIP_TRY((tk::launch_ttm_batched<float, float>(m, f32p, n == 0, stream)));
  else if (ydt == TUCKER_F32) HIP_TRY((tk::launch_ttm_batched<float, double>(m, f32p, n == 0, stream)));
  else HIP_TRY((tk::launch_ttm_batched<double, double>(m, f32p, n == 0, stream)));
  return TUCKER_OK;
}

tucker_status batch_enqueue_eig(tucker_batch* b, int s, hipStream_t stream) {
  const int n = b->order[s];
  tk::EigBatch e{};
  e.count = b->count;
  e.Jmax = b->Jmax[s];
  e.J = b->Jd[s];
  e.S = b->S;
  e.A = b->A;
  e.Zt = b->Zt;
  e.d = b->dd;
  e.e = b->ee;
  e.tau = b->tau;
  e.lam = b->lam[n];
  e.scal = b->scal;
  e.U = b->U[n];
  e.R = b->R[n];
  e.disc = b->disc[n];
  e.nx2 = b->nx2;
  HIP_TRY(tk::launch_eig_truncate_batched(e, b->eps * b->eps / b->N, stream));
  hipLaunchKernelGGL(batch_set_rank_kernel, dim3(ceil_div(b->count, 256)), dim3(256), 0, stream, b->R[n], b->count,
                     b->N, n, b->cur);
  HIP_TRY(hipGetLastError());
  return TUCKER_OK;
}

tucker_status batch_enqueue_all(tucker_batch* b, hipStream_t stream) {
  const int64_t nc = (int64_t)b->count * b->N;
  hipLaunchKernelGGL(batch_reset_cur_kernel, dim3(ceil_div(nc, 256)), dim3(256), 0, stream, b->dims0, b->cur, nc);
  hipLaunchKernelGGL(batch_zero_int_kernel, dim3(ceil_div(b->count, 256)), dim3(256), 0, stream, b->status,
                     (int64_t)b->count);
  HIP_TRY(hipGetLastError());
  tucker_status st;
  for (int s = 0; s < b->N; ++s) {
    if ((st = batch_enqueue_gram(b, s, stream))) return st;
    if ((st = batch_enqueue_eig(b, s, stream))) return st;
    if ((st = batch_enqueue_ttm(b, s, stream))) return st;
  }
  return TUCKER_OK;
}

// Upload the step plans for `tiles` (items, first-item table).
tucker_status batch_upload_plans(tucker_batch* b, const BatchTiles& tiles, int64_t& part_max, int& items_max) {
  part_max = 0;
  items_max = 0;
  for (int s = 0; s < b->N; ++s) {
    std::vector<int64_t> gi, ti;
    std::vector<int> gf;
    int nsmall = 0;
    int64_t pe = 0;
    plan_step_items(b, s, tiles, gi, gf, nsmall, ti, pe);
    // one workgroup per item (512 threads for the Gram, 256 for the product):
    // the work-items of a launch stay below 2^32
    if (gi.size() / 4 >= (size_t(1) << 23) || ti.size() / 3 >= (size_t(1) << 24))
      return fail(TUCKER_EUNSUPPORTED, "step %d: %zu Gram and %zu product work items, above 2^23 and 2^24", s,
                  gi.size() / 4, ti.size() / 3);
    HIP_TRY(b->upload(&b->gitems[s], gi));
    HIP_TRY(b->upload(&b->gfirst[s], gf));
    HIP_TRY(b->upload(&b->titems[s], ti));
    b->gn[s] = (int)(gi.size() / 4);
    b->gsmall[s] = nsmall;
    b->tn[s] = (int)(ti.size() / 3);
    part_max = std::max(part_max, pe);
    items_max = std::max(items_max, b->gn[s]);
  }
  return TUCKER_OK;
}

std::string tune_key(const tucker_batch* b) {
  // shape class: count, N, precision, input type and the total size to within 2x
  int64_t tot = 0;
  for (int t = 0; t < b->count; ++t) {
    int64_t e = 1;
    for (int k = 0; k < b->N; ++k) e *= b->dims[(size_t)t * b->N + k];
    tot += e;
  }
  int lg = 0;
  while ((int64_t(1) << lg) < tot) ++lg;
  char buf[128];
  snprintf(buf, sizeof buf, "%d/%d/%d/%d/%d", b->count, b->N, (int)b->prec, (int)b->in_dt, lg);
  return buf;
}

}  // namespace

extern "C" {

tucker_status tucker_batch_create(int count, const void* const* data, tucker_dtype dtype, const int64_t* dims, int N,
                                  double eps, const int* mode_order, tucker_gram_prec prec, hipStream_t stream,
                                  tucker_batch** out) {
  if (!out) return fail(TUCKER_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1) return fail(TUCKER_EINVAL, "count=%d < 1", count);
  // one workgroup of up to 1024 threads per tensor in the batched eigensolver:
  // the work-items of a launch stay below 2^32
  if (count >= (1 << 22)) return fail(TUCKER_EINVAL, "count=%d above %d", count, (1 << 22) - 1);
  if (!data || !dims) return fail(TUCKER_EINVAL, "NULL argument");
  if (dtype != TUCKER_F32 && dtype != TUCKER_F64) return fail(TUCKER_EINVAL, "bad dtype");
  if (prec < TUCKER_GRAM_FP64 || prec > TUCKER_GRAM_AUTO) return fail(TUCKER_EINVAL, "bad Gram precision");
  if (prec != TUCKER_GRAM_FP64 && prec != TUCKER_GRAM_AUTO && dtype != TUCKER_F32)
    return fail(TUCKER_EINVAL, "reduced-precision Gram needs FP32 data");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(TUCKER_EINVAL, "eps must be finite and >= 0");
  tucker_status st;
  if (N < 1 || N > TUCKER_MAX_MODES) return fail(TUCKER_EINVAL, "N=%d outside 1..%d", N, TUCKER_MAX_MODES);
  if (prec == TUCKER_GRAM_AUTO) prec = resolve_auto(dtype, N, eps, false);
  for (int t = 0; t < count; ++t) {
    if (!data[t]) return fail(TUCKER_EINVAL, "data[%d] is NULL", t);
    if ((st = validate_dims(dims + (size_t)t * N, N))) return st;
    for (int k = 0; k < N; ++k)
      if (dims[(size_t)t * N + k] > tk::kBatchMaxJ)
        return fail(TUCKER_EUNSUPPORTED, "tensor %d mode %d has size %lld; the batched form supports up to %d", t, k,
                    (long long)dims[(size_t)t * N + k], tk::kBatchMaxJ);
  }
  int order[TUCKER_MAX_MODES];
  if ((st = validate_order(mode_order, N, order))) return st;
  if ((st = ensure_device())) return st;

  struct Guard {
    tucker_batch* b;
    ~Guard() {
      if (b) {
        b->release();
        delete b;
      }
    }
  } g{new tucker_batch};
  tucker_batch* b = g.b;
  b->count = count;
  b->N = N;
  std::memcpy(b->order, order, sizeof(int) * N);
  b->prec = prec;
  b->in_dt = dtype;
  b->wdt = (prec == TUCKER_GRAM_FP64) ? TUCKER_F64 : TUCKER_F32;
  b->eps = eps;
  b->alloc_stream = stream;
  b->dims.assign(dims, dims + (size_t)count * N);
  b->off.resize(count + 1);
  b->off[0] = 0;
  for (int t = 0; t < count; ++t) {
    int64_t e = 1;
    for (int k = 0; k < N; ++k) e *= dims[(size_t)t * N + k];
    b->off[t + 1] = b->off[t] + e;
  }
  const int64_t total = b->off[count];
  int Jall = 0;
  for (int s = 0; s < N; ++s) {
    int m = 0;
    for (int t = 0; t < count; ++t) m = std::max<int>(m, (int)dims[(size_t)t * N + order[s]]);
    b->Jmax[s] = m;
    Jall = std::max(Jall, m);
  }
  const size_t ws = wsize(b->wdt);
  HIP_TRY(b->upload(&b->dims0, b->dims));
  HIP_TRY(b->alloc((void**)&b->cur, sizeof(int64_t) * (size_t)count * N));
  HIP_TRY(b->alloc(&b->buf[0], ws * (size_t)total));
  if (N > 1) HIP_TRY(b->alloc(&b->buf[1], ws * (size_t)total));
  // per-step operand and result pointers
  for (int s = 0; s < N; ++s) {
    std::vector<const void*> py(count);
    std::vector<void*> pz(count);
    std::vector<int> Jv(count);
    for (int t = 0; t < count; ++t) {
      py[t] = (s == 0) ? data[t] : static_cast<const char*>(b->buf[(s - 1) % 2]) + ws * b->off[t];
      pz[t] = static_cast<char*>(b->buf[s % 2]) + ws * b->off[t];
      Jv[t] = (int)dims[(size_t)t * N + order[s]];
    }
    HIP_TRY(b->upload((const void***)&b->ptrY[s], py));
    HIP_TRY(b->upload(&b->ptrZ[s], pz));
    HIP_TRY(b->upload(&b->Jd[s], Jv));
  }
  const size_t J2 = (size_t)Jall * Jall;
  HIP_TRY(b->alloc((void**)&b->S, sizeof(double) * J2 * count));
  HIP_TRY(b->alloc((void**)&b->A, sizeof(double) * J2 * count));
  HIP_TRY(b->alloc((void**)&b->Zt, sizeof(double) * J2 * count));
  HIP_TRY(b->alloc((void**)&b->dd, sizeof(double) * Jall * count));
  HIP_TRY(b->alloc((void**)&b->ee, sizeof(double) * Jall * count));
  HIP_TRY(b->alloc((void**)&b->tau, sizeof(double) * Jall * count));
  HIP_TRY(b->alloc((void**)&b->scal, sizeof(double) * 8 * count));
  HIP_TRY(b->alloc((void**)&b->nx2, sizeof(double) * count));
  HIP_TRY(b->alloc((void**)&b->sqs, sizeof(double) * count * N));
  HIP_TRY(b->alloc((void**)&b->gflag, sizeof(int) * count));
  HIP_TRY(b->alloc((void**)&b->status, sizeof(int) * count));
  for (int s = 0; s < N; ++s) {
    const int n = order[s];
    const size_t Jn = (size_t)b->Jmax[s];
    HIP_TRY(b->alloc((void**)&b->U[n], sizeof(double) * Jn * Jn * count));
    HIP_TRY(b->alloc((void**)&b->lam[n], sizeof(double) * Jn * count));
    HIP_TRY(b->alloc((void**)&b->R[n], sizeof(int64_t) * count));
    HIP_TRY(b->alloc((void**)&b->disc[n], sizeof(double) * count));
  }
  // tile choice: remembered per shape class, else tuned on this batch's first step
  const std::string key = tune_key(b);
  bool have = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& kv : g_tuned)
      if (kv.first == key) {
        b->tiles = kv.second;
        have = true;
      }
  }
  const BatchTiles cands[] = {{16, 2}, {64, 8}, {256, 32}};
  int64_t part_max = 0;
  int items_max = 0;
  if (!have) {
    // allocate for the largest plan among the candidates
    int64_t pm = 0;
    int im = 0;
    for (const BatchTiles& c : cands) {
      for (int s = 0; s < N; ++s) {
        std::vector<int64_t> gi, ti;
        std::vector<int> gf;
        int ns = 0;
        int64_t pe = 0;
        plan_step_items(b, s, c, gi, gf, ns, ti, pe);
        pm = std::max(pm, pe);
        im = std::max(im, (int)(gi.size() / 4));
      }
    }
    HIP_TRY(b->alloc((void**)&b->part, sizeof(double) * std::max<int64_t>(pm, 1)));
    HIP_TRY(b->alloc((void**)&b->sq, sizeof(double) * std::max(im, 1)));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float bestg = 1e30f, bestt = 1e30f;
    BatchTiles best = cands[1];
    int64_t nc = (int64_t)count * N;
    for (const BatchTiles& c : cands) {
      if ((st = batch_upload_plans(b, c, part_max, items_max))) return st;
      hipLaunchKernelGGL(batch_reset_cur_kernel, dim3(ceil_div(nc, 256)), dim3(256), 0, stream, b->dims0, b->cur, nc);
      float tg = 0.f, tt = 0.f;
      for (int rep = 0; rep < 3; ++rep) {  // first repetition warms up
        HIP_TRY(hipEventRecord(e0, stream));
        if ((st = batch_enqueue_gram(b, 0, stream))) return st;
        HIP_TRY(hipEventRecord(e1, stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) tg += ms;
        if (rep == 0 && (st = batch_enqueue_eig(b, 0, stream))) return st;
        HIP_TRY(hipEventRecord(e0, stream));
        if ((st = batch_enqueue_ttm(b, 0, stream))) return st;
        HIP_TRY(hipEventRecord(e1, stream));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) tt += ms;
      }
      if (tg < bestg) {
        bestg = tg;
        best.gram_chunks = c.gram_chunks;
      }
      if (tt < bestt) {
        bestt = tt;
        best.ttm_tiles = c.ttm_tiles;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->tiles = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.push_back({key, best});
  }
  if ((st = batch_upload_plans(b, b->tiles, part_max, items_max))) return st;
  if (have) {
    HIP_TRY(b->alloc((void**)&b->part, sizeof(double) * std::max<int64_t>(part_max, 1)));
    HIP_TRY(b->alloc((void**)&b->sq, sizeof(double) * std::max(items_max, 1)));
  }
  HIP_TRY(hipStreamSynchronize(stream));  // uploads done; host vectors may go
  *out = g.b;
  g.b = nullptr;
  return TUCKER_OK;
}

tucker_status tucker_batch_run(tucker_batch* b, hipStream_t stream) {
  if (!b) return fail(TUCKER_EINVAL, "batch is NULL");
  b->run_stream = stream;
  b->ran = true;
  return batch_enqueue_all(b, stream);
}

tucker_status tucker_sthosvd_batched(int count, const void* const* data, tucker_dtype dtype, const int64_t* dims,
                                     int N, double eps, const int* mode_order, tucker_gram_prec prec,
                                     hipStream_t stream, tucker_batch** out) {
  tucker_status st = tucker_batch_create(count, data, dtype, dims, N, eps, mode_order, prec, stream, out);
  if (st) return st;
  st = tucker_batch_run(*out, stream);
  if (st) {
    tucker_batch_free(*out);
    *out = nullptr;
  }
  return st;
}

}  // extern "C"

namespace {

tucker_status batch_sync(tucker_batch* b) {
  // re-read every time: a captured run may have been replayed since
  if (!b->ran) return fail(TUCKER_EINVAL, "the batch has not been run");
  HIP_TRY(hipStreamSynchronize(b->run_stream));
  const int C = b->count, N = b->N;
  b->hR.assign((size_t)C * N, 0);
  b->hdisc.assign((size_t)C * N, 0.0);
  b->hnorm2.assign(C, 0.0);
  std::vector<int64_t> r(C);
  std::vector<double> d(C);
  for (int n = 0; n < N; ++n) {
    HIP_TRY(hipMemcpy(r.data(), b->R[n], sizeof(int64_t) * C, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(d.data(), b->disc[n], sizeof(double) * C, hipMemcpyDeviceToHost));
    for (int t = 0; t < C; ++t) {
      b->hR[(size_t)t * N + n] = r[t];
      b->hdisc[(size_t)t * N + n] = d[t];
    }
  }
  HIP_TRY(hipMemcpy(b->hnorm2.data(), b->nx2, sizeof(double) * C, hipMemcpyDeviceToHost));
  b->hstatus.assign(C, 0);
  HIP_TRY(hipMemcpy(b->hstatus.data(), b->status, sizeof(int) * C, hipMemcpyDeviceToHost));
  return TUCKER_OK;
}

}  // namespace

extern "C" {

tucker_status tucker_batch_ranks(tucker_batch* b, int64_t* ranks_out) {
  if (!b || !ranks_out) return fail(TUCKER_EINVAL, "NULL argument");
  tucker_status st = batch_sync(b);
  if (st) return st;
  std::memcpy(ranks_out, b->hR.data(), sizeof(int64_t) * b->hR.size());
  return TUCKER_OK;
}

tucker_status tucker_batch_norm2(tucker_batch* b, double* norm2_out) {
  if (!b || !norm2_out) return fail(TUCKER_EINVAL, "NULL argument");
  tucker_status st = batch_sync(b);
  if (st) return st;
  std::memcpy(norm2_out, b->hnorm2.data(), sizeof(double) * b->count);
  return TUCKER_OK;
}

tucker_status tucker_batch_status(tucker_batch* b, int* status_out) {
  if (!b || !status_out) return fail(TUCKER_EINVAL, "NULL argument");
  tucker_status st = batch_sync(b);
  if (st) return st;
  std::memcpy(status_out, b->hstatus.data(), sizeof(int) * b->count);
  return TUCKER_OK;
}

tucker_status tucker_batch_tiles(const tucker_batch* b, int* gram_chunks, int* ttm_tiles) {
  if (!b || !gram_chunks || !ttm_tiles) return fail(TUCKER_EINVAL, "NULL argument");
  *gram_chunks = b->tiles.gram_chunks;
  *ttm_tiles = b->tiles.ttm_tiles;
  return TUCKER_OK;
}

tucker_status tucker_batch_item(tucker_batch* b, int i, tucker_t** out) {
  if (!b || !out) return fail(TUCKER_EINVAL, "NULL argument");
  *out = nullptr;
  if (i < 0 || i >= b->count) return fail(TUCKER_EINVAL, "item %d outside 0..%d", i, b->count - 1);
  tucker_status st = batch_sync(b);
  if (st) return st;
  const int N = b->N;
  hipStream_t s = b->run_stream;
  HandleGuard g(new tucker_t);
  tucker_t* t = g.t;
  t->N = N;
  t->stream = s;
  std::memcpy(t->dims, &b->dims[(size_t)i * N], sizeof(int64_t) * N);
  std::memcpy(t->order, b->order, sizeof(int) * N);
  std::memcpy(t->ranks, &b->hR[(size_t)i * N], sizeof(int64_t) * N);
  std::memcpy(t->disc, &b->hdisc[(size_t)i * N], sizeof(double) * N);
  t->norm2 = b->hnorm2[i];
  t->core_dtype = b->wdt;
  for (int k = 0; k < N; ++k) t->prec_used[k] = b->prec;
  int64_t cur[TUCKER_MAX_MODES];
  std::memcpy(cur, t->dims, sizeof(int64_t) * N);
  for (int s2 = 0; s2 < N; ++s2) {
    const int n = b->order[s2];
    const int64_t J = cur[n], R = t->ranks[n], Jm = b->Jmax[s2];
    HIP_TRY(t->alloc((void**)&t->U[n], sizeof(double) * J * J));
    HIP_TRY(t->alloc((void**)&t->lam[n], sizeof(double) * J));
    t->eigcount[n] = J;
    HIP_TRY(hipMemcpyAsync(t->U[n], b->U[n] + (size_t)i * Jm * Jm, sizeof(double) * J * R, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(t->lam[n], b->lam[n] + (size_t)i * Jm, sizeof(double) * J, hipMemcpyDeviceToDevice, s));
    cur[n] = R;
  }
  int64_t ce = 1;
  for (int k = 0; k < N; ++k) ce *= cur[k];
  const size_t ws = wsize(b->wdt);
  HIP_TRY(t->alloc(&t->core, ws * ce));
  HIP_TRY(hipMemcpyAsync(t->core, static_cast<char*>(b->buf[(N - 1) % 2]) + ws * b->off[i], ws * ce,
                         hipMemcpyDeviceToDevice, s));
  HIP_TRY(t->alloc((void**)&t->scalars, sizeof(double) * 2));
  HIP_TRY(hipStreamSynchronize(s));
  *out = g.take();
  return TUCKER_OK;
}

void tucker_batch_free(tucker_batch* b) {
  if (!b) return;
  b->release();
  delete b;
}

}  // extern "C"
