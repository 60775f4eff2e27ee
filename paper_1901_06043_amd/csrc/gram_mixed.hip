// Mixed-precision Gram (FP32 inputs): placeholder until the FP32/BF16x3 MFMA
// kernels are in place; reports "not supported".
#include "common.hpp"
#include "kernels.hpp"

namespace tk {

GramPlan plan_gram_mixed(int J, uint64_t L, uint64_t K) {
  GramPlan p = plan_gram_f64(J, L, K);
  return p;
}

hipError_t launch_gram_mixed(const float*, int, uint64_t, uint64_t, int, const GramPlan&, double*, double*, double*,
                             double*, hipStream_t, hipEvent_t) {
  return hipErrorNotSupported;
}

}  // namespace tk
