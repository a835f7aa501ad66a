// The factored FP32-comp dS kernel of the (5, 4) family (3He), built with the
// instruction scheduler that favours instruction-level parallelism; the
// kernel code itself is in ds_kernel.hpp.
#include "ds_kernel.hpp"

namespace mbc {

hipError_t launch_ds_5_4_factored_f32(const mbc_plan* p, const BwdArgs& a, int nb, size_t lds, hipStream_t st) {
  return launch_ds_one<float, 5, 4, 512, 10, true>(p, a, nb, lds, st);
}

}  // namespace mbc
