// Instantiates the pass kernels for one group of transform lengths.
#include "funnel_lengths.hpp"
#include "funnel_passes.hpp"

namespace funnel {
#define INST(n)                                                                                              \
  template unsigned col_variant_mask_t<n, kPrecFP32>();                                                                 \
  template unsigned row_variant_mask_t<n, kPrecFP32>();                                                                 \
  template hipError_t launch_r2c_t<n, kPrecFP32>(int, bool, const float*, float2*, int, int, int, ImgMap, float,       \
                                      const float2*, int, hipStream_t);                               \
  template hipError_t launch_c2r_t<n, kPrecFP32>(int, bool, bool, const float2*, float*, int, int, int, ImgMap, float,  \
                                      const float2*, int, hipStream_t);                    \
  template hipError_t launch_row_t<n, kPrecFP32>(int, bool, float2*, int, int, int, long long, const float2*, int, hipStream_t);
FUNNEL_LENGTHS_G0(INST)
#undef INST
}  // namespace funnel
