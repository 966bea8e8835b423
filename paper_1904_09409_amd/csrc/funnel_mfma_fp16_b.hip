// Instantiates the split-precision (fp16 hi + lo) pass kernels for one group of
// power-of-two lengths.
#include "funnel_passes.hpp"

namespace funnel {
#define INST(n)                                                                                              \
  template unsigned col_variant_mask_t<n, kPrecFP16x3>();                                                            \
  template unsigned row_variant_mask_t<n, kPrecFP16x3>();                                                            \
  template hipError_t launch_r2c_t<n, kPrecFP16x3>(int, bool, const float*, float2*, int, int, int, ImgMap, float,   \
                                                const float2*, int, hipStream_t);                            \
  template hipError_t launch_c2r_t<n, kPrecFP16x3>(int, bool, bool, const float2*, float*, int, int, int, ImgMap,    \
                                                float, const float2*, int, hipStream_t);                     \
  template hipError_t launch_row_t<n, kPrecFP16x3>(int, bool, float2*, int, int, int, long long, const float2*, int,      \
                                                hipStream_t);
INST(2048) INST(4096)
#undef INST
}  // namespace funnel
