// funnel_kernels.hip -- length dispatch of the pass launchers (the kernels
// themselves are in funnel_passes.hpp, instantiated by funnel_len_g*.hip).
#include <hip/hip_runtime.h>

#include "funnel_internal.hpp"
#include "funnel_lengths.hpp"

namespace funnel {

template <int L>
unsigned col_variant_mask_t();
template <int M>
unsigned row_variant_mask_t();
template <int L>
hipError_t launch_r2c_t(int variant, bool trans, const float* in, float2* out, int nlines, int lin, int off,
                        ImgMap map, float scale, const float2* tw, int batch, hipStream_t s);
template <int L>
hipError_t launch_c2r_t(int variant, bool trans, bool accum, const float2* in, float* out, int nlines, int r0,
                        int nout, ImgMap map, float scale, const float2* tw, int batch, hipStream_t s);
template <int M>
hipError_t launch_row_t(int variant, bool adj, float2* data, int Lp, int h, long long img_stride,
                        const float2* tw, int batch, hipStream_t s);

bool length_supported(int L) {
  switch (L) {
#define CASE(n) case n: return true;
    FUNNEL_LENGTHS(CASE)
#undef CASE
    default: return false;
  }
}

unsigned col_variant_mask(int L) {
  switch (L) {
#define CASE(n) case n: return col_variant_mask_t<n>();
    FUNNEL_LENGTHS(CASE)
#undef CASE
    default: return 0;
  }
}

unsigned row_variant_mask(int M) {
  switch (M) {
#define CASE(n) case n: return row_variant_mask_t<n>();
    FUNNEL_LENGTHS(CASE)
#undef CASE
    default: return 0;
  }
}

hipError_t launch_r2c(int L, int variant, bool trans, const float* in, float2* out, int nlines, int lin, int off,
                      ImgMap map, float scale, const float2* tw, int batch, hipStream_t s) {
  switch (L) {
#define CASE(n) \
  case n: return launch_r2c_t<n>(variant, trans, in, out, nlines, lin, off, map, scale, tw, batch, s);
    FUNNEL_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_c2r(int L, int variant, bool trans, bool accum, const float2* in, float* out, int nlines, int r0,
                      int nout, ImgMap map, float scale, const float2* tw, int batch, hipStream_t s) {
  switch (L) {
#define CASE(n)                                                                                         \
  case n:                                                                                               \
    return launch_c2r_t<n>(variant, trans, accum, in, out, nlines, r0, nout, map, scale, tw, batch, s);
    FUNNEL_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row(int M, int variant, bool adj, float2* data, int Lp, int h, long long img_stride, const float2* tw,
                      int batch, hipStream_t s) {
  switch (M) {
#define CASE(n) case n: return launch_row_t<n>(variant, adj, data, Lp, h, img_stride, tw, batch, s);
    FUNNEL_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace funnel
