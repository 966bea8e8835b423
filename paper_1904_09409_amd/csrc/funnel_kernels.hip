// funnel_kernels.hip -- length dispatch of the pass launchers (the kernels
// themselves are in funnel_passes.hpp, instantiated by funnel_len_g*.hip).
#include <hip/hip_runtime.h>

#include "funnel_internal.hpp"
#include "funnel_lengths.hpp"

namespace funnel {

template <int L>
hipError_t launch_r2c_t(bool trans, const float* in, float2* out, int nlines, int lin, int off, long long in_img,
                        long long out_img, float scale, const float2* tw, int batch, hipStream_t s);
template <int L>
hipError_t launch_c2r_t(bool trans, bool accum, const float2* in, float* out, int nlines, int r0, int nout,
                        long long in_img, long long out_img, float scale, const float2* tw, int batch, hipStream_t s);
template <int M>
hipError_t launch_row_t(bool adj, float2* data, int Lp, int h, long long img_stride, const float2* tw, int batch,
                        hipStream_t s);

bool length_supported(int L) {
  switch (L) {
#define CASE(n) case n: return true;
    FUNNEL_LENGTHS(CASE)
#undef CASE
    default: return false;
  }
}

hipError_t launch_r2c(int L, bool trans, const float* in, float2* out, int nlines, int lin, int off,
                      long long in_img, long long out_img, float scale, const float2* tw, int batch,
                      hipStream_t s) {
  switch (L) {
#define CASE(n) \
  case n: return launch_r2c_t<n>(trans, in, out, nlines, lin, off, in_img, out_img, scale, tw, batch, s);
    FUNNEL_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_c2r(int L, bool trans, bool accum, const float2* in, float* out, int nlines, int r0, int nout,
                      long long in_img, long long out_img, float scale, const float2* tw, int batch,
                      hipStream_t s) {
  switch (L) {
#define CASE(n)                                                                                         \
  case n:                                                                                               \
    return launch_c2r_t<n>(trans, accum, in, out, nlines, r0, nout, in_img, out_img, scale, tw, batch, s);
    FUNNEL_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row(int M, bool adj, float2* data, int Lp, int h, long long img_stride, const float2* tw,
                      int batch, hipStream_t s) {
  switch (M) {
#define CASE(n) case n: return launch_row_t<n>(adj, data, Lp, h, img_stride, tw, batch, s);
    FUNNEL_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace funnel
