// funnel_kernels.hip -- length and precision dispatch of the pass launchers
// (the kernels themselves are in funnel_passes.hpp, instantiated by
// funnel_len_g*.hip for FP32 and funnel_mfma_*.hip for the split precisions).
#include <hip/hip_runtime.h>

#include "funnel_internal.hpp"
#include "funnel_lengths.hpp"

namespace funnel {

template <int L, int PREC>
unsigned col_variant_mask_t();
template <int M, int PREC>
unsigned row_variant_mask_t();
template <int L, int PREC>
hipError_t launch_r2c_t(int variant, bool trans, const float* in, float2* out, int nlines, int lin, int off,
                        ImgMap map, float scale, const float2* tw, int batch, hipStream_t s);
template <int L, int PREC>
hipError_t launch_c2r_t(int variant, bool trans, bool accum, const float2* in, float* out, int nlines, int r0,
                        int nout, ImgMap map, float scale, const float2* tw, int batch, hipStream_t s);
template <int M, int PREC>
hipError_t launch_row_t(int variant, bool adj, float2* data, int Lp, int h, int rpf, long long img_stride,
                        const float2* tw, int batch, hipStream_t s);

// lengths with split-precision kernels
#define FUNNEL_MFMA_LENGTHS(X) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

bool length_supported(int L) {
  switch (L) {
#define CASE(n) case n: return true;
    FUNNEL_LENGTHS(CASE)
#undef CASE
    default: return false;
  }
}

unsigned col_variant_mask(int L, int prec) {
  if (prec == kPrecFP32) {
    switch (L) {
#define CASE(n) case n: return col_variant_mask_t<n, kPrecFP32>();
      FUNNEL_LENGTHS(CASE)
#undef CASE
      default: return 0;
    }
  }
  switch (L) {
#define CASE(n) \
  case n: return prec == kPrecBF16x3 ? col_variant_mask_t<n, kPrecBF16x3>() : col_variant_mask_t<n, kPrecFP16x3>();
    FUNNEL_MFMA_LENGTHS(CASE)
#undef CASE
    default: return 0;
  }
}

unsigned row_variant_mask(int M, int prec) {
  if (prec == kPrecFP32) {
    switch (M) {
#define CASE(n) case n: return row_variant_mask_t<n, kPrecFP32>();
      FUNNEL_LENGTHS(CASE)
#undef CASE
      default: return 0;
    }
  }
  switch (M) {
#define CASE(n) \
  case n: return prec == kPrecBF16x3 ? row_variant_mask_t<n, kPrecBF16x3>() : row_variant_mask_t<n, kPrecFP16x3>();
    FUNNEL_MFMA_LENGTHS(CASE)
#undef CASE
    default: return 0;
  }
}

hipError_t launch_r2c(int L, int variant, int prec, bool trans, const float* in, float2* out, int nlines, int lin,
                      int off, ImgMap map, float scale, const float2* tw, int batch, hipStream_t s) {
  if (prec == kPrecFP32) {
    switch (L) {
#define CASE(n) \
  case n: return launch_r2c_t<n, kPrecFP32>(variant, trans, in, out, nlines, lin, off, map, scale, tw, batch, s);
      FUNNEL_LENGTHS(CASE)
#undef CASE
      default: return hipErrorInvalidValue;
    }
  }
  switch (L) {
#define CASE(n)                                                                                                   \
  case n:                                                                                                         \
    return prec == kPrecBF16x3                                                                                    \
               ? launch_r2c_t<n, kPrecBF16x3>(variant, trans, in, out, nlines, lin, off, map, scale, tw, batch, s) \
               : launch_r2c_t<n, kPrecFP16x3>(variant, trans, in, out, nlines, lin, off, map, scale, tw, batch, s);
    FUNNEL_MFMA_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_c2r(int L, int variant, int prec, bool trans, bool accum, const float2* in, float* out, int nlines,
                      int r0, int nout, ImgMap map, float scale, const float2* tw, int batch, hipStream_t s) {
  if (prec == kPrecFP32) {
    switch (L) {
#define CASE(n)                                                                                                   \
  case n:                                                                                                         \
    return launch_c2r_t<n, kPrecFP32>(variant, trans, accum, in, out, nlines, r0, nout, map, scale, tw, batch, s);
      FUNNEL_LENGTHS(CASE)
#undef CASE
      default: return hipErrorInvalidValue;
    }
  }
  switch (L) {
#define CASE(n)                                                                                                      \
  case n:                                                                                                            \
    return prec == kPrecBF16x3 ? launch_c2r_t<n, kPrecBF16x3>(variant, trans, accum, in, out, nlines, r0, nout, map, \
                                                               scale, tw, batch, s)                                  \
                               : launch_c2r_t<n, kPrecFP16x3>(variant, trans, accum, in, out, nlines, r0, nout, map, \
                                                               scale, tw, batch, s);
    FUNNEL_MFMA_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row(int M, int variant, int prec, bool adj, float2* data, int Lp, int h, int rpf, long long img_stride,
                      const float2* tw, int batch, hipStream_t s) {
  if (prec == kPrecFP32) {
    switch (M) {
#define CASE(n) case n: return launch_row_t<n, kPrecFP32>(variant, adj, data, Lp, h, rpf, img_stride, tw, batch, s);
      FUNNEL_LENGTHS(CASE)
#undef CASE
      default: return hipErrorInvalidValue;
    }
  }
  switch (M) {
#define CASE(n)                                                                                        \
  case n:                                                                                              \
    return prec == kPrecBF16x3                                                                         \
               ? launch_row_t<n, kPrecBF16x3>(variant, adj, data, Lp, h, rpf, img_stride, tw, batch, s)     \
               : launch_row_t<n, kPrecFP16x3>(variant, adj, data, Lp, h, rpf, img_stride, tw, batch, s);
    FUNNEL_MFMA_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace funnel
