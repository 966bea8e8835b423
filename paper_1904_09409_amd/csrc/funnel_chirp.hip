// funnel_chirp.hip -- the band-limited (chirp-z) NVMT fused with the DFT
// along x', per frequency row, in place.
//
// For row n2 with ratio s = 2 n2 / Np the pass computes
//   G[m1] = s sum_x S[x] exp(-j 2 pi s m1 x / W),   x, m1 in [-W/2, W/2),
// the spectrum of the row resampled at x' = s x by band-limited
// interpolation (the chirp-z realisation of the NVMT the paper adopts at the
// opening of Sec. IV; cost of about two FFTs per row, Remark 1 and Sec. V).
// With m1 x = (m1^2 + x^2 - (m1 - x)^2) / 2 this is Bluestein's convolution:
//   G[m1] = w(m1) sum_x [w(x) S[x]] c(m1 - x) * s,
//   w(k) = exp(-j pi s k^2 / W),  c(k) = exp(+j pi s k^2 / W),
// evaluated as a cyclic convolution of length L = 2W by FFT:
//   G = w . IDFT_L( DFT_L(w . S, zero-padded) . Cz ),  Cz = (s / L) DFT_L(c').
// The tables Cz[n2][0..L) and w[n2][0..W) are built in FP64 on the host at
// plan creation.  A block takes one row n2 for IPB images: it loads the row's
// tables into registers once and runs the images ROWS at a time.
//
// The forward transform (radices largest-first) leaves each thread holding
// outputs t + P b + q L/R_last; the inverse transform with the radix order
// reversed reads exactly those elements as its first-pass inputs, so the
// pointwise product needs no LDS exchange between the two transforms.  Its
// outputs come back on the forward engine's input positions, so the same w
// registers serve the pre- and the post-multiplication.
//
// The adjoint: the operator's matrix s exp(-j 2 pi s m1 x / W) is symmetric,
// so its conjugate transpose is the same pass applied to the conjugated
// input, with the output conjugated.
#include <hip/hip_runtime.h>

#include "fft_core.hpp"
#include "funnel_internal.hpp"

namespace funnel {

// (elements per thread, target threads per block, images per block, PF: load
// the next image's row while the current one is transformed)
#define FUNNEL_CHIRP_VARIANTS(X)                                                                      \
  X(0, 16, 256, 8, 0) X(1, 16, 256, 4, 0) X(2, 16, 256, 16, 0) X(3, 16, 128, 8, 0) X(4, 16, 256, 8, 1) \
  X(5, 16, 128, 8, 1) X(6, 16, 256, 16, 1) X(7, 16, 128, 16, 1)

template <int W, int E_, int TPB, int IPB, int PF>
struct ChirpCfg {
  static constexpr int L = 2 * W;
  static constexpr bool POW2 = (L & (L - 1)) == 0;
  static constexpr int P = POW2 ? (L / E_ > 0 ? L / E_ : 1) : cdiv(L, E_);
  static constexpr int ROWS0 = TPB / P > 0 ? TPB / P : 1;
  static constexpr int ROWS = ROWS0 < IPB ? ROWS0 : IPB;
  static constexpr int THREADS = ROWS * P;
  using Fwd = FftR<L, P, false, false>;
  using Inv = FftR<L, P, true, true>;
  static constexpr int E = Fwd::EM;
  static constexpr int R0 = Fwd::kPlan.r[0];
  static constexpr bool valid = W >= 32 && L <= 4096 && radix_plan(L).n > 0 && P >= 2 && Fwd::EM == Inv::EM &&
                                (POW2 ? L % E_ == 0 : E * 2 <= 3 * E_) && IPB % ROWS == 0 &&
                                THREADS <= 1024 && THREADS >= 32 && LayRow<ROWS, L>::size(L) * 8 + L * 4 <= 80 * 1024;
};

template <int W, int E_, int TPB, int IPB, int PF, bool ADJ>
__global__ void __launch_bounds__((ChirpCfg<W, E_, TPB, IPB, PF>::THREADS))
    k_row_chirp(float2* __restrict__ data, int h, int batch, long long img_stride, const float2* __restrict__ cz,
                const float2* __restrict__ wz, const float2* __restrict__ tw) {
  using Cfg = ChirpCfg<W, E_, TPB, IPB, PF>;
  constexpr int L = Cfg::L, P = Cfg::P, ROWS = Cfg::ROWS;
  using Fwd = typename Cfg::Fwd;
  using Inv = typename Cfg::Inv;
  constexpr int E = Fwd::EM;
  constexpr RadixPlan PL = Fwd::kPlan;
  constexpr int LAST = PL.n - 1;
  constexpr int R0 = PL.r[0], NB0 = L / R0, BPT0 = Fwd::template bpt<0, false>();
  constexpr int RL = PL.r[LAST], NBL = L / RL, BPTL = Fwd::template bpt<LAST, false>();
  constexpr int H0 = R0 / 2;   // inputs j + r NB0 with r < R0/2 are the W row samples, the rest are zero
  static_assert(Inv::kPlan.r[0] == RL && Inv::kPlan.r[LAST] == R0, "inverse engine runs the radices reversed");
  static_assert(Inv::template bpt<LAST, false>() == BPT0, "inverse outputs land on the forward input slots");
  using Lay = LayRow<ROWS, L>;
  __shared__ float2 lds[Lay::size(L)];
  __shared__ float2 twl[L / 2];   // the FFT twiddles: every index a pass reads is below L / R <= L / 2

  const int tid = threadIdx.x;
  const int row = tid / P, t = tid % P;
  const int groups = (batch + IPB - 1) / IPB;
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int n2 = lin / groups + 1;
  const int grp = lin % groups;
  if (n2 > h) return;   // uniform over the block

  // The twiddles come from LDS: read from global memory inside the
  // transforms, each of their waits on the in-order load counter would also
  // wait for the next image's row loads and void the prefetch.  Staged
  // first, so the loads after them stay in flight.
  for (int i = tid; i < L / 2; i += Cfg::THREADS) twl[i] = tw[i];

  // this row's tables, held for all images of the block
  const float2* czr = cz + (long long)(n2 - 1) * L;
  const float2* wzr = wz + (long long)(n2 - 1) * W;
  float2 cr[E], wr[BPT0 * H0];
#pragma unroll
  for (int b = 0; b < BPTL; ++b)
#pragma unroll
    for (int q = 0; q < RL; ++q)
      cr[b * RL + q] = Fwd::template ok<LAST, false>(t, b) ? czr[t + P * b + q * NBL] : make_float2(0.f, 0.f);
#pragma unroll
  for (int b = 0; b < BPT0; ++b)
#pragma unroll
    for (int r = 0; r < H0; ++r)
      wr[b * H0 + r] = Fwd::template ok<0, false>(t, b) ? wzr[t + P * b + r * NB0] : make_float2(0.f, 0.f);

  // the row samples of image `img` that this thread feeds to the first pass
  constexpr int NIN = BPT0 * H0;
  auto load_row = [&](int img, float2 (&xin)[NIN]) {
    const bool act = img < batch;
    const float2* rp = data + (long long)(act ? img : 0) * img_stride + (long long)(n2 - 1) * W;
#pragma unroll
    for (int b = 0; b < BPT0; ++b)
#pragma unroll
      for (int r = 0; r < H0; ++r)
        xin[b * H0 + r] = act && Fwd::template ok<0, false>(t, b) ? rp[t + P * b + r * NB0] : make_float2(0.f, 0.f);
  };
  float2 nxt[NIN];
  if constexpr (PF) load_row(grp * IPB + row, nxt);
  __syncthreads();   // twl

#pragma unroll 1
  for (int it = 0; it < IPB / ROWS; ++it) {
    const int img = grp * IPB + it * ROWS + row;
    const bool active = img < batch;
    float2* rowp = data + (long long)(active ? img : 0) * img_stride + (long long)(n2 - 1) * W;
    float2 cur[NIN];
    if constexpr (PF) {
#pragma unroll
      for (int i = 0; i < NIN; ++i) cur[i] = nxt[i];
      if (it + 1 < IPB / ROWS) load_row(img + ROWS, nxt);   // in flight during the transforms
    } else {
      load_row(img, cur);
    }
    float2 v[E];
#pragma unroll
    for (int s2 = 0; s2 < E; ++s2) v[s2] = make_float2(0.f, 0.f);
#pragma unroll
    for (int b = 0; b < BPT0; ++b)
#pragma unroll
      for (int r = 0; r < H0; ++r) {
        float2 x = cur[b * H0 + r];
        if (ADJ) x.y = -x.y;
        v[b * R0 + r] = c_mul(x, wr[b * H0 + r]);
      }
    Fwd::template run<false, false, false, Lay>(v, row, t, lds, twl);
#pragma unroll
    for (int s2 = 0; s2 < BPTL * RL; ++s2) v[s2] = c_mul(v[s2], cr[s2]);
    Inv::template run<false, false, false, Lay>(v, row, t, lds, twl);
    if (!active) continue;
#pragma unroll
    for (int b = 0; b < BPT0; ++b)
#pragma unroll
      for (int q = 0; q < H0; ++q) {
        if (!Inv::template ok<LAST, false>(t, b)) continue;
        float2 y = c_mul(v[b * R0 + q], wr[b * H0 + q]);
        if (ADJ) y.y = -y.y;
        rowp[t + P * b + q * NB0] = y;
      }
  }
}

template <int W>
unsigned chirp_variant_mask_t() {
  unsigned m = 0;
#define FUNNEL_V(i, e, tpb, ipb, pf) \
  if constexpr (ChirpCfg<W, e, tpb, ipb, pf>::valid) m |= 1u << i;
  FUNNEL_CHIRP_VARIANTS(FUNNEL_V)
#undef FUNNEL_V
  return m;
}

template <int W>
hipError_t launch_chirp_t(int variant, bool adj, float2* data, int h, long long img_stride, const float2* cz,
                          const float2* wz, const float2* tw, int batch, hipStream_t s) {
  switch (variant) {
#define FUNNEL_V(i, e, tpb, ipb, pf)                                                                            \
  case i:                                                                                                       \
    if constexpr (ChirpCfg<W, e, tpb, ipb, pf>::valid) {                                                        \
      using F = ChirpCfg<W, e, tpb, ipb, pf>;                                                                   \
      dim3 grid(h * ((batch + ipb - 1) / ipb)), block(F::THREADS);                                              \
      if (adj)                                                                                                  \
        k_row_chirp<W, e, tpb, ipb, pf, true><<<grid, block, 0, s>>>(data, h, batch, img_stride, cz, wz, tw);  \
      else                                                                                                      \
        k_row_chirp<W, e, tpb, ipb, pf, false><<<grid, block, 0, s>>>(data, h, batch, img_stride, cz, wz, tw); \
      return hipGetLastError();                                                                                  \
    }                                                                                                            \
    break;
    FUNNEL_CHIRP_VARIANTS(FUNNEL_V)
#undef FUNNEL_V
    default: break;
  }
  return hipErrorInvalidValue;
}

#define FUNNEL_CHIRP_LENGTHS(X) X(64) X(128) X(256) X(512) X(1024) X(2048)

unsigned chirp_variant_mask(int W) {
  switch (W) {
#define CASE(n) case n: return chirp_variant_mask_t<n>();
    FUNNEL_CHIRP_LENGTHS(CASE)
#undef CASE
    default: return 0;
  }
}

hipError_t launch_chirp(int W, int variant, bool adj, float2* data, int h, long long img_stride, const float2* cz,
                        const float2* wz, const float2* tw, int batch, hipStream_t s) {
  if (h <= 0 || batch <= 0) return hipSuccess;
  switch (W) {
#define CASE(n) case n: return launch_chirp_t<n>(variant, adj, data, h, img_stride, cz, wz, tw, batch, s);
    FUNNEL_CHIRP_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace funnel
