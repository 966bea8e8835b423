// fft_mfma.hpp -- DFT passes on the matrix cores with split-precision operands.
//
// FftM computes the same Stockham transform as FftR (same pass formula, same
// twiddle table, FP32 twiddle products) but evaluates every R-point DFT as a
// small real matrix product on the MFMA units.  Writing a complex input as
// (re, im) pairs, the R-point DFT of 16 butterflies at once is
//
//     [Y_re; Y_im] = [[C, +-S], [-+S, C]] [X_re; X_im]     (C, S: cos, sin of 2 pi m r / R)
//
// and each operand is split into a high and a low half-precision part,
// X = X_hi + X_lo, A = A_hi + A_lo, keeping A_hi X_hi + A_hi X_lo + A_lo X_hi
// with FP32 accumulation (the dropped A_lo X_lo is below the representation
// error of the split).  BF16 needs no scaling (FP32's exponent range); FP16
// operands are scaled per butterfly by a power of two that puts the largest
// input magnitude in [2^14, 2^15), undone exactly after the product.
//
// Radix 16 uses v_mfma_f32_16x16x32 (K = 32 = 16 complex inputs): lane
// (g, n) of a wave, g = lane / 16, n = lane % 16, holds inputs 4g .. 4g+3 of
// butterfly n of a group of 16 and receives outputs 4g .. 4g+3.  Radix 8 uses
// v_mfma_f32_16x16x16 (K = 16 = 8 complex inputs) with inputs and outputs
// 2g, 2g+1.  The K order is free as long as A and B agree; pairing the real
// and imaginary part of one input in adjacent K slots lets a lane read and
// write whole complex values.
//
// Interface: identical to FftR::run.  The caller's registers hold pass 0's
// inputs in FftR's layout (including the Hermitian pairing of a paired first
// pass) and receive the last pass's outputs in FftR's layout; FftM moves
// them through LDS into its own layout on entry and back on exit.
#pragma once

#include "fft_core.hpp"
#include "funnel_internal.hpp"

namespace funnel {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// Radices 16 then 8 only (the two shapes the matrix cores take): power-of-two
// lengths 64 .. 4096.
constexpr RadixPlan mfma_plan(int L) {
  RadixPlan p{0, {}};
  int a = 0, rem = L;
  while (rem % 2 == 0) { rem /= 2; ++a; }
  if (rem != 1 || a < 6 || a > 12) return p;
  const int y = (3 * a) % 4;  // radix-8 passes: 3y = a (mod 4)
  const int x = (a - 3 * y) / 4;
  for (int i = 0; i < x; ++i) p.r[p.n++] = 16;
  for (int i = 0; i < y; ++i) p.r[p.n++] = 8;
  return p;
}

template <int PREC>
struct Half;

template <>
struct Half<kPrecBF16x3> {
  using T = __bf16;
  using V8 = bf16x8;
  using V4 = bf16x4;
  static constexpr bool kScaled = false;
  __device__ static __forceinline__ f32x4 mma16(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ f32x4 mma8(V4 a, V4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(i16x4, a), __builtin_bit_cast(i16x4, b), c,
                                                     0, 0, 0);
  }
};

template <>
struct Half<kPrecFP16x3> {
  using T = _Float16;
  using V8 = f16x8;
  using V4 = f16x4;
  static constexpr bool kScaled = true;
  __device__ static __forceinline__ f32x4 mma16(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ f32x4 mma8(V4 a, V4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};

// x = hi + lo, each rounded to nearest
template <class T>
__device__ __forceinline__ void split2(float x, T& hi, T& lo) {
  hi = (T)x;
  lo = (T)(x - (float)hi);
}

// Power of two s with m s in [2^14, 2^15) (clamped to normal floats), and 1/s.
__device__ __forceinline__ void fp16_scale(float m, float& s, float& inv) {
  const int e = (int)((__float_as_uint(m) >> 23) & 0xff);
  int b = 268 - e;
  b = b < 1 ? 1 : (b > 253 ? 253 : b);
  s = __uint_as_float((uint32_t)b << 23);
  inv = __uint_as_float((uint32_t)(254 - b) << 23);
}

// coefficient of input part pk (0 re, 1 im) in output part pm of the R-point
// DFT, for the angle index mr = m r mod R (tables of 16)
template <int R, bool INV>
__device__ __forceinline__ float dft_coef(int mr, int pm, int pk) {
  const int k16 = (mr * (16 / R)) & 15;
  const float c = kCos16[k16], s = kSin16[k16];
  // forward e^{-i t}: re += xr c + xi s, im += xi c - xr s; inverse flips s
  const float ss = INV ? -s : s;
  if (pm == pk) return c;
  return pm == 0 ? ss : -ss;
}

template <int L, int P, bool INV, bool REV, int PREC, int NLINES, bool LINE_FASTEST>
struct FftM {
  using Outer = FftR<L, P, INV, REV>;
  using H = Half<PREC>;
  using T = typename H::T;
  static constexpr RadixPlan kPlan = Outer::kPlan;  // the caller-facing layout
  static constexpr RadixPlan kM = mfma_plan(L);
  static constexpr int E = L / P;
  static constexpr int EM = E;
  static constexpr int THREADS = NLINES * P;
  static_assert(kM.n > 0, "matrix-core passes need a power-of-two length in 64 .. 4096");
  // caller-facing butterfly counts and guards: FftR's (exact for powers of two)
  template <int I, bool PAIRED>
  static constexpr int bpt() { return Outer::template bpt<I, PAIRED>(); }
  template <int I, bool PAIRED>
  __device__ static __forceinline__ bool ok(int t, int b) { return Outer::template ok<I, PAIRED>(t, b); }
  static_assert(THREADS % 64 == 0, "whole waves");
  static_assert(E % 4 == 0, "four elements per lane and group");

  template <int I>
  static constexpr int ns() {
    int p = 1;
    for (int i = 0; i < I; ++i) p *= kM.r[i];
    return p;
  }
  // elements of one butterfly a lane holds, and groups of 16 butterflies per lane
  template <int I>
  static constexpr int per() { return kM.r[I] / 4; }
  template <int I>
  static constexpr int groups() { return E / per<I>(); }

  // butterfly id of group c for this lane -> (line, j)
  template <int I>
  __device__ static __forceinline__ void which(int c, int& line, int& j) {
    constexpr int NB = L / kM.r[I];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int B = (w * groups<I>() + c) * 16 + (lane & 15);
    if constexpr (LINE_FASTEST) {
      line = B % NLINES;
      j = B / NLINES;
    } else {
      line = B / NB;
      j = B % NB;
    }
  }

  template <bool SPLIT, class Lay, class Buf, class WR, class RD>
  __device__ static __forceinline__ void xchg(float2 (&v)[E], Buf* lds, WR wr, RD rd) {
    if constexpr (!SPLIT) {
      __syncthreads();
#pragma unroll
      for (int s = 0; s < E; ++s) {
        int ln, idx;
        wr(s, ln, idx);
        lds[Lay::addr(ln, idx)] = v[s];
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < E; ++s) {
        int ln, idx;
        rd(s, ln, idx);
        v[s] = lds[Lay::addr(ln, idx)];
      }
    } else {
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        __syncthreads();
#pragma unroll
        for (int s = 0; s < E; ++s) {
          int ln, idx;
          wr(s, ln, idx);
          lds[Lay::addr(ln, idx)] = part ? v[s].y : v[s].x;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < E; ++s) {
          int ln, idx;
          rd(s, ln, idx);
          const float f = lds[Lay::addr(ln, idx)];
          if (part) v[s].y = f;
          else v[s].x = f;
        }
      }
    }
  }

  // inputs of pass I: slot s holds input r = (lane/16) per + s % per of butterfly (group s / per)
  template <int I>
  __device__ static __forceinline__ void in_pos(int s, int& ln, int& idx) {
    constexpr int PER = per<I>(), NB = L / kM.r[I];
    int j;
    which<I>(s / PER, ln, j);
    const int r = (int)(threadIdx.x & 63) / 16 * PER + s % PER;
    idx = j + r * NB;
  }
  template <int I>
  __device__ static __forceinline__ void out_pos(int s, int& ln, int& idx) {
    constexpr int PER = per<I>(), NS = ns<I>(), R = kM.r[I];
    int j;
    which<I>(s / PER, ln, j);
    const int q = (int)(threadIdx.x & 63) / 16 * PER + s % PER;
    idx = (j / NS) * NS * R + (j % NS) + q * NS;
  }

  // A operands of the radix-16 product (rows: outputs; lane holds row n,
  // K slots 8g .. 8g+7) and of the radix-8 product (rows 4g'+2i'+p', lane
  // holds row n, K slots 4g .. 4g+3)
  struct Coef {
    typename H::V8 re_hi, re_lo, im_hi, im_lo;
    typename H::V4 r8_hi, r8_lo;
  };
  __device__ static __forceinline__ void coefs(Coef& A) {
    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = 4 * g + (k >> 1), pk = k & 1;
      T h, l;
      split2(dft_coef<16, INV>(n * r, 0, pk), h, l);
      A.re_hi[k] = h;
      A.re_lo[k] = l;
      split2(dft_coef<16, INV>(n * r, 1, pk), h, l);
      A.im_hi[k] = h;
      A.im_lo[k] = l;
    }
    const int q = 2 * (n >> 2) + ((n >> 1) & 1), pm = n & 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = 2 * g + (k >> 1), pk = k & 1;
      T h, l;
      split2(dft_coef<8, INV>(q * r, pm, pk), h, l);
      A.r8_hi[k] = h;
      A.r8_lo[k] = l;
    }
  }

  template <int I>
  __device__ static __forceinline__ void compute(float2 (&v)[E], const Coef& A, const float2* __restrict__ tw) {
    constexpr int R = kM.r[I], NS = ns<I>(), PER = per<I>();
    const int g = (int)(threadIdx.x & 63) >> 4;
#pragma unroll
    for (int c = 0; c < groups<I>(); ++c) {
      float2* x = v + c * PER;
      if constexpr (NS > 1) {
        int ln, j;
        which<I>(c, ln, j);
        const int st = (j % NS) * (L / (NS * R));
#pragma unroll
        for (int i = 0; i < PER; ++i) {
          float2 w = tw[(g * PER + i) * st];   // each power from the table
          if (INV) w.y = -w.y;
          x[i] = c_mul(x[i], w);
        }
      }
      float sc = 1.f, inv = 1.f;
      if constexpr (H::kScaled) {
        float m = 0.f;
#pragma unroll
        for (int i = 0; i < PER; ++i) m = fmaxf(m, fmaxf(fabsf(x[i].x), fabsf(x[i].y)));
        m = fmaxf(m, __shfl_xor(m, 16));
        m = fmaxf(m, __shfl_xor(m, 32));
        fp16_scale(m, sc, inv);
      }
      if constexpr (R == 16) {
        typename H::V8 bh, bl;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          T h, l;
          split2(x[i].x * sc, h, l);
          bh[2 * i] = h;
          bl[2 * i] = l;
          split2(x[i].y * sc, h, l);
          bh[2 * i + 1] = h;
          bl[2 * i + 1] = l;
        }
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
        f32x4 yr = H::mma16(A.re_lo, bh, z);
        yr = H::mma16(A.re_hi, bl, yr);
        yr = H::mma16(A.re_hi, bh, yr);
        f32x4 yi = H::mma16(A.im_lo, bh, z);
        yi = H::mma16(A.im_hi, bl, yi);
        yi = H::mma16(A.im_hi, bh, yi);
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = make_float2(yr[i] * inv, yi[i] * inv);
      } else {
        static_assert(R == 8, "radix 16 or 8");
        typename H::V4 bh, bl;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          T h, l;
          split2(x[i].x * sc, h, l);
          bh[2 * i] = h;
          bl[2 * i] = l;
          split2(x[i].y * sc, h, l);
          bh[2 * i + 1] = h;
          bl[2 * i + 1] = l;
        }
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
        f32x4 y = H::mma8(A.r8_lo, bh, z);
        y = H::mma8(A.r8_hi, bl, y);
        y = H::mma8(A.r8_hi, bh, y);
        x[0] = make_float2(y[0] * inv, y[1] * inv);
        x[1] = make_float2(y[2] * inv, y[3] * inv);
      }
    }
  }

  template <int I, bool SPLIT, class Lay, class Buf>
  __device__ static __forceinline__ void passes(float2 (&v)[E], Buf* lds, const Coef& A,
                                                const float2* __restrict__ tw) {
    compute<I>(v, A, tw);
    if constexpr (I + 1 < kM.n) {
      xchg<SPLIT, Lay>(
          v, lds, [](int s, int& ln, int& idx) { out_pos<I>(s, ln, idx); },
          [](int s, int& ln, int& idx) { in_pos<I + 1>(s, ln, idx); });
      passes<I + 1, SPLIT, Lay>(v, lds, A, tw);
    }
  }

  // (FftR's calling convention; the split-precision kernels always run with
  // every thread of the block in a transform, so `live` is always true here)
  template <bool PAIRED_FIRST, bool PAIRED_LAST, bool SPLIT, class Lay, class Buf>
  __device__ static __forceinline__ void run(float2 (&v)[E], int line, int t, Buf* lds,
                                             const float2* __restrict__ tw, bool /*live*/ = true) {
    constexpr int R0 = kPlan.r[0], NB0 = L / R0;
    constexpr int LAST = kPlan.n - 1, RL = kPlan.r[LAST], NBL = L / RL;
    Coef A;
    coefs(A);
    xchg<SPLIT, Lay>(
        v, lds,
        [&](int s, int& ln, int& idx) {
          ln = line;
          idx = Outer::template bfly<0, PAIRED_FIRST>(t, s / R0) + (s % R0) * NB0;
        },
        [](int s, int& ln, int& idx) { in_pos<0>(s, ln, idx); });
    passes<0, SPLIT, Lay>(v, lds, A, tw);
    xchg<SPLIT, Lay>(
        v, lds, [](int s, int& ln, int& idx) { out_pos<kM.n - 1>(s, ln, idx); },
        [&](int s, int& ln, int& idx) {
          ln = line;
          idx = Outer::template bfly<LAST, PAIRED_LAST>(t, s / RL) + (s % RL) * NBL;
        });
  }
};

// The engine a kernel of precision PREC uses: FftR for FP32, FftM otherwise.
template <int PREC, int L, int P, bool INV, bool REV, int NLINES, bool LINE_FASTEST>
struct EngSel {
  using type = FftM<L, P, INV, REV, PREC, NLINES, LINE_FASTEST>;
};
template <int L, int P, bool INV, bool REV, int NLINES, bool LINE_FASTEST>
struct EngSel<kPrecFP32, L, P, INV, REV, NLINES, LINE_FASTEST> {
  using type = FftR<L, P, INV, REV>;
};

// whether FftM can run a transform of length L with E elements per thread in
// a block of THREADS threads
constexpr bool mfma_fits(int L, int E, int THREADS) {
  return mfma_plan(L).n > 0 && THREADS % 64 == 0 && E % 4 == 0;
}

}  // namespace funnel
