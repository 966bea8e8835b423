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
// Interface: run() is FftR::run's.  The caller's registers hold pass 0's
// inputs in FftR's layout (including the Hermitian pairing of a paired first
// pass) and receive the last pass's outputs in FftR's layout; FftM moves
// them through LDS into its own layout on entry and back on exit.  run_ex()
// skips either move for callers that load the inputs, or store the outputs,
// in FftM's own layout (native_in / native_out give each slot's element).
#pragma once

#include <type_traits>

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

// Lane twiddle tables of the matrix-core passes, stored after the length-L
// table w^m = exp(-+i 2 pi m / L): for each pass I >= 1 (NS = the product of
// the earlier radices, R = its radix, PER = R / 4 inputs per lane), entry
// (m 4 + g) PER + i holds w^((g PER + i) m L / (NS R)) for m < NS, g < 4,
// i < PER -- the same table values, ordered so that the lane holding inputs
// g PER .. g PER + PER-1 of a butterfly with m = j mod NS reads its PER
// twiddles as consecutive 16-byte loads.  mfma_lane_twiddles(L) entries in
// all, pass I's from entry mfma_lane_twiddle_offset(L, I).
constexpr int mfma_lane_twiddle_offset(int L, int I) {
  const RadixPlan p = mfma_plan(L);
  int off = 0, ns = 1;
  for (int i = 0; i < I && i < p.n; ++i) {
    if (i >= 1) off += ns * p.r[i];
    ns *= p.r[i];
  }
  return off;
}
constexpr int mfma_lane_twiddles(int L) { return mfma_plan(L).n > 0 ? mfma_lane_twiddle_offset(L, mfma_plan(L).n) : 0; }

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

// split2 of a complex value (a, b), the parts packed as (a, b) pairs.  BF16:
// one packed conversion for the two high parts, whose FP32 values are the
// packed bits shifted into place (exact), and one for the two low parts --
// the same values as split2, in a third of the instructions.  FP16: packed
// conversions for the high and the low parts (both round to nearest, as
// split2's), the high parts widened back one by one.
template <class T>
__device__ __forceinline__ void split2_pair(float a, float b, T& ha, T& hb, T& la, T& lb) {
  if constexpr (std::is_same<T, _Float16>::value) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef _Float16 h2v __attribute__((ext_vector_type(2)));
    const h2v h = __builtin_convertvector((f2v){a, b}, h2v);
    const h2v l = __builtin_convertvector((f2v){a - (float)h[0], b - (float)h[1]}, h2v);
    ha = h[0];
    hb = h[1];
    la = l[0];
    lb = l[1];
  } else if constexpr (std::is_same<T, __bf16>::value) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef __bf16 b2v __attribute__((ext_vector_type(2)));
    const b2v h = __builtin_convertvector((f2v){a, b}, b2v);
    const uint32_t u = __builtin_bit_cast(uint32_t, h);
    const b2v l = __builtin_convertvector((f2v){a - __uint_as_float(u << 16), b - __uint_as_float(u & 0xffff0000u)}, b2v);
    ha = h[0];
    hb = h[1];
    la = l[0];
    lb = l[1];
  } else {
    split2(a, ha, la);
    split2(b, hb, lb);
  }
}

// Maximum of m over the four 16-lane rows of the wave (lanes n, n+16, n+32,
// n+48): each lane swap exchanges rows between two copies of the value, so
// the larger of the two results is the maximum over the swapped pair, with
// no trip through the LDS crossbar.
__device__ __forceinline__ float max_over_rows(float m) {
  const unsigned u = __float_as_uint(m);
  const auto p = __builtin_amdgcn_permlane16_swap(u, u, false, false);   // rows 0<->1, 2<->3
  m = fmaxf(__uint_as_float(p[0]), __uint_as_float(p[1]));
  const unsigned v = __float_as_uint(m);
  const auto q = __builtin_amdgcn_permlane32_swap(v, v, false, false);   // halves 0-31 <-> 32-63
  return fmaxf(__uint_as_float(q[0]), __uint_as_float(q[1]));
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

  // The thread index, passed through an empty asm after each barrier, so
  // that slot addresses are computed where they are used and not hoisted to
  // the kernel's start and kept live across the passes.
  __device__ static __forceinline__ int opaque() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t & 1023;   // (blocks hold at most 1024 threads: known range for the index algebra)
  }

  // butterfly id of group c for thread tid -> (line, j).  Unsigned
  // arithmetic: the divisions by powers of two are plain shifts; constexpr,
  // so that the layout checks below can evaluate it.
  template <int I>
  static constexpr void which(int tid, int c, int& line, int& j) {
    constexpr unsigned NB = L / kM.r[I];
    const unsigned ut = (unsigned)tid;
    const unsigned B = ((ut >> 6) * (unsigned)groups<I>() + (unsigned)c) * 16u + (ut & 15u);
    if constexpr (LINE_FASTEST) {
      line = (int)(B % (unsigned)NLINES);
      j = (int)(B / (unsigned)NLINES);
    } else {
      line = (int)(B / NB);
      j = (int)(B % NB);
    }
  }

  // inputs of pass I: slot s holds input r = (lane/16) per + s % per of butterfly (group s / per)
  template <int I>
  static constexpr void in_pos(int tid, int s, int& ln, int& idx) {
    constexpr unsigned PER = per<I>(), NB = L / kM.r[I];
    int j = 0;
    which<I>(tid, s / PER, ln, j);
    const unsigned r = (((unsigned)tid & 63u) >> 4) * PER + (unsigned)s % PER;
    idx = (int)((unsigned)j + r * NB);
  }
  template <int I>
  static constexpr void out_pos(int tid, int s, int& ln, int& idx) {
    constexpr unsigned PER = per<I>(), NS = ns<I>(), R = kM.r[I];
    int j = 0;
    which<I>(tid, s / PER, ln, j);
    const unsigned uj = (unsigned)j;
    const unsigned q = (((unsigned)tid & 63u) >> 4) * PER + (unsigned)s % PER;
    idx = (int)((uj / NS) * NS * R + (uj % NS) + q * NS);
  }

  // LDS slot of element s on one side of an exchange: the outputs of pass I
  // (OUT) or its inputs.  Where, for every thread of the block, slot s lies
  // a fixed distance K(s) from the thread's slot 0 (checked exhaustively at
  // compile time), an exchange computes one address per thread and reaches
  // the rest by immediate offsets instead of per-slot index arithmetic.
  template <int I, bool OUT, class Lay>
  static constexpr int pos_addr(int tid, int s) {
    int ln = 0, idx = 0;
    if constexpr (OUT) out_pos<I>(tid, s, ln, idx);
    else in_pos<I>(tid, s, ln, idx);
    return Lay::caddr(ln, idx);
  }
  struct Offs {
    int k[E];
  };
  template <int I, bool OUT, class Lay>
  static constexpr Offs offsets() {
    Offs o{};
    for (int s = 0; s < E; ++s) o.k[s] = pos_addr<I, OUT, Lay>(0, s) - pos_addr<I, OUT, Lay>(0, 0);
    return o;
  }
  template <int I, bool OUT, class Lay>
  static constexpr bool lin_pos() {
    constexpr Offs K = offsets<I, OUT, Lay>();
    for (int tid = 0; tid < THREADS; ++tid) {
      const int a0 = pos_addr<I, OUT, Lay>(tid, 0);
      for (int s = 1; s < E; ++s)
        if (pos_addr<I, OUT, Lay>(tid, s) - a0 != K.k[s]) return false;
    }
    return true;
  }

  // element index (not LDS slot) of slot s relative to slot 0, the same for
  // every thread, and slot s in the thread's slot-0 transform: then callers
  // that load or store in the native layout address slot s as their slot-0
  // element plus a constant
  template <int I, bool OUT>
  static constexpr void pos_idx(int tid, int s, int& ln, int& idx) {
    if constexpr (OUT) out_pos<I>(tid, s, ln, idx);
    else in_pos<I>(tid, s, ln, idx);
  }
  template <int I, bool OUT>
  static constexpr Offs idx_offsets() {
    Offs o{};
    int l0 = 0, i0 = 0;
    pos_idx<I, OUT>(0, 0, l0, i0);
    for (int s = 0; s < E; ++s) {
      int l = 0, i = 0;
      pos_idx<I, OUT>(0, s, l, i);
      o.k[s] = i - i0;
    }
    return o;
  }
  template <int I, bool OUT>
  static constexpr bool lin_idx() {
    constexpr Offs K = idx_offsets<I, OUT>();
    for (int tid = 0; tid < THREADS; ++tid) {
      int l0 = 0, i0 = 0;
      pos_idx<I, OUT>(tid, 0, l0, i0);
      for (int s = 1; s < E; ++s) {
        int l = 0, i = 0;
        pos_idx<I, OUT>(tid, s, l, i);
        if (l != l0 || i - i0 != K.k[s]) return false;
      }
    }
    return true;
  }

  // store v to (load v from) the LDS slots of pass I's outputs (OUT) or
  // inputs; part: the real (0) or imaginary (1) halves of a SPLIT exchange
  template <int I, bool OUT, bool SPLIT, class Lay, class Buf>
  __device__ static __forceinline__ void lds_put(const float2 (&v)[E], Buf* lds, int tid, int part) {
    constexpr bool LIN = lin_pos<I, OUT, Lay>();
    constexpr Offs K = offsets<I, OUT, Lay>();
    Buf* base = lds + pos_addr<I, OUT, Lay>(tid, 0);
#pragma unroll
    for (int s = 0; s < E; ++s) {
      Buf* a = LIN ? base + K.k[s] : lds + pos_addr<I, OUT, Lay>(tid, s);
      if constexpr (SPLIT) *a = part ? v[s].y : v[s].x;
      else *a = v[s];
    }
  }
  template <int I, bool OUT, bool SPLIT, class Lay, class Buf>
  __device__ static __forceinline__ void lds_get(float2 (&v)[E], const Buf* lds, int tid, int part) {
    constexpr bool LIN = lin_pos<I, OUT, Lay>();
    constexpr Offs K = offsets<I, OUT, Lay>();
    const Buf* base = lds + pos_addr<I, OUT, Lay>(tid, 0);
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const Buf* a = LIN ? base + K.k[s] : lds + pos_addr<I, OUT, Lay>(tid, s);
      if constexpr (SPLIT) {
        if (part) v[s].y = *a;
        else v[s].x = *a;
      } else {
        v[s] = *a;
      }
    }
  }

  // exchange between pass I and pass I + 1 (outputs of I -> inputs of I + 1)
  template <int I, bool SPLIT, class Lay, class Buf>
  __device__ static __forceinline__ void xchg_pass(float2 (&v)[E], Buf* lds) {
#pragma unroll
    for (int part = 0; part < (SPLIT ? 2 : 1); ++part) {
      __syncthreads();
      lds_put<I, true, SPLIT, Lay>(v, lds, opaque(), part);
      __syncthreads();
      lds_get<I + 1, false, SPLIT, Lay>(v, lds, opaque(), part);
    }
  }

  // entry: FftR's layout (slot s = butterfly bfly(t, s / R0), input s % R0)
  // -> the first pass's inputs; exit: the last pass's outputs -> FftR's
  // layout (PAIRED map of the first / last pass as the caller uses it)
  template <bool PAIRED, bool SPLIT, class Lay, class Buf>
  __device__ static __forceinline__ void xchg_entry(float2 (&v)[E], Buf* lds, int line, int t) {
    constexpr int R0 = kPlan.r[0], NB0 = L / R0;
#pragma unroll
    for (int part = 0; part < (SPLIT ? 2 : 1); ++part) {
      __syncthreads();
#pragma unroll
      for (int s = 0; s < E; ++s) {
        Buf* a = lds + Lay::addr(line, Outer::template bfly<0, PAIRED>(t, s / R0) + (s % R0) * NB0);
        if constexpr (SPLIT) *a = part ? v[s].y : v[s].x;
        else *a = v[s];
      }
      __syncthreads();
      lds_get<0, false, SPLIT, Lay>(v, lds, opaque(), part);
    }
  }
  template <bool PAIRED, bool SPLIT, class Lay, class Buf>
  __device__ static __forceinline__ void xchg_exit(float2 (&v)[E], Buf* lds, int line, int t) {
    constexpr int LAST = kPlan.n - 1, RL = kPlan.r[LAST], NBL = L / RL;
#pragma unroll
    for (int part = 0; part < (SPLIT ? 2 : 1); ++part) {
      __syncthreads();
      lds_put<kM.n - 1, true, SPLIT, Lay>(v, lds, opaque(), part);
      __syncthreads();
#pragma unroll
      for (int s = 0; s < E; ++s) {
        const Buf* a = lds + Lay::addr(line, Outer::template bfly<LAST, PAIRED>(t, s / RL) + (s % RL) * NBL);
        if constexpr (SPLIT) {
          if (part) v[s].y = *a;
          else v[s].x = *a;
        } else {
          v[s] = *a;
        }
      }
    }
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

  // twiddles and (FP16) scale of group c's inputs, then the hi / lo operands
  template <int I, class V>
  __device__ static __forceinline__ void operands(float2 (&v)[E], int c, int tid, const float2* __restrict__ tw,
                                                  V& bh, V& bl, float& inv) {
    constexpr int R = kM.r[I], NS = ns<I>(), PER = per<I>();
    const int g = (tid & 63) >> 4;
    float2* x = v + c * PER;
    if constexpr (NS > 1) {
      int ln = 0, j = 0;
      which<I>(tid, c, ln, j);
      // the lane's PER powers, consecutive in the lane table behind the
      // length-L table (see mfma_lane_twiddle_offset)
      const unsigned m = (unsigned)j % (unsigned)NS;
      const float4* lt = reinterpret_cast<const float4*>(
          tw + L + mfma_lane_twiddle_offset(L, I) + (m * 4u + (unsigned)g) * PER);
      float2 w[PER];
#pragma unroll
      for (int q = 0; q < PER / 2; ++q) {
        const float4 t4 = lt[q];
        w[2 * q] = make_float2(t4.x, t4.y);
        w[2 * q + 1] = make_float2(t4.z, t4.w);
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        if (INV) w[i].y = -w[i].y;
        x[i] = c_mul(x[i], w[i]);
      }
    }
    float sc = 1.f;
    inv = 1.f;
    if constexpr (H::kScaled) {
      float mx = 0.f;
#pragma unroll
      for (int i = 0; i < PER; ++i) mx = fmaxf(mx, fmaxf(fabsf(x[i].x), fabsf(x[i].y)));
      fp16_scale(max_over_rows(mx), sc, inv);
    }
    static_assert(R == 16 || R == 8, "radix 16 or 8");
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      T ha, hb, la, lb;
      split2_pair(x[i].x * sc, x[i].y * sc, ha, hb, la, lb);
      bh[2 * i] = ha;
      bh[2 * i + 1] = hb;
      bl[2 * i] = la;
      bl[2 * i + 1] = lb;
    }
  }

  // NG groups at a time: their operands first, then their products issued
  // interleaved, so that 2 NG (radix 16: real and imaginary rows) or NG
  // (radix 8) independent accumulation chains cover each other's latency
  // (every chain still accumulates lo.hi, hi.lo, hi.hi in that order)
  template <int I>
  __device__ static __forceinline__ void compute(float2 (&v)[E], const Coef& A, const float2* __restrict__ tw) {
    constexpr int R = kM.r[I], PER = per<I>(), G = groups<I>();
    constexpr int NG = R == 16 ? 2 : 4;
    static_assert(G % NG == 0, "whole group sets");
    const int tid = opaque();
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c0 = 0; c0 < G; c0 += NG) {
      if constexpr (R == 16) {
        typename H::V8 bh[NG], bl[NG];
        float inv[NG];
#pragma unroll
        for (int k = 0; k < NG; ++k) operands<I>(v, c0 + k, tid, tw, bh[k], bl[k], inv[k]);
        f32x4 yr[NG], yi[NG];
#pragma unroll
        for (int k = 0; k < NG; ++k) {
          yr[k] = H::mma16(A.re_lo, bh[k], z);
          yi[k] = H::mma16(A.im_lo, bh[k], z);
        }
#pragma unroll
        for (int k = 0; k < NG; ++k) {
          yr[k] = H::mma16(A.re_hi, bl[k], yr[k]);
          yi[k] = H::mma16(A.im_hi, bl[k], yi[k]);
        }
#pragma unroll
        for (int k = 0; k < NG; ++k) {
          yr[k] = H::mma16(A.re_hi, bh[k], yr[k]);
          yi[k] = H::mma16(A.im_hi, bh[k], yi[k]);
        }
#pragma unroll
        for (int k = 0; k < NG; ++k) {
          float2* x = v + (c0 + k) * PER;
#pragma unroll
          for (int i = 0; i < 4; ++i) x[i] = make_float2(yr[k][i] * inv[k], yi[k][i] * inv[k]);
        }
      } else {
        typename H::V4 bh[NG], bl[NG];
        float inv[NG];
#pragma unroll
        for (int k = 0; k < NG; ++k) operands<I>(v, c0 + k, tid, tw, bh[k], bl[k], inv[k]);
        f32x4 y[NG];
#pragma unroll
        for (int k = 0; k < NG; ++k) y[k] = H::mma8(A.r8_lo, bh[k], z);
#pragma unroll
        for (int k = 0; k < NG; ++k) y[k] = H::mma8(A.r8_hi, bl[k], y[k]);
#pragma unroll
        for (int k = 0; k < NG; ++k) y[k] = H::mma8(A.r8_hi, bh[k], y[k]);
#pragma unroll
        for (int k = 0; k < NG; ++k) {
          float2* x = v + (c0 + k) * PER;
          x[0] = make_float2(y[k][0] * inv[k], y[k][1] * inv[k]);
          x[1] = make_float2(y[k][2] * inv[k], y[k][3] * inv[k]);
        }
      }
    }
  }

  template <int I, bool SPLIT, class Lay, class Buf>
  __device__ static __forceinline__ void passes(float2 (&v)[E], Buf* lds, const Coef& A,
                                                const float2* __restrict__ tw) {
    compute<I>(v, A, tw);
    if constexpr (I + 1 < kM.n) {
      xchg_pass<I, SPLIT, Lay>(v, lds);
      passes<I + 1, SPLIT, Lay>(v, lds, A, tw);
    }
  }

  // Native layout: slot s of a lane holds input element idx of transform ln
  // of the first matrix-core pass (native_in) and receives output element
  // idx of the last one (native_out).  Callers that load or store in this
  // layout skip the re-layout through LDS on that side (run_ex).
  __device__ static __forceinline__ void native_in(int tid, int s, int& ln, int& idx) { in_pos<0>(tid, s, ln, idx); }
  __device__ static __forceinline__ void native_out(int tid, int s, int& ln, int& idx) {
    out_pos<kM.n - 1>(tid, s, ln, idx);
  }
  // every slot of a thread in its slot-0 transform, element = slot 0's + K(s)
  static constexpr bool kNativeInLin = lin_idx<0, false>();
  static constexpr bool kNativeOutLin = lin_idx<kM.n - 1, true>();
  static constexpr Offs kNativeInOff = idx_offsets<0, false>();
  static constexpr Offs kNativeOutOff = idx_offsets<kM.n - 1, true>();
  // every slot of a lane belongs to one transform, in the first and in the
  // last pass (line-major butterfly numbering and whole waves per line)
  template <int I>
  static constexpr bool one_line() {
    return !LINE_FASTEST && (L / kM.r[I]) % (groups<I>() * 16) == 0;
  }
  static constexpr bool kLaneOneLine = one_line<0>() && one_line<kM.n - 1>();

  // NATIVE_IN: v holds the first pass's inputs in the native layout (else in
  // FftR's, PAIRED_FIRST map); NATIVE_OUT: v receives the last pass's outputs
  // in the native layout (else FftR's, PAIRED_LAST map).
  template <bool NATIVE_IN, bool NATIVE_OUT, bool PAIRED_FIRST, bool PAIRED_LAST, bool SPLIT, class Lay, class Buf>
  __device__ static __forceinline__ void run_ex(float2 (&v)[E], int line, int t, Buf* lds,
                                                const float2* __restrict__ tw) {
    Coef A;
    coefs(A);
    if constexpr (!NATIVE_IN) xchg_entry<PAIRED_FIRST, SPLIT, Lay>(v, lds, line, t);
    passes<0, SPLIT, Lay>(v, lds, A, tw);
    if constexpr (!NATIVE_OUT) xchg_exit<PAIRED_LAST, SPLIT, Lay>(v, lds, line, t);
  }

  // (FftR's calling convention; the split-precision kernels always run with
  // every thread of the block in a transform, so `live` is always true here)
  template <bool PAIRED_FIRST, bool PAIRED_LAST, bool SPLIT, class Lay, class Buf>
  __device__ static __forceinline__ void run(float2 (&v)[E], int line, int t, Buf* lds,
                                             const float2* __restrict__ tw, bool /*live*/ = true) {
    run_ex<false, false, PAIRED_FIRST, PAIRED_LAST, SPLIT, Lay>(v, line, t, lds, tw);
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
