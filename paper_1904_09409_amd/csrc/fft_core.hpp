// fft_core.hpp -- device building blocks of the funnel transform's 1D DFTs.
//
// A transform of length L is computed by P cooperating threads with the
// Stockham self-sorting formulation: for a pass of radix R after the radices
// already applied (product NS), butterfly j reads x[j + r L/R], r = 0..R-1,
// multiplies input r by w_L^(r (j mod NS) L/(NS R)), takes the R-point DFT and
// writes output q to (j/NS) NS R + (j mod NS) + q NS.  The first pass reads
// through a caller functor (a global load, or the NVMT gather) and the last
// pass writes through another, so only the exchanges in between touch LDS.
// Radix schedules are fixed at compile time from the factorisation of L
// (16/8/4/2 for the power-of-two part, then 7, 5, 3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace funnel {

// ---------------------------------------------------------------- complex ops

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 c_mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// multiply by exp(-+ i 2 pi m / R) given (cos, sin) of 2 pi m / R
template <bool INV>
__device__ __forceinline__ float2 c_rot(float2 a, float c, float s) {
  const float ss = INV ? s : -s;
  return make_float2(a.x * c - a.y * ss, a.x * ss + a.y * c);
}

// ---------------------------------------------------------------- radix plan

struct RadixPlan {
  int n;
  int r[24];
};

constexpr RadixPlan radix_plan(int L) {
  RadixPlan p{0, {}};
  int rem = L, a = 0;
  while (rem % 2 == 0) { rem /= 2; ++a; }
  while (a >= 4) { p.r[p.n++] = 16; a -= 4; }
  if (a == 3) p.r[p.n++] = 8;
  else if (a == 2) p.r[p.n++] = 4;
  else if (a == 1) p.r[p.n++] = 2;
  while (rem % 7 == 0) { p.r[p.n++] = 7; rem /= 7; }
  while (rem % 5 == 0) { p.r[p.n++] = 5; rem /= 5; }
  while (rem % 3 == 0) { p.r[p.n++] = 3; rem /= 3; }
  if (rem != 1) p.n = 0;  // not 7-smooth: rejected at compile time below
  return p;
}

constexpr int max_radix(int L) {
  RadixPlan p = radix_plan(L);
  int m = 1;
  for (int i = 0; i < p.n; ++i) m = p.r[i] > m ? p.r[i] : m;
  return m;
}

// threads cooperating on one transform of length L
constexpr int threads_per_transform(int L) { return L / max_radix(L); }

// ---------------------------------------------------------------- small DFTs

template <bool INV>
__device__ __forceinline__ void dft2(float2& a0, float2& a1) {
  const float2 t = a0;
  a0 = c_add(t, a1);
  a1 = c_sub(t, a1);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = c_add(a0, a2), t1 = c_sub(a0, a2);
  const float2 t2 = c_add(a1, a3), t3 = c_mul_mi<INV>(c_sub(a1, a3));
  a0 = c_add(t0, t2);
  a2 = c_sub(t0, t2);
  a1 = c_add(t1, t3);
  a3 = c_sub(t1, t3);
}

// cos and sin of 2 pi m / 16
__device__ constexpr float kCos16[16] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508978f,
    0.0f, -0.38268343236508978f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508978f,
    0.0f, 0.38268343236508978f, 0.70710678118654752f, 0.92387953251128674f};
__device__ constexpr float kSin16[16] = {
    0.0f, 0.38268343236508978f, 0.70710678118654752f, 0.92387953251128674f,
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508978f,
    0.0f, -0.38268343236508978f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508978f};

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __device__ static __forceinline__ void run(float2* v) { dft2<INV>(v[0], v[1]); }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ static __forceinline__ void run(float2* v) { dft4<INV>(v[0], v[1], v[2], v[3]); }
};

// 8 = 2 x 4: even and odd 4-point DFTs, then one twiddled radix-2 stage
template <bool INV>
struct Dft<8, INV> {
  __device__ static __forceinline__ void run(float2* v) {
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    o1 = c_rot<INV>(o1, kCos16[2], kSin16[2]);
    o2 = c_mul_mi<INV>(o2);
    o3 = c_rot<INV>(o3, kCos16[6], kSin16[6]);
    v[0] = c_add(e0, o0); v[4] = c_sub(e0, o0);
    v[1] = c_add(e1, o1); v[5] = c_sub(e1, o1);
    v[2] = c_add(e2, o2); v[6] = c_sub(e2, o2);
    v[3] = c_add(e3, o3); v[7] = c_sub(e3, o3);
  }
};

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
template <bool INV>
struct Dft<16, INV> {
  __device__ static __forceinline__ void run(float2* v) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // v[n2 + 4 k1] now holds Y[n2][k1]; twiddle by w16^(n2 k1)
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
      for (int k1 = 1; k1 < 4; ++k1) {
        const int m = (n2 * k1) & 15;
        v[n2 + 4 * k1] = c_rot<INV>(v[n2 + 4 * k1], kCos16[m], kSin16[m]);
      }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4x4 index
    float2 t[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) t[i] = v[i];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[4 * k1 + k2];
  }
};

// odd prime radices by the symmetric form: t_n = a_n + a_{R-n}, d_n = a_n - a_{R-n},
// X_k = a0 + sum_n C(nk) t_n -+ i sum_n S(nk) d_n,  X_{R-k} with the opposite sign
template <int R>
struct OddTrig;
template <>
struct OddTrig<3> {
  __device__ static constexpr float c(int m) { return m == 0 ? 1.0f : -0.5f; }
  __device__ static constexpr float s(int m) {
    return m == 0 ? 0.0f : (m == 1 ? 0.86602540378443865f : -0.86602540378443865f);
  }
};
template <>
struct OddTrig<5> {
  __device__ static constexpr float c(int m) {
    return m == 0 ? 1.0f : (m == 1 || m == 4) ? 0.30901699437494742f : -0.80901699437494742f;
  }
  __device__ static constexpr float s(int m) {
    return m == 0 ? 0.0f
           : m == 1 ? 0.95105651629515357f
           : m == 2 ? 0.58778525229247313f
           : m == 3 ? -0.58778525229247313f
                    : -0.95105651629515357f;
  }
};
template <>
struct OddTrig<7> {
  __device__ static constexpr float c(int m) {
    return m == 0 ? 1.0f
           : (m == 1 || m == 6) ? 0.62348980185873353f
           : (m == 2 || m == 5) ? -0.22252093395631440f
                                : -0.90096886790241913f;
  }
  __device__ static constexpr float s(int m) {
    return m == 0 ? 0.0f
           : m == 1 ? 0.78183148246802981f
           : m == 2 ? 0.97492791218182361f
           : m == 3 ? 0.43388373911755812f
           : m == 4 ? -0.43388373911755812f
           : m == 5 ? -0.97492791218182361f
                    : -0.78183148246802981f;
  }
};

template <int R, bool INV>
struct DftOdd {
  __device__ static __forceinline__ void run(float2* v) {
    constexpr int H = (R - 1) / 2;
    float2 t[H + 1], d[H + 1];
#pragma unroll
    for (int n = 1; n <= H; ++n) {
      t[n] = c_add(v[n], v[R - n]);
      d[n] = c_sub(v[n], v[R - n]);
    }
    const float2 a0 = v[0];
    float2 x0 = a0;
#pragma unroll
    for (int n = 1; n <= H; ++n) x0 = c_add(x0, t[n]);
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      float2 re = a0, im = make_float2(0.f, 0.f);
#pragma unroll
      for (int n = 1; n <= H; ++n) {
        const int m = (n * k) % R;
        re.x += OddTrig<R>::c(m) * t[n].x;
        re.y += OddTrig<R>::c(m) * t[n].y;
        im.x += OddTrig<R>::s(m) * d[n].x;
        im.y += OddTrig<R>::s(m) * d[n].y;
      }
      // forward: X_k = re - i im, X_{R-k} = re + i im ; inverse: signs swapped
      const float2 mi = INV ? make_float2(-im.y, im.x) : make_float2(im.y, -im.x);
      v[k] = c_add(re, mi);
      v[R - k] = c_sub(re, mi);
    }
    v[0] = x0;
  }
};
template <bool INV>
struct Dft<3, INV> : DftOdd<3, INV> {};
template <bool INV>
struct Dft<5, INV> : DftOdd<5, INV> {};
template <bool INV>
struct Dft<7, INV> : DftOdd<7, INV> {};

// ---------------------------------------------------------------- LDS layouts

// Several transforms interleaved (transform index fastest); a pad float2 every
// 16 elements keeps radix-16 strides off a single bank.
template <int LINES>
struct LayInter {
  __device__ static __forceinline__ int addr(int line, int idx) { return (idx + (idx >> 4)) * LINES + line; }
  static constexpr int size(int L) { return (L + L / 16 + 1) * LINES; }
};

// One transform after another.
template <int LINES, int L>
struct LayRow {
  static constexpr int kStride = L + L / 16 + 1;
  __device__ static __forceinline__ int addr(int line, int idx) { return line * kStride + idx + (idx >> 4); }
  static constexpr int caddr(int line, int idx) { return line * kStride + idx + (idx >> 4); }   // (same, constexpr)
  static constexpr int size(int) { return kStride * LINES; }
  // addr(line, x + d) = addr(line, x) + coff(d) when (x mod 16) + (d mod 16) < 16
  static constexpr int coff(int d) { return d + (d >> 4); }
};

// ---------------------------------------------------------------- Stockham driver

// FL: float2 (int idx) -- input element idx of this thread's transform (first pass)
// LS: void (int idx, float2 v) -- output element idx (last pass)
// Every thread of the block must call run(); t in [0, P) identifies the thread
// within its transform, line selects the transform's LDS region.
template <int L, int P, bool INV, class Lay>
struct Fft {
  static constexpr RadixPlan kPlan = radix_plan(L);
  static_assert(kPlan.n > 0, "transform length must be 7-smooth");

  template <int I, int NS, class FL, class LS>
  __device__ static __forceinline__ void pass(int line, int t, float2* lds, const float2* __restrict__ tw,
                                              FL& fl, LS& ls) {
    constexpr int R = kPlan.r[I];
    constexpr int NB = L / R;
    constexpr int BPT = (NB + P - 1) / P;
    constexpr bool FIRST = (I == 0);
    constexpr bool LAST = (I == kPlan.n - 1);
    float2 v[BPT][R];
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int j = t + b * P;
      if ((NB % P == 0) || j < NB) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int idx = j + r * NB;
          if constexpr (FIRST) v[b][r] = fl(idx);
          else v[b][r] = lds[Lay::addr(line, idx)];
        }
        if constexpr (NS > 1) {
          const int k = j % NS;
          constexpr int STRIDE = L / (NS * R);
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 w = tw[r * k * STRIDE];
            if (INV) w.y = -w.y;
            v[b][r] = c_mul(v[b][r], w);
          }
        }
        Dft<R, INV>::run(v[b]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int j = t + b * P;
      if ((NB % P == 0) || j < NB) {
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int idx = base + q * NS;
          if constexpr (LAST) ls(idx, v[b][q]);
          else lds[Lay::addr(line, idx)] = v[b][q];
        }
      }
    }
    if constexpr (!LAST) {
      __syncthreads();
      pass<I + 1, NS * R>(line, t, lds, tw, fl, ls);
    }
  }

  template <class FL, class LS>
  __device__ static __forceinline__ void run(int line, int t, float2* lds, const float2* __restrict__ tw, FL& fl,
                                             LS& ls) {
    pass<0, 1>(line, t, lds, tw, fl, ls);
  }
};

// floor(a / d) for d > 0 from a float reciprocal inv = 1/d: the estimate is
// within one of the quotient while |a| < 2^26 and |a / d| < 2^21, and one
// remainder test makes it exact (larger quotients may stay off by one; the
// callers only use quotients that land in a row of at most 4096 samples).
__device__ __forceinline__ int floor_div_rcp(int a, int d, float inv) {
  int q = (int)floorf((float)a * inv);
  const int r = a - q * d;
  q += (r >= d) - (r < 0);
  return q;
}
__device__ __forceinline__ int ceil_div_rcp(int a, int d, float inv) { return -floor_div_rcp(-a, d, inv); }

// floor(a / b) and ceil(a / b) for b > 0 and any sign of a
__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
__device__ __forceinline__ int ceil_div(int a, int b) { return a >= 0 ? (a + b - 1) / b : -((-a) / b); }

}  // namespace funnel

namespace funnel {

// ---------------------------------------------------------------- register-resident engine
//
// FftR keeps a thread's elements in registers for the whole transform; pass I
// sees them as BPT_I butterflies of radix R_I, and between passes the data
// goes through LDS once.  With SPLIT the real and the imaginary parts are
// exchanged one after the other through a float buffer of half the size.
//
// Butterfly maps: slot b of pass I is butterfly t + P b, except in a PAIRED
// pass, where slot 2c is ja = t + P c (ja < NB/2) and slot 2c+1 its Hermitian
// partner NB - ja (NB/2 for ja = 0).  In the first pass (NS = 1) partners read
// inputs idx and L - idx; in the last pass (NS = NB) they write outputs idx and
// L - idx.  Keeping both in one thread lets a real-input transform separate
// its two columns, and a Hermitian inverse build its input, in registers.
//
// BPT_I = ceil(NB_I / P) (pairs: ceil(NB_I/2 / P)), so P need not divide the
// butterfly counts of mixed-radix lengths: slots past the last butterfly are
// computed on whatever they hold and never written to LDS or read from it
// (ok() is false there).  When P divides every count the guards fold away.
// Registers: v[EM], EM = the largest BPT_I R_I over the passes.

constexpr RadixPlan reversed(RadixPlan p) {
  RadixPlan q = p;
  for (int i = 0; i < p.n; ++i) q.r[i] = p.r[p.n - 1 - i];
  return q;
}

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// REV runs the radices smallest-first (for the radix-16 lengths the pairing
// then falls on the small last radix of the forward order).
template <int L, int P, bool INV, bool REV = false>
struct FftR {
  static constexpr RadixPlan kPlan = REV ? reversed(radix_plan(L)) : radix_plan(L);
  static_assert(kPlan.n > 0, "transform length must be 7-smooth");

  template <int I, bool PAIRED>
  static constexpr int bpt() {
    constexpr int NB = L / kPlan.r[I];
    return PAIRED ? 2 * cdiv(NB / 2, P) : cdiv(NB, P);
  }
  // every butterfly slot of pass I is a real butterfly for every thread
  template <int I, bool PAIRED>
  static constexpr bool exact() {
    constexpr int NB = L / kPlan.r[I];
    return PAIRED ? (NB / 2) % P == 0 : NB % P == 0;
  }
  // the paired pass is the first one of a reversed engine (Hermitian input)
  // and the last one of a forward engine (two real columns out)
  static constexpr int slots() {
    int m = 0;
    for (int i = 0; i < kPlan.n; ++i) {
      const int NB = L / kPlan.r[i];
      const int a = cdiv(NB, P) * kPlan.r[i];
      m = a > m ? a : m;
      if (i == (REV ? 0 : kPlan.n - 1)) {
        const int b = 2 * cdiv(NB / 2, P) * kPlan.r[i];
        m = b > m ? b : m;
      }
    }
    return m;
  }
  static constexpr int EM = slots();
  static constexpr int E = EM;

  template <int I>
  static constexpr int ns() {
    int p = 1;
    for (int i = 0; i < I; ++i) p *= kPlan.r[i];
    return p;
  }

  template <int I, bool PAIRED>
  __device__ static __forceinline__ int bfly(int t, int b) {
    constexpr int NB = L / kPlan.r[I];
    if constexpr (!PAIRED) {
      return t + P * b;
    } else {
      const int ja = t + P * (b >> 1);
      if ((b & 1) == 0) return ja;
      return ja == 0 ? NB / 2 : NB - ja;
    }
  }
  // slot b of pass I holds a butterfly of this thread
  template <int I, bool PAIRED>
  __device__ static __forceinline__ bool ok(int t, int b) {
    constexpr int NB = L / kPlan.r[I];
    if constexpr (exact<I, PAIRED>()) return true;
    else if constexpr (PAIRED) return t + P * (b >> 1) < NB / 2;
    else return t + P * b < NB;
  }

  // twiddle (base from the table, powers by balanced products) + R-point DFT.
  // One table read per butterfly instead of R - 1 keeps the memory pipeline
  // free for the data; the powers carry the table entry's rounding times r
  // (a few 1e-7 relative, well inside the FP32 error budget).
  template <int I, bool PAIRED>
  __device__ static __forceinline__ void compute(float2 (&v)[EM], int t, const float2* __restrict__ tw) {
    constexpr int R = kPlan.r[I], NS = ns<I>(), BPT = bpt<I, PAIRED>();
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      float2* x = v + b * R;
      if constexpr (NS > 1) {
        const int j = bfly<I, PAIRED>(t, b);
        const int k = j % NS;
        float2 w[R];
        w[1] = tw[k * (L / (NS * R))];
        if (INV) w[1].y = -w[1].y;
#pragma unroll
        for (int r = 2; r < R; ++r) w[r] = c_mul(w[r / 2], w[r - r / 2]);
#pragma unroll
        for (int r = 1; r < R; ++r) x[r] = c_mul(x[r], w[r]);
      }
      Dft<R, INV>::run(x);
    }
  }

  // LDS exchange: outputs of pass I -> inputs of pass I+1.  Lay::addr(line, idx)
  // addresses a float (SPLIT) or float2 slot.
  //
  // Unpaired exact maps put every index of a thread at x(t) + d with d a
  // compile-time constant and no carry out of the low 4 bits of x(t), so the
  // address is one per-thread base plus an immediate (Lay::coff): writes of a
  // pass with NS | P (x = (t/NS) NS R + t mod NS, d = P R b + q NS), reads
  // with x = t, d = P b + r L/R.  Other maps keep per-slot addresses.
  // (checked exhaustively at compile time: every thread t, slot and offset)
  template <int I, bool PAIRED_OUT>
  static constexpr bool lin_write() {
    constexpr int R = kPlan.r[I], NS = ns<I>();
    if (PAIRED_OUT || !exact<I, false>() || P % NS != 0) return false;
    for (int t = 0; t < P; ++t)
      for (int b = 0; b < bpt<I, false>(); ++b)
        for (int q = 0; q < R; ++q) {
          const int j = t + P * b, x = (t / NS) * NS * R + t % NS, d = P * R * b + q * NS;
          if (x + d != (j / NS) * NS * R + j % NS + q * NS || x % 16 + d % 16 >= 16) return false;
        }
    return true;
  }
  template <int I, bool PAIRED_IN>
  static constexpr bool lin_read() {
    constexpr int R = kPlan.r[I], NB = L / R;
    if (PAIRED_IN || !exact<I, false>()) return false;
    for (int t = 0; t < P; ++t)
      for (int b = 0; b < bpt<I, false>(); ++b)
        for (int r = 0; r < R; ++r)
          if (t % 16 + (P * b + r * NB) % 16 >= 16) return false;
    return true;
  }

  template <int I, bool PAIRED_OUT, class Lay, class Buf, class GET>
  __device__ static __forceinline__ void xwrite(int line, int t, Buf* lds, GET get) {
    constexpr int R = kPlan.r[I], NS = ns<I>(), BPT = bpt<I, PAIRED_OUT>();
    if constexpr (lin_write<I, PAIRED_OUT>()) {
      Buf* base = lds + Lay::addr(line, (t / NS) * NS * R + t % NS);
#pragma unroll
      for (int b = 0; b < BPT; ++b)
#pragma unroll
        for (int q = 0; q < R; ++q) base[Lay::coff(P * R * b + q * NS)] = get(b * R + q);
    } else {
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        if (!ok<I, PAIRED_OUT>(t, b)) continue;
        const int j = bfly<I, PAIRED_OUT>(t, b);
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int q = 0; q < R; ++q) lds[Lay::addr(line, base + q * NS)] = get(b * R + q);
      }
    }
  }

  template <int I, bool PAIRED_IN, class Lay, class Buf, class PUT>
  __device__ static __forceinline__ void xread(int line, int t, const Buf* lds, PUT put) {
    constexpr int R2 = kPlan.r[I], NB2 = L / R2, BPT2 = bpt<I, PAIRED_IN>();
    if constexpr (lin_read<I, PAIRED_IN>()) {
      const Buf* base = lds + Lay::addr(line, t);
#pragma unroll
      for (int b = 0; b < BPT2; ++b)
#pragma unroll
        for (int r = 0; r < R2; ++r) put(b * R2 + r, base[Lay::coff(P * b + r * NB2)]);
    } else {
#pragma unroll
      for (int b = 0; b < BPT2; ++b) {
        if (!ok<I, PAIRED_IN>(t, b)) continue;
        const int j = bfly<I, PAIRED_IN>(t, b);
#pragma unroll
        for (int r = 0; r < R2; ++r) put(b * R2 + r, lds[Lay::addr(line, j + r * NB2)]);
      }
    }
  }

  // The thread's coordinates pass through an empty asm after the barrier, so
  // that the exchange's LDS addresses are computed there and not hoisted into
  // the register-heavy butterflies before it (where they were spilled).
  __device__ static __forceinline__ void pin(int& line, int& t) { asm volatile("" : "+v"(line), "+v"(t)); }

  // live = false: a thread of the block that holds no part of a transform
  // (blocks sized for a larger tile); it keeps every barrier but touches no
  // LDS.
  template <int I, bool PAIRED_OUT, bool PAIRED_IN, bool SPLIT, class Lay, class Buf>
  __device__ static __forceinline__ void exchange(float2 (&v)[EM], int line, int t, Buf* lds, bool live) {
    if constexpr (!SPLIT) {
      __syncthreads();
      pin(line, t);
      if (live) xwrite<I, PAIRED_OUT, Lay>(line, t, lds, [&](int s) { return v[s]; });
      __syncthreads();
      if (live) xread<I + 1, PAIRED_IN, Lay>(line, t, lds, [&](int s, float2 f) { v[s] = f; });
    } else {
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        __syncthreads();
        pin(line, t);
        if (live) xwrite<I, PAIRED_OUT, Lay>(line, t, lds, [&](int s) { return part ? v[s].y : v[s].x; });
        __syncthreads();
        if (live)
          xread<I + 1, PAIRED_IN, Lay>(line, t, lds, [&](int s, float f) {
            if (part) v[s].y = f;
            else v[s].x = f;
          });
      }
    }
  }

  // All passes after the caller loaded pass 0's inputs into v (with the
  // PAIRED_FIRST map, slots b with ok<0>).  On return v holds the last pass's
  // outputs (with the PAIRED_LAST map): slot b, output q is element
  // j + q * (L / R_last), for the slots with ok<last>.
  template <bool PAIRED_FIRST, bool PAIRED_LAST, bool SPLIT, class Lay, class Buf, int I = 0>
  __device__ static __forceinline__ void run(float2 (&v)[EM], int line, int t, Buf* lds,
                                             const float2* __restrict__ tw, bool live = true) {
    static_assert(!(PAIRED_FIRST && !REV) && !(PAIRED_LAST && REV), "EM counts the paired pass of this order only");
    constexpr bool FIRST = I == 0, LAST = I == kPlan.n - 1;
    constexpr bool PAIRED = (FIRST && PAIRED_FIRST) || (LAST && PAIRED_LAST);
    compute<I, PAIRED>(v, t, tw);
    if constexpr (!LAST) {
      constexpr bool NEXT_PAIRED = (I + 1 == kPlan.n - 1) && PAIRED_LAST;
      exchange<I, PAIRED, NEXT_PAIRED, SPLIT, Lay>(v, line, t, lds, live);
      run<PAIRED_FIRST, PAIRED_LAST, SPLIT, Lay, Buf, I + 1>(v, line, t, lds, tw, live);
    }
  }
};

// Layouts for the register engine: element slots of LINES transforms,
// transform index fastest, one pad slot every 16 elements.
template <int LINES>
struct LayInterR {
  __device__ static __forceinline__ int addr(int line, int idx) { return (idx + (idx >> 4)) * LINES + line; }
  static constexpr int caddr(int line, int idx) { return (idx + (idx >> 4)) * LINES + line; }   // (same, constexpr)
  static constexpr int size(int L) { return (L + L / 16 + 1) * LINES; }
  // addr(line, x + d) = addr(line, x) + coff(d) when (x mod 16) + (d mod 16) < 16
  static constexpr int coff(int d) { return (d + (d >> 4)) * LINES; }
};

// Map the linear block index so that consecutive logical tiles run on the same
// XCD (blocks are dealt round-robin over the 8 XCDs): neighbouring column tiles
// then share their cache lines in one L2.
__device__ __forceinline__ int xcd_remap(int lin, int total) {
  constexpr int X = 8;
  const int xcd = lin % X, slot = lin / X;
  const int q = total / X, r = total % X;
  return xcd * q + (xcd < r ? xcd : r) + slot;
}

}  // namespace funnel
