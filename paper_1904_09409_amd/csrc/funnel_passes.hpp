// funnel_passes.hpp -- the three passes of the funnel transform and of its
// adjoint, for gfx950.
//
// Pass A  (Sec. 3.1 step 1, Sec. 4.2): DFT along y of every column of the
//         expanded image; only rows n2 = 1 .. Np/2-1 of the half spectrum are
//         kept (the rest follow by conjugate symmetry).  Two real columns ride
//         in one complex transform (z = a + i b) and are separated afterwards.
// Pass B  (steps 2 and 3, Eq. 17): per frequency row, the NVMT as a linear-
//         interpolation gather from the LDS copy of the row, fused into the
//         first butterfly pass of the DFT along x'.
// Pass C  (step 4): Hermitian inverse DFT along omega_2 of every column,
//         again two columns per complex transform, scaled by 1/Np.
// The inverse space (dual form, Sec. 3.1) is pass A reading image rows
// instead of columns; passes B and C are unchanged.  The adjoint runs the
// transposed passes in reverse order.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_core.hpp"
#include "fft_mfma.hpp"
#include "funnel_internal.hpp"

namespace funnel {

// ------------------------------------------------------------------ tiling

constexpr int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

// LDS-resident kernels (any 7-smooth length).  Variant V sets the threads
// per transform P (each thread takes ceil(L/R / P) butterflies of a radix-R
// pass) and with it how many column pairs share a block:
//   V = 0: P = L / (largest radix), pairs a power of two <= 16;
//   V = 1: P <= 128, as many pairs as 1024 threads and ~150 KB of LDS allow;
//   V = 2: P <= 64, likewise.
// More pairs per block means wider row segments in HBM for the column
// passes; fewer threads per transform means more butterflies per thread.
constexpr int kGenVariants = 3;

template <int L, int V = 0>
struct ColCfg {
  static constexpr int TPT = threads_per_transform(L);
  static constexpr int P = V == 0 ? TPT : (V == 1 ? (TPT < 128 ? TPT : 128) : (TPT < 64 ? TPT : 64));
  static constexpr int lines_by_threads = 1024 / P > 0 ? 1024 / P : 1;
  static constexpr int lines_by_lds = (150 * 1024) / (8 * (L + L / 16 + 1));
  static constexpr int LINES0 = lines_by_threads < lines_by_lds ? lines_by_threads : lines_by_lds;
  static constexpr int LINES = V == 0 ? pow2_floor(LINES0 > 16 ? 16 : (LINES0 < 1 ? 1 : LINES0))
                                      : (LINES0 < 1 ? 1 : LINES0);
  static constexpr int THREADS = LINES * P;
  // a variant other than 0 exists only where it differs from variant 0
  static constexpr bool distinct() {
    return V == 0 || (V < kGenVariants && (P != ColCfg<L, 0>::P || LINES != ColCfg<L, 0>::LINES) &&
                      (V == 1 || P != ColCfg<L, 1>::P));
  }
};

// V = 0: up to 256 threads per block; V = 1: up to 512
constexpr int kGenRowVariants = 2;

template <int M, int V = 0>
struct RowCfg {
  static constexpr int P = threads_per_transform(M);
  static constexpr int TPB = V == 0 ? 256 : 512;
  static constexpr int rows_by_threads = TPB / P > 0 ? TPB / P : 1;
  static constexpr int rows_by_lds = (64 * 1024) / (8 * (M + M / 16 + 1));
  static constexpr int ROWS0 = rows_by_threads < rows_by_lds ? rows_by_threads : rows_by_lds;
  static constexpr int ROWS = ROWS0 < 1 ? 1 : ROWS0;
  static constexpr int THREADS = ROWS * P;
  static constexpr bool distinct() { return V == 0 || (V < kGenRowVariants && ROWS != RowCfg<M, 0>::ROWS); }
};

// ------------------------------------------------------------------ pass A / adjoint of C
//
// Real lines of length `lin` placed at offset `off` in a zero frame of length
// L -> half spectrum X[k], k = 1 .. L/2-1, times scale * (-1)^k (the (-1)^k
// moves the origin to the frame centre).  TRANS = false: lines are the
// columns of a row-major [lin][nlines] array; TRANS = true: lines are the rows
// of a row-major [nlines][lin] array.  Output: complex [L/2-1][nlines].
template <int L, bool TRANS, int V>
__global__ void __launch_bounds__((ColCfg<L, V>::THREADS))
    k_r2c_half(const float* __restrict__ in, float2* __restrict__ out, int nlines, int lin, int off,
               ImgMap map, float scale, const float2* __restrict__ tw) {
  using Cfg = ColCfg<L, V>;
  constexpr int P = Cfg::P, LINES = Cfg::LINES, H = L / 2 - 1;
  using Lay = typename std::conditional<TRANS, LayRow<LINES, L>, LayInter<LINES>>::type;
  __shared__ float2 lds[Lay::size(L)];

  const int tid = threadIdx.x;
  const int pair = TRANS ? tid / P : tid % LINES;
  const int t = TRANS ? tid % P : tid / LINES;
  const int npairs = nlines >> 1;
  const int pg = blockIdx.x * LINES + pair;
  const bool active = pg < npairs;
  const float* src = in + map.in(blockIdx.y);

  auto fl = [&](int idx) -> float2 {
    const int r = idx - off;
    float2 z = make_float2(0.f, 0.f);
    if (active && r >= 0 && r < lin) {
      if constexpr (TRANS) {
        z.x = src[(long long)(2 * pg) * lin + r];
        z.y = src[(long long)(2 * pg + 1) * lin + r];
      } else {
        z = *reinterpret_cast<const float2*>(src + (long long)r * nlines + 2 * pg);
      }
    }
    return z;
  };
  auto ls = [&](int idx, float2 v) { lds[Lay::addr(pair, idx)] = v; };
  Fft<L, P, false, Lay>::run(pair, t, lds, tw, fl, ls);
  __syncthreads();

  // separate the two real columns: A = (Z_k + conj Z_{L-k})/2, B = (Z_k - conj Z_{L-k})/(2i)
  float4* dst = reinterpret_cast<float4*>(out + map.out(blockIdx.y));
  const int halfw = nlines >> 1;  // float4 per output row
  for (int e = tid; e < H * LINES; e += Cfg::THREADS) {
    const int p = e % LINES, k = 1 + e / LINES;
    const int pgl = blockIdx.x * LINES + p;
    if (pgl >= npairs) continue;
    const float2 zk = lds[Lay::addr(p, k)], zm = lds[Lay::addr(p, L - k)];
    const float sc = (k & 1) ? -0.5f * scale : 0.5f * scale;
    const float ux = zk.x - zm.x, uy = zk.y + zm.y;
    float4 o;
    o.x = sc * (zk.x + zm.x);
    o.y = sc * (zk.y - zm.y);
    o.z = sc * uy;
    o.w = -sc * ux;
    dst[(long long)(k - 1) * halfw + pgl] = o;
  }
}

// ------------------------------------------------------------------ pass C / adjoint of A
//
// Half spectrum X[k], k = 1 .. L/2-1 (complex [L/2-1][nlines]) -> real lines
// x[r] = scale * sum_k X~[k] e^{+i 2 pi k r / L} over the Hermitian completion
// X~[k] = (-1)^k X[k], X~[L-k] = conj X~[k], X~[0] = X~[L/2] = 0.  Only rows
// r in [r0, r0 + nout) are stored.  TRANS = false: out is [nout][nlines];
// TRANS = true: out is [nlines][nout].  ACCUM adds to out instead of storing.
template <int L, bool TRANS, bool ACCUM, int V>
__global__ void __launch_bounds__((ColCfg<L, V>::THREADS))
    k_c2r_half(const float2* __restrict__ in, float* __restrict__ out, int nlines, int r0, int nout,
               ImgMap map, float scale, const float2* __restrict__ tw) {
  using Cfg = ColCfg<L, V>;
  constexpr int P = Cfg::P, LINES = Cfg::LINES, H = L / 2 - 1;
  using Lay = typename std::conditional<TRANS, LayRow<LINES, L>, LayInter<LINES>>::type;
  static_assert((L / 2) * LINES * 2 <= Lay::size(L), "staging must fit the transform buffer");
  __shared__ float2 lds[Lay::size(L)];
  float4* stg = reinterpret_cast<float4*>(lds);

  const int tid = threadIdx.x;
  const int pair = TRANS ? tid / P : tid % LINES;
  const int t = TRANS ? tid % P : tid / LINES;
  const int npairs = nlines >> 1;
  const int pg = blockIdx.x * LINES + pair;
  const bool active = pg < npairs;

  const float4* src = reinterpret_cast<const float4*>(in + map.in(blockIdx.y));
  for (int e = tid; e < H * LINES; e += Cfg::THREADS) {
    const int p = e % LINES, k = 1 + e / LINES;
    const int pgl = blockIdx.x * LINES + p;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (pgl < npairs) v = src[(long long)(k - 1) * npairs + pgl];
    if (k & 1) v = make_float4(-v.x, -v.y, -v.z, -v.w);
    stg[k * LINES + p] = v;
  }
  __syncthreads();

  auto fl = [&](int idx) -> float2 {
    if (idx == 0 || idx == L / 2) return make_float2(0.f, 0.f);
    if (idx < L / 2) {
      const float4 v = stg[idx * LINES + pair];
      return make_float2(v.x - v.w, v.y + v.z);  // A + iB
    }
    const float4 v = stg[(L - idx) * LINES + pair];
    return make_float2(v.x + v.w, v.z - v.y);    // conj(A) + i conj(B)
  };
  float* dst = out + map.out(blockIdx.y);
  auto ls = [&](int idx, float2 z) {
    const int r = idx - r0;
    if (!active || r < 0 || r >= nout) return;
    const float a = scale * z.x, b = scale * z.y;
    if constexpr (TRANS) {
      float* pa = dst + (long long)(2 * pg) * nout + r;
      float* pb = pa + nout;
      if constexpr (ACCUM) { *pa += a; *pb += b; }
      else { *pa = a; *pb = b; }
    } else {
      float2* p2 = reinterpret_cast<float2*>(dst + (long long)r * nlines + 2 * pg);
      if constexpr (ACCUM) { float2 o = *p2; o.x += a; o.y += b; *p2 = o; }
      else *p2 = make_float2(a, b);
    }
  };
  Fft<L, P, true, Lay>::run(pair, t, lds, tw, fl, ls);
}

// ------------------------------------------------------------------ pass B and its adjoint
//
// data: complex [h * rpf][M], rows (n2-1) rpf .. n2 rpf - 1 hold frequency row
// n2 (rpf = 1 for images; rpf > 1 for the rows of a volume's slices, which
// share their slice's ratio), in place.
// Forward: g[x'] = (1-t) f[i0] + t f[i0+1] with i0 = floor((x' Lp + M n2)/(2 n2)),
//          then G[m1] = sum_x' g[x'] e^{-i 2 pi m1 x'/M} over centred x', m1.
// Adjoint: dg[x'] = sum_m1 dG[m1] e^{+i 2 pi m1 x'/M}, then
//          dS[i] = (1-t_a) dg[x_a] + t_b dg[x_b] where x_a is the sample whose
//          i0 is i and x_b the one whose i0 is i-1 (at most one each, as the
//          sampling ratio 2 n2 / Lp is below 1).
template <int M, bool ADJ, int V>
__global__ void __launch_bounds__((RowCfg<M, V>::THREADS))
    k_row_nvmt(float2* __restrict__ data, int Lp, int h, int rpf, long long img_stride,
               const float2* __restrict__ tw) {
  using Cfg = RowCfg<M, V>;
  constexpr int P = Cfg::P, ROWS = Cfg::ROWS;
  using Lay = LayRow<ROWS, M>;
  __shared__ float2 lds[Lay::size(M)];

  const int tid = threadIdx.x;
  const int row = tid / P, t = tid % P;
  const int gr = blockIdx.x * ROWS + row;   // data row; frequency row n2 = gr / rpf + 1
  const int n2 = gr / rpf + 1;
  const bool active = gr < h * rpf;
  float2* base = data + (long long)blockIdx.y * img_stride;

  for (int e = tid; e < ROWS * M; e += Cfg::THREADS) {
    const int rr = e / M, i = e % M;
    const int grr = blockIdx.x * ROWS + rr;
    float2 v = make_float2(0.f, 0.f);
    if (grr < h * rpf) v = base[(long long)grr * M + i];
    if (ADJ && (i & 1)) v = make_float2(-v.x, -v.y);
    lds[Lay::addr(rr, i)] = v;
  }
  __syncthreads();

  const int den = 2 * n2;
  const int mn2 = M * n2;
  const float rden = 1.0f / (float)den, rlp = 1.0f / (float)Lp;
  if constexpr (!ADJ) {
    auto fl = [&](int q) -> float2 {
      const int num = (q - M / 2) * Lp + mn2;
      const int i0 = floor_div_rcp(num, den, rden);
      const float tt = (float)(num - i0 * den) * rden;
      float2 f0 = make_float2(0.f, 0.f), f1 = make_float2(0.f, 0.f);
      if (i0 >= 0 && i0 < M) f0 = lds[Lay::addr(row, i0)];
      if (i0 + 1 >= 0 && i0 + 1 < M) f1 = lds[Lay::addr(row, i0 + 1)];
      const float s = (q & 1) ? -1.f : 1.f;
      return make_float2(s * ((1.f - tt) * f0.x + tt * f1.x), s * ((1.f - tt) * f0.y + tt * f1.y));
    };
    auto ls = [&](int p, float2 v) {
      if (!active) return;
      if ((p + M / 2) & 1) v = make_float2(-v.x, -v.y);
      base[(long long)gr * M + p] = v;
    };
    Fft<M, P, false, Lay>::run(row, t, lds, tw, fl, ls);
  } else {
    auto fl = [&](int p) -> float2 { return lds[Lay::addr(row, p)]; };
    auto ls = [&](int q, float2 v) {
      if ((q + M / 2) & 1) v = make_float2(-v.x, -v.y);
      lds[Lay::addr(row, q)] = v;
    };
    Fft<M, P, true, Lay>::run(row, t, lds, tw, fl, ls);
    __syncthreads();
    if (!active) return;
    for (int i = t; i < M; i += P) {
      float2 acc = make_float2(0.f, 0.f);
      // sample with i0 == i
      const int xa = ceil_div_rcp(i * den - mn2, Lp, rlp);
      const int na = xa * Lp + mn2;
      if (xa >= -M / 2 && xa < M / 2 && na < (i + 1) * den) {
        const float w = 1.f - (float)(na - i * den) * rden;
        const float2 g = lds[Lay::addr(row, xa + M / 2)];
        acc.x += w * g.x;
        acc.y += w * g.y;
      }
      // sample with i0 == i-1
      const int xb = ceil_div_rcp((i - 1) * den - mn2, Lp, rlp);
      const int nb = xb * Lp + mn2;
      if (xb >= -M / 2 && xb < M / 2 && nb < i * den) {
        const float w = (float)(nb - (i - 1) * den) * rden;
        const float2 g = lds[Lay::addr(row, xb + M / 2)];
        acc.x += w * g.x;
        acc.y += w * g.y;
      }
      base[(long long)gr * M + i] = acc;
    }
  }
}

// ------------------------------------------------------------------ register-resident column passes
//
// Lengths 128 .. 4096.  Each thread keeps about E elements of one transform in
// registers (P threads per transform), LINES column pairs per transform group,
// real and imaginary parts exchanged separately through a float LDS buffer.
// The R2C kernel keeps each output k and its mirror L-k in one thread, so the
// two real columns are separated in registers and written straight to HBM;
// the C2R kernel builds its Hermitian input the same way from one read of
// each stored coefficient.
//
// NT > 1: a block owns NT adjacent groups of LINES pairs.  It issues the loads
// of all groups first and then transforms and stores them one after the other
// through the same LDS buffer, so the later groups' loads are in flight during
// the first transform and the first group's stores drain during the later
// ones (the LDS barriers do not wait for global memory).  The row segments in
// HBM are NT * LINES pairs wide.

template <int L, int E_, int LINES_, int NT_ = 1>
struct FastCfg {
  static constexpr int NT = NT_;
  static constexpr int LINES = LINES_;
  static constexpr bool POW2 = (L & (L - 1)) == 0;
  // threads per transform: L / E for powers of two, ceil(L / E) otherwise
  static constexpr int P = POW2 ? (L / E_ > 0 ? L / E_ : 1) : cdiv(L, E_);
  static constexpr int THREADS = LINES * P;
  static constexpr int rmin() {
    const RadixPlan p = radix_plan(L);
    int m = 1 << 30;
    for (int i = 0; i < p.n; ++i) m = p.r[i] < m ? p.r[i] : m;
    return m;
  }
  static constexpr int em() {
    const int a = FftR<L, P, false, false>::EM, b = FftR<L, P, true, true>::EM;
    return a > b ? a : b;
  }
  // registers per thread (the larger of the forward and the reversed engine)
  static constexpr int E = em();
  static constexpr bool pow2_ok() {
    // every pass divides evenly and the paired pass (smallest radix) has an
    // even number of butterflies per thread
    return L % E_ == 0 && E_ % rmin() == 0 && (E_ / rmin()) % 2 == 0;
  }
  static constexpr bool mixed_ok() {
    // the paired pass (the last radix of the forward order, the first of the
    // reversed one) pairs butterflies j and NB - j, so NB must be even; at
    // most 1.5 E_ registers of data per thread
    const RadixPlan p = radix_plan(L);
    return p.n > 0 && (L / p.r[p.n - 1]) % 2 == 0 && em() * 2 <= 3 * E_ && P >= 2;
  }
  static constexpr bool valid = (L >= 128) && L <= 4096 && (POW2 ? pow2_ok() : mixed_ok()) && THREADS >= 64 &&
                                THREADS <= 1024 && (L + L / 16 + 1) * LINES * 4 <= 150 * 1024 &&
                                (NT == 1 || em() * NT <= 2 * E_);
};

// column-pass variants: (elements per thread, column pairs per group, groups per block)
#define FUNNEL_COL_VARIANTS(X) \
  X(0, 16, 4, 1) X(1, 16, 8, 1) X(2, 16, 16, 1) X(3, 32, 4, 1) X(4, 32, 8, 1) X(5, 32, 16, 1) X(6, 16, 8, 2) X(7, 16, 4, 2)
constexpr int kColVariants = 8;   // register tiles 0-7; 8-10 are the LDS-resident tiles

// Raw buffer access: 32-bit byte offsets from a per-block base, and hardware
// range checking (offsets at or beyond `bytes`, including negative offsets,
// read 0 and drop stores), which replaces per-element bounds tests and
// 64-bit address arithmetic in the column kernels.
//
// LD and ST are the cache-policy bits of the loads and the stores (0, or kNT:
// the non-temporal hint, the line is among the first to be evicted).
constexpr int kNT = 2;
template <int LD = 0, int ST = 0>
struct GBufT {
  __amdgpu_buffer_rsrc_t r;
  __device__ GBufT(const void* base, long long bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                            (int)(bytes < 0x7fffffffll ? bytes : 0x7fffffffll), 0x00020000)) {}
  // (values move through vector registers component by component: a bit_cast
  // to HIP's float2/float4 structs would go through scratch memory)
  __device__ __forceinline__ float ld1(int off) const {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, LD));
  }
  __device__ __forceinline__ float2 ld2(int off) const {
    const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, LD);
    return make_float2(__uint_as_float(u[0]), __uint_as_float(u[1]));
  }
  __device__ __forceinline__ float4 ld4(int off) const {
    const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, LD);
    return make_float4(__uint_as_float(u[0]), __uint_as_float(u[1]), __uint_as_float(u[2]), __uint_as_float(u[3]));
  }
  __device__ __forceinline__ void st1(float v, int off) const {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, ST);
  }
  __device__ __forceinline__ void st2(float2 v, int off) const {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const u2 u = {__float_as_uint(v.x), __float_as_uint(v.y)};
    __builtin_amdgcn_raw_buffer_store_b64(u, r, off, 0, ST);
  }
  __device__ __forceinline__ void st4(float4 v, int off) const {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4 u = {__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z), __float_as_uint(v.w)};
    __builtin_amdgcn_raw_buffer_store_b128(u, r, off, 0, ST);
  }
};

using GBuf = GBufT<>;

__device__ __forceinline__ float2 sel2(bool c, float2 a, float2 b) {
  return make_float2(c ? a.x : b.x, c ? a.y : b.y);
}

// Pass A output for frequency row k of column pair pg, from Z_k and Z_{L-k}
// of the pair's complex transform: A = (Z_k + conj Z_{L-k})/2 and
// B = (Z_k - conj Z_{L-k})/(2i), times scale (-1)^k.  Rows outside 1 .. H fall
// outside the buffer and are dropped.
template <class Buf>
__device__ __forceinline__ void emit_pair(Buf dst, int k, float2 zk, float2 zm, float scale, int npairs, int pg) {
  const float sc = (k & 1) ? -0.5f * scale : 0.5f * scale;
  const float ux = zk.x - zm.x, uy = zk.y + zm.y;
  dst.st4(make_float4(sc * (zk.x + zm.x), sc * (zk.y - zm.y), sc * uy, -sc * ux), ((k - 1) * npairs + pg) * 16);
}

__device__ __forceinline__ float2 herm_direct(float4 x) { return make_float2(x.x - x.w, x.y + x.z); }  // A + iB
__device__ __forceinline__ float2 herm_mirror(float4 x) { return make_float2(x.x + x.w, x.z - x.y); }  // conj A + i conj B

// Slot s of the matrix-core engine's native layout (element idx of transform
// ln) from slot 0's, by a compile-time offset where the engine's layout
// checks allow it (OUT: the last pass's outputs, else the first's inputs).
template <class Eng, bool OUT>
__device__ __forceinline__ void native_slot(int tid, int s, int ln0, int idx0, int& ln, int& idx) {
  constexpr bool LIN = OUT ? Eng::kNativeOutLin : Eng::kNativeInLin;
  if constexpr (LIN) {
    ln = ln0;
    idx = idx0 + (OUT ? Eng::kNativeOutOff.k[s] : Eng::kNativeInOff.k[s]);
  } else if constexpr (OUT) {
    Eng::native_out(tid, s, ln, idx);
  } else {
    Eng::native_in(tid, s, ln, idx);
  }
}

// The column passes as tile functions: column tile `tile` (NT groups of
// LINES column pairs) of image `img`, computed by threads tid = 0 ..
// Cfg::THREADS-1 of a block with the LDS buffer `lds` of
// LayInterR<LINES>::size(L) floats.  Threads of a larger block past THREADS
// pass live = false: they keep every barrier and touch no memory.  The
// kernels below run one tile per block; the work-queue kernels of ragged
// batches (funnel_queue.hip) run many tiles of several lengths per block.
template <int L, int E_, int LINES_, int NT, bool TRANS, int PREC>
__device__ __forceinline__ void r2c_tile(const float* __restrict__ in, float2* __restrict__ out, int nlines, int lin,
                                         int off, ImgMap map, float scale, const float2* __restrict__ tw, int tile,
                                         int img, int tid, bool live, float* lds) {
  using Cfg = FastCfg<L, E_, LINES_, NT>;
  constexpr int P = Cfg::P, LINES = Cfg::LINES, H = L / 2 - 1;
  using Eng = typename EngSel<PREC, L, P, false, false, LINES, true>::type;
  constexpr int E = Eng::EM;
  constexpr RadixPlan PL = Eng::kPlan;
  constexpr int LAST = PL.n - 1;
  constexpr int R0 = PL.r[0], NB0 = L / R0, BPT0 = Eng::template bpt<0, false>();
  constexpr int RL = PL.r[LAST], NBL = L / RL, BPTL = Eng::template bpt<LAST, true>();
  using Lay = LayInterR<LINES>;

  const int npairs = nlines >> 1;
  const int pair = live ? tid % LINES : 0, t = live ? tid / LINES : 0;
  // one image's lin x nlines block (rows of the padded frame off .. off+lin-1);
  // non-temporal loads where each load instruction reads whole 128-byte lines
  // (FP32 lane layout, one group of at least 16 pairs, not transposed): no
  // other tile reads them.  Where a line is split between groups or tiles,
  // the hint would evict it before its second reader.
  constexpr int kLd = (PREC == kPrecFP32 && !TRANS && NT == 1 && LINES * 8 >= 128) ? kNT : 0;
  const GBufT<kLd, 0> src(in + map.in(img), (long long)lin * nlines * 4);

  float2 v[NT][E];
  if constexpr (PREC != kPrecFP32) {
    // the matrix-core engine's own layout: slot s holds element idx of
    // transform (column pair) ln, so the loads skip its entry re-layout
    static_assert(NT == 1, "split-precision tiles hold one group");
    int ln0, idx0;
    Eng::native_in(tid, 0, ln0, idx0);
#pragma unroll
    for (int s2 = 0; s2 < E; ++s2) {
      int ln, idx;
      native_slot<Eng, false>(tid, s2, ln0, idx0, ln, idx);
      const int pg = tile * LINES + ln;
      const int rr = idx - off;
      float2 z = make_float2(0.f, 0.f);
      if constexpr (TRANS) {
        const int o = (2 * pg * lin + rr) * 4;
        if (pg < npairs && (unsigned)rr < (unsigned)lin) z = make_float2(src.ld1(o), src.ld1(o + lin * 4));
      } else {
        // rows outside [0, lin) fall outside the buffer and read 0
        if (pg < npairs) z = src.ld2((rr * nlines + 2 * pg) * 4);
      }
      v[0][s2] = z;
    }
  } else {
#pragma unroll
    for (int g = 0; g < NT; ++g) {
      const int pg = (tile * NT + g) * LINES + pair;
      const bool active = pg < npairs;
      if constexpr (TRANS) {
        // line 2pg and 2pg+1 of the image rows; rows outside [0, lin) are zero
        const int o0 = (2 * pg * lin + t - off) * 4;
#pragma unroll
        for (int b = 0; b < BPT0; ++b)
#pragma unroll
          for (int r = 0; r < R0; ++r) {
            const int rr = t + P * b + r * NB0 - off;
            const int o = o0 + (P * b + r * NB0) * 4;
            float2 z = make_float2(0.f, 0.f);
            if (active && Eng::template ok<0, false>(t, b) && (unsigned)rr < (unsigned)lin)
              z = make_float2(src.ld1(o), src.ld1(o + lin * 4));
            v[g][b * R0 + r] = z;
          }
      } else {
        // columns 2pg, 2pg+1; rows outside [0, lin) fall outside the buffer and read 0
        const int o0 = ((t - off) * nlines + 2 * pg) * 4;
        const int rs = nlines * 4;
#pragma unroll
        for (int b = 0; b < BPT0; ++b)
#pragma unroll
          for (int r = 0; r < R0; ++r)
            v[g][b * R0 + r] = Eng::template ok<0, false>(t, b) ? src.ld2(o0 + (P * b + r * NB0) * rs)
                                                                : make_float2(0.f, 0.f);
      }
    }
  }

  // half-spectrum rows 1 .. H: rows k outside that range fall outside the buffer
  const GBuf dst(out + map.out(img), (long long)H * npairs * 16);
#pragma unroll
  for (int g = 0; g < NT; ++g) {
    if constexpr (PREC != kPrecFP32) Eng::template run_ex<true, false, false, true, true, Lay>(v[g], pair, t, lds, tw);
    else Eng::template run<false, true, true, Lay>(v[g], pair, t, lds, tw, live);
    const int pg = (tile * NT + g) * LINES + pair;
    if (!live || pg >= npairs) continue;
#pragma unroll
    for (int c = 0; c < BPTL / 2; ++c) {
      if (!Eng::template ok<LAST, true>(t, 2 * c)) continue;
      const int ja = t + P * c;
      const bool zero = ja == 0;
      const int jb = zero ? NBL / 2 : NBL - ja;
      const float2* va = v[g] + (2 * c) * RL;
      const float2* vb = v[g] + (2 * c + 1) * RL;
#pragma unroll
      for (int q = 0; q < RL; ++q) {
        // partners chosen by value (a select of array elements would make the
        // compiler keep the arrays in scratch memory)
        const float2 pa = sel2(zero, va[(RL - q) % RL], vb[RL - 1 - q]);
        const float2 pb = sel2(zero, vb[RL - 1 - q], va[RL - 1 - q]);
        emit_pair(dst, ja + q * NBL, va[q], pa, scale, npairs, pg);
        emit_pair(dst, jb + q * NBL, vb[q], pb, scale, npairs, pg);
      }
    }
  }
}

// One column tile per block on a 1D grid of `total` = tiles x images blocks;
// consecutive tiles map to one XCD (xcd_remap).
template <int L, int E_, int LINES_, int NT, bool TRANS, int PREC>
__global__ void __launch_bounds__((FastCfg<L, E_, LINES_, NT>::THREADS))
    k_r2c_fast(const float* __restrict__ in, float2* __restrict__ out, int nlines, int lin, int off,
               ImgMap map, float scale, const float2* __restrict__ tw, int tiles, int total) {
  __shared__ float lds[LayInterR<FastCfg<L, E_, LINES_, NT>::LINES>::size(L)];
  const int logical = xcd_remap(blockIdx.x, total);
  r2c_tile<L, E_, LINES_, NT, TRANS, PREC>(in, out, nlines, lin, off, map, scale, tw, logical % tiles,
                                           logical / tiles, threadIdx.x, true, lds);
}

template <int L, int E_, int LINES_, int NT, bool TRANS, bool ACCUM, int PREC>
__device__ __forceinline__ void c2r_tile(const float2* __restrict__ in, float* __restrict__ out, int nlines, int r0,
                                         int nout, ImgMap map, float scale, const float2* __restrict__ tw, int tile,
                                         int img, int tid, bool live, float* lds) {
  using Cfg = FastCfg<L, E_, LINES_, NT>;
  constexpr int P = Cfg::P, LINES = Cfg::LINES;
  using Eng = typename EngSel<PREC, L, P, true, true, LINES, true>::type;
  constexpr int E = Eng::EM;
  constexpr RadixPlan PL = Eng::kPlan;
  constexpr int LAST = PL.n - 1;
  constexpr int R0 = PL.r[0], NB0 = L / R0, BPT0 = Eng::template bpt<0, true>();
  constexpr int RL = PL.r[LAST], NBL = L / RL, BPTL = Eng::template bpt<LAST, false>();
  using Lay = LayInterR<LINES>;

  const int npairs = nlines >> 1;
  const int pair = live ? tid % LINES : 0, t = live ? tid / LINES : 0;
  // half-spectrum rows 1 .. L/2-1; row 0 (and anything outside) reads 0.
  // Cache policy as in the column R2C: non-temporal loads of the spectrum
  // (read in the paired layout at every precision) where each load
  // instruction covers whole 128-byte lines.  With the FP32 engine's output
  // layout also non-temporal reads of an accumulated output under the same
  // rule, and non-temporal stores of the image gradient (the transposed
  // output and the accumulated one: no later pass reads it); from the
  // matrix-core engine's layout the hint on those stores is measured slower.
  constexpr bool kF32 = PREC == kPrecFP32;
  constexpr int kLd = (!TRANS && NT == 1 && LINES * 16 >= 128) ? kNT : 0;
  constexpr int kLdAcc = (kF32 && !TRANS && NT == 1 && LINES * 8 >= 128) ? kNT : 0;
  constexpr int kSt = (kF32 && (TRANS || ACCUM)) ? kNT : 0;
  const GBufT<kLd, 0> src(in + map.in(img), (long long)(L / 2 - 1) * npairs * 16);

  // Butterfly ja reads inputs ja + r NB0.  Below L/2 (r < NA) they are stored
  // coefficients; above, the mirror L - idx = jb + (R0-1-r) NB0 is one of
  // jb's stored coefficients, and jb (r < NBH stored) likewise mirrors ja's.
  // For ja = 0 the butterflies 0 and NB0/2 are their own partners; index 0
  // (DC, read as 0 from outside the buffer) and L/2 (Nyquist) are zero.
  constexpr int NA = (R0 + 1) / 2, NBH = R0 / 2;
  float2 v[NT][E];
#pragma unroll
  for (int g = 0; g < NT; ++g) {
    const int pg = (tile * NT + g) * LINES + pair;
    auto load = [src, npairs, pg](int k) -> float4 {  // coefficient k (1 .. L/2-1) times (-1)^k; 0 for k = 0
      float4 x = src.ld4(((k - 1) * npairs + pg) * 16);
      if (k & 1) x = make_float4(-x.x, -x.y, -x.z, -x.w);
      return x;
    };
#pragma unroll
    for (int s2 = 0; s2 < E; ++s2) v[g][s2] = make_float2(0.f, 0.f);
#pragma unroll
    for (int c = 0; c < BPT0 / 2; ++c) {
      if (!Eng::template ok<0, true>(t, 2 * c)) continue;
      const int ja = t + P * c;
      const bool zero = ja == 0;
      const int jb = zero ? NB0 / 2 : NB0 - ja;
      float4 xa[NA], xb[NBH > 0 ? NBH : 1];
#pragma unroll
      for (int r = 0; r < NA; ++r) xa[r] = load(ja + r * NB0);
#pragma unroll
      for (int r = 0; r < NBH; ++r) xb[r] = load(jb + r * NB0);
      float2* va = v[g] + (2 * c) * R0;
      float2* vb = v[g] + (2 * c + 1) * R0;
      if (!zero) {
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          va[r] = r < NA ? herm_direct(xa[r]) : herm_mirror(xb[R0 - 1 - r]);
          vb[r] = r < NBH ? herm_direct(xb[r]) : herm_mirror(xa[R0 - 1 - r]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          // butterfly 0: inputs r NB0 (mirror (R0 - r) NB0); Nyquist at r = R0/2 for even R0
          if (r < NA) va[r] = herm_direct(xa[r]);
          else if (2 * r == R0) va[r] = make_float2(0.f, 0.f);
          else va[r] = herm_mirror(xa[R0 - r]);
          // butterfly NB0/2: inputs NB0/2 + r NB0 (mirror (R0-1-r)); Nyquist at r = (R0-1)/2 for odd R0
          if (r < NBH) vb[r] = herm_direct(xb[r]);
          else if (2 * r + 1 == R0) vb[r] = make_float2(0.f, 0.f);
          else vb[r] = herm_mirror(xb[R0 - 1 - r]);
        }
      }
    }
  }

  // one image's nout x nlines block (or nlines x nout, transposed)
  const GBufT<kLdAcc, kSt> dst(out + map.out(img), (long long)nout * nlines * 4);
  const int step = TRANS ? 4 : nlines * 4;
#pragma unroll
  for (int g = 0; g < NT; ++g) {
    if constexpr (PREC != kPrecFP32) {
      // stores from the matrix-core engine's own layout (no exit re-layout):
      // slot s holds output row idx of column pair ln
      static_assert(NT == 1, "split-precision tiles hold one group");
      Eng::template run_ex<false, true, true, false, true, Lay>(v[0], pair, t, lds, tw);
      const int ntid = Eng::opaque();
      int ln0, idx0;
      Eng::native_out(ntid, 0, ln0, idx0);
      // byte offset of slot s2's output (the first of its two values), and
      // whether the slot stores at all
      auto where = [&](int s2, int& o, bool& st) {
        int ln, idx;
        native_slot<Eng, true>(ntid, s2, ln0, idx0, ln, idx);
        const int pgs = tile * LINES + ln, r = idx - r0;
        if constexpr (TRANS) {
          o = (2 * pgs * nout + r) * 4;
          st = pgs < npairs && r >= 0 && r < nout;
        } else {
          o = (r * nlines + 2 * pgs) * 4;   // rows outside [0, nout) fall outside the buffer
          st = pgs < npairs;
        }
      };
      auto put = [&](int s2, float2 old) {
        int o;
        bool st;
        where(s2, o, st);
        if (!st) return;
        float a = scale * v[0][s2].x, bb = scale * v[0][s2].y;
        if constexpr (ACCUM) {
          a += old.x;
          bb += old.y;
        }
        if constexpr (TRANS) {
          dst.st1(a, o);
          dst.st1(bb, o + nout * 4);
        } else {
          dst.st2(make_float2(a, bb), o);
        }
      };
      if constexpr (ACCUM) {
        // read-modify-write CH slots at a time, the next CH slots' old values
        // read before this chunk's stores so that they are in flight together
        // (every slot is a different output, so the reordering is safe)
        constexpr int CH = 4;
        static_assert(E % CH == 0, "whole chunks");
        auto fetch = [&](int c, float2 (&o2)[CH]) {
#pragma unroll
          for (int k = 0; k < CH; ++k) {
            int o;
            bool st;
            where(c * CH + k, o, st);
            if constexpr (TRANS) o2[k] = st ? make_float2(dst.ld1(o), dst.ld1(o + nout * 4)) : make_float2(0.f, 0.f);
            else o2[k] = st ? dst.ld2(o) : make_float2(0.f, 0.f);
          }
        };
        float2 cur[CH], nxt[CH];
        fetch(0, cur);
#pragma unroll
        for (int c = 0; c < E / CH; ++c) {
          if (c + 1 < E / CH) fetch(c + 1, nxt);
#pragma unroll
          for (int k = 0; k < CH; ++k) put(c * CH + k, cur[k]);
#pragma unroll
          for (int k = 0; k < CH; ++k) cur[k] = nxt[k];
        }
      } else {
#pragma unroll
        for (int s2 = 0; s2 < E; ++s2) put(s2, make_float2(0.f, 0.f));
      }
      continue;
    } else {
      Eng::template run<true, false, true, Lay>(v[g], pair, t, lds, tw, live);
    }
    const int pg = (tile * NT + g) * LINES + pair;
    if (!live || pg >= npairs) continue;
    // output row r = t + P b + q NBL - r0: offsets at o0 + (P b + q NBL) * step
    const int o0 = TRANS ? (2 * pg * nout + t - r0) * 4 : ((t - r0) * nlines + 2 * pg) * 4;
    if constexpr (ACCUM) {
      // read-modify-write, one butterfly slot (RL outputs) at a time with the
      // next slot's old values already in flight: two slots of registers
      // instead of all E, so the wide tiles fit in registers.  The slot's
      // base offset passes through an empty asm after the previous slot's
      // stores, so the compiler cannot hoist every load to the front.
      float2 old[2][RL];
      auto fetch = [&](int b, float2 (&o)[RL]) {
        int base = o0 + P * b * step;
        asm volatile("" : "+v"(base));
#pragma unroll
        for (int q = 0; q < RL; ++q) {
          const int ofs = base + q * NBL * step;
          if constexpr (TRANS) o[q] = make_float2(dst.ld1(ofs), dst.ld1(ofs + nout * 4));
          else o[q] = dst.ld2(ofs);
        }
      };
      fetch(0, old[0]);
#pragma unroll
      for (int b = 0; b < BPTL; ++b) {
        if (b + 1 < BPTL) fetch(b + 1, old[(b + 1) & 1]);
        if (!Eng::template ok<LAST, false>(t, b)) continue;
#pragma unroll
        for (int q = 0; q < RL; ++q) {
          const int r = t + P * b + q * NBL - r0;
          const int o = o0 + (P * b + q * NBL) * step;
          const float a = scale * v[g][b * RL + q].x + old[b & 1][q].x;
          const float bb = scale * v[g][b * RL + q].y + old[b & 1][q].y;
          if constexpr (TRANS) {
            if (r < 0 || r >= nout) continue;
            dst.st1(a, o);
            dst.st1(bb, o + nout * 4);
          } else {
            dst.st2(make_float2(a, bb), o);
          }
        }
      }
      continue;
    }
#pragma unroll
    for (int b = 0; b < BPTL; ++b) {
      if (!Eng::template ok<LAST, false>(t, b)) continue;
#pragma unroll
      for (int q = 0; q < RL; ++q) {
        const int r = t + P * b + q * NBL - r0;
        const int o = o0 + (P * b + q * NBL) * step;
        const float a = scale * v[g][b * RL + q].x, bb = scale * v[g][b * RL + q].y;
        if constexpr (TRANS) {
          // rows outside [0, nout) would land in the neighbouring line
          if (r < 0 || r >= nout) continue;
          dst.st1(a, o);
          dst.st1(bb, o + nout * 4);
        } else {
          dst.st2(make_float2(a, bb), o);   // rows outside [0, nout) fall outside the buffer
        }
      }
    }
  }
}

template <int L, int E_, int LINES_, int NT, bool TRANS, bool ACCUM, int PREC>
__global__ void __launch_bounds__((FastCfg<L, E_, LINES_, NT>::THREADS))
    k_c2r_fast(const float2* __restrict__ in, float* __restrict__ out, int nlines, int r0, int nout,
               ImgMap map, float scale, const float2* __restrict__ tw, int tiles, int total) {
  __shared__ float lds[LayInterR<FastCfg<L, E_, LINES_, NT>::LINES>::size(L)];
  const int logical = xcd_remap(blockIdx.x, total);
  c2r_tile<L, E_, LINES_, NT, TRANS, ACCUM, PREC>(in, out, nlines, r0, nout, map, scale, tw, logical % tiles,
                                                  logical / tiles, threadIdx.x, true, lds);
}

// ------------------------------------------------------------------ register-resident row pass
//
// Power-of-two row lengths >= 64: 16 elements per thread, ROWS rows per block.
// The whole row is staged in LDS with 16-byte loads issued before any use;
// the NVMT gather feeds the first butterfly pass directly from that copy.

template <int M, int E_, int TPB>
struct RowFastCfg {
  static constexpr bool POW2 = (M & (M - 1)) == 0;
  static constexpr int P = POW2 ? (M / E_ > 0 ? M / E_ : 1) : cdiv(M, E_);
  static constexpr int ROWS = TPB / P > 0 ? TPB / P : 1;
  static constexpr int THREADS = ROWS * P;
  static constexpr int E = FftR<M, P, false, false>::EM;   // registers per thread
  static constexpr bool valid = (M >= 64) && M <= 4096 && radix_plan(M).n > 0 && P >= 2 &&
                                (POW2 ? (M % E_ == 0 && (M / 16) % P == 0) : E * 2 <= 3 * E_) &&
                                THREADS <= 1024 && THREADS >= 32 && (M + M / 16 + 1) * ROWS * 8 <= 64 * 1024;
};

// row-pass variants: (elements per thread, target threads per block)
#define FUNNEL_ROW_VARIANTS(X) X(0, 16, 256) X(1, 16, 128) X(2, 16, 512) X(3, 32, 256)
constexpr int kRowVariants = 4;

// the row tile runs the matrix-core engine in its own layout on both sides
template <class Eng, int PREC>
constexpr bool native_rows() {
  if constexpr (PREC == kPrecFP32) return false;
  else return Eng::kLaneOneLine;
}

// Rows blk * ROWS .. blk * ROWS + ROWS-1 of image img, by threads tid = 0 ..
// THREADS-1 with the LDS buffer `lds` of LayRow<ROWS, M>::size(M) float2
// (threads past THREADS of a larger block pass live = false, as for the
// column tiles).
template <int M, int E_, int TPB, bool ADJ, int PREC>
__device__ __forceinline__ void row_tile(float2* __restrict__ data, int Lp, int h, int rpf, long long img_stride,
                                         const float2* __restrict__ tw, int blk, int img, int tid, bool live,
                                         float2* lds) {
  using Cfg = RowFastCfg<M, E_, TPB>;
  constexpr int P = Cfg::P, ROWS = Cfg::ROWS;
  using Eng = typename EngSel<PREC, M, P, ADJ, false, ROWS, false>::type;
  constexpr int E = Eng::EM;
  constexpr RadixPlan PL = Eng::kPlan;
  constexpr int LAST = PL.n - 1;
  constexpr int R0 = PL.r[0], NB0 = M / R0, BPT0 = Eng::template bpt<0, false>();
  constexpr int RL = PL.r[LAST], NBL = M / RL, BPTL = Eng::template bpt<LAST, false>();
  constexpr int ES = cdiv(M / 2, P);   // float4 (two elements) per thread when staging the row
  constexpr int EG = cdiv(M, P);       // elements per thread in the transposed gather
  using Lay = LayRow<ROWS, M>;

  const int row = live ? tid / P : 0, t = live ? tid % P : 0;
  const int gr = blk * ROWS + row;   // data row; frequency row n2 = gr / rpf + 1
  const int n2 = gr / rpf + 1;
  const bool active = live && gr < h * rpf;
  float2* rowp = data + (long long)img * img_stride + (long long)gr * M;

  {  // stage this thread's share of its row: ES float4 loads, all in flight
    float4 st[ES];
    const float4* src4 = reinterpret_cast<const float4*>(rowp);
#pragma unroll
    for (int i = 0; i < ES; ++i)
      st[i] = active && ((M / 2) % P == 0 || t + P * i < M / 2) ? src4[t + P * i] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int i = 0; i < ES; ++i) {
      if (!live || ((M / 2) % P != 0 && t + P * i >= M / 2)) continue;
      const int e0 = 2 * (t + P * i);
      float4 x = st[i];
      if (ADJ) { x.z = -x.z; x.w = -x.w; }   // (-1)^p on the odd element
      lds[Lay::addr(row, e0)] = make_float2(x.x, x.y);
      lds[Lay::addr(row, e0 + 1)] = make_float2(x.z, x.w);
    }
  }
  __syncthreads();

  const int den = 2 * n2;
  const int mn2 = M * n2;
  const float rden = 1.0f / (float)den, rlp = 1.0f / (float)Lp;
  float2 v[E];
#pragma unroll
  for (int s2 = 0; s2 < E; ++s2) v[s2] = make_float2(0.f, 0.f);
  if constexpr (native_rows<Eng, PREC>()) {
    // The matrix-core engine in its own layout on both sides: the gather
    // (forward) or the staged row (adjoint) feeds slot s with element idx of
    // the lane's row directly, and the outputs leave from the same layout,
    // so no re-layout through LDS on entry or exit.  Every slot of a lane
    // lies in one row (kLaneOneLine).
    int lr, i00;
    Eng::native_in(tid, 0, lr, i00);
    const int grl = blk * ROWS + lr, n2l = grl / rpf + 1;
    const bool act = grl < h * rpf;
    float2* rowl = data + (long long)img * img_stride + (long long)grl * M;
    const int denl = 2 * n2l, mnl = M * n2l;
    const float rdl = 1.0f / (float)denl;
    if constexpr (!ADJ) {
#pragma unroll
      for (int s2 = 0; s2 < E; ++s2) {
        int ln, q;
        native_slot<Eng, false>(tid, s2, lr, i00, ln, q);
        const int num = (q - M / 2) * Lp + mnl;
        const int i0 = floor_div_rcp(num, denl, rdl);
        const float tt = (float)(num - i0 * denl) * rdl;
        float2 f0 = make_float2(0.f, 0.f), f1 = make_float2(0.f, 0.f);
        if (i0 >= 0 && i0 < M) f0 = lds[Lay::addr(lr, i0)];
        if (i0 + 1 >= 0 && i0 + 1 < M) f1 = lds[Lay::addr(lr, i0 + 1)];
        const float sg = (q & 1) ? -1.f : 1.f;
        v[s2] = make_float2(sg * ((1.f - tt) * f0.x + tt * f1.x), sg * ((1.f - tt) * f0.y + tt * f1.y));
      }
      Eng::template run_ex<true, true, false, false, false, Lay>(v, row, t, lds, tw);
      if (!act) return;
      const int ntid = Eng::opaque();
      int lo0, po0;
      Eng::native_out(ntid, 0, lo0, po0);
#pragma unroll
      for (int s2 = 0; s2 < E; ++s2) {
        int ln, p;
        native_slot<Eng, true>(ntid, s2, lo0, po0, ln, p);
        float2 g = v[s2];
        if ((p + M / 2) & 1) g = make_float2(-g.x, -g.y);
        rowl[p] = g;
      }
      return;
    } else {
#pragma unroll
      for (int s2 = 0; s2 < E; ++s2) {
        int ln, q;
        native_slot<Eng, false>(tid, s2, lr, i00, ln, q);
        v[s2] = lds[Lay::addr(lr, q)];
      }
      Eng::template run_ex<true, true, false, false, false, Lay>(v, row, t, lds, tw);
      __syncthreads();
      const int ntid = Eng::opaque();
      int lo0, xo0;
      Eng::native_out(ntid, 0, lo0, xo0);
#pragma unroll
      for (int s2 = 0; s2 < E; ++s2) {
        int ln, x;
        native_slot<Eng, true>(ntid, s2, lo0, xo0, ln, x);
        float2 g = v[s2];
        if ((x + M / 2) & 1) g = make_float2(-g.x, -g.y);
        lds[Lay::addr(lr, x)] = g;
      }
      __syncthreads();
      // (the transposed gather below reads each thread's own row)
    }
  } else if constexpr (!ADJ) {
#pragma unroll
    for (int b = 0; b < BPT0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        if (!Eng::template ok<0, false>(t, b)) continue;
        const int q = t + P * b + r * NB0;
        const int num = (q - M / 2) * Lp + mn2;
        const int i0 = floor_div_rcp(num, den, rden);
        const float tt = (float)(num - i0 * den) * rden;
        float2 f0 = make_float2(0.f, 0.f), f1 = make_float2(0.f, 0.f);
        if (i0 >= 0 && i0 < M) f0 = lds[Lay::addr(row, i0)];
        if (i0 + 1 >= 0 && i0 + 1 < M) f1 = lds[Lay::addr(row, i0 + 1)];
        const float sg = (q & 1) ? -1.f : 1.f;
        v[b * R0 + r] = make_float2(sg * ((1.f - tt) * f0.x + tt * f1.x), sg * ((1.f - tt) * f0.y + tt * f1.y));
      }
    Eng::template run<false, false, false, Lay>(v, row, t, lds, tw, live);
    if (!active) return;
#pragma unroll
    for (int b = 0; b < BPTL; ++b)
#pragma unroll
      for (int q = 0; q < RL; ++q) {
        if (!Eng::template ok<LAST, false>(t, b)) continue;
        const int p = t + P * b + q * NBL;
        float2 g = v[b * RL + q];
        if ((p + M / 2) & 1) g = make_float2(-g.x, -g.y);
        rowp[p] = g;
      }
  } else {
#pragma unroll
    for (int b = 0; b < BPT0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r)
        if (Eng::template ok<0, false>(t, b)) v[b * R0 + r] = lds[Lay::addr(row, t + P * b + r * NB0)];
    Eng::template run<false, false, false, Lay>(v, row, t, lds, tw, live);
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BPTL; ++b)
#pragma unroll
      for (int q = 0; q < RL; ++q) {
        if (!live || !Eng::template ok<LAST, false>(t, b)) continue;
        const int x = t + P * b + q * NBL;
        float2 g = v[b * RL + q];
        if ((x + M / 2) & 1) g = make_float2(-g.x, -g.y);
        lds[Lay::addr(row, x)] = g;
      }
    __syncthreads();
  }
  if constexpr (ADJ) {
    if (!active) return;
    // transposed interpolation as a gather: at most two samples land on i
#pragma unroll
    for (int e = 0; e < EG; ++e) {
      const int i = t + P * e;
      if (M % P != 0 && i >= M) continue;
      float2 acc = make_float2(0.f, 0.f);
      const int xa = ceil_div_rcp(i * den - mn2, Lp, rlp);
      const int na = xa * Lp + mn2;
      if (xa >= -M / 2 && xa < M / 2 && na < (i + 1) * den) {
        const float w = 1.f - (float)(na - i * den) * rden;
        const float2 g = lds[Lay::addr(row, xa + M / 2)];
        acc.x += w * g.x;
        acc.y += w * g.y;
      }
      const int xb = ceil_div_rcp((i - 1) * den - mn2, Lp, rlp);
      const int nb = xb * Lp + mn2;
      if (xb >= -M / 2 && xb < M / 2 && nb < i * den) {
        const float w = (float)(nb - (i - 1) * den) * rden;
        const float2 g = lds[Lay::addr(row, xb + M / 2)];
        acc.x += w * g.x;
        acc.y += w * g.y;
      }
      rowp[i] = acc;
    }
  }
}

template <int M, int E_, int TPB, bool ADJ, int PREC>
__global__ void __launch_bounds__((RowFastCfg<M, E_, TPB>::THREADS))
    k_row_fast(float2* __restrict__ data, int Lp, int h, int rpf, long long img_stride,
               const float2* __restrict__ tw) {
  using Cfg = RowFastCfg<M, E_, TPB>;
  __shared__ float2 lds[LayRow<Cfg::ROWS, M>::size(M)];
  row_tile<M, E_, TPB, ADJ, PREC>(data, Lp, h, rpf, img_stride, tw, blockIdx.x, blockIdx.y, threadIdx.x, true, lds);
}

// ------------------------------------------------------------------ launchers
//
// PREC = kPrecFP32 runs FftR; the split-precision values run FftM and exist
// only for the register-resident tile variants FftM fits.

template <int L, int PREC>
unsigned col_variant_mask_t() {
  unsigned m = 0;
#define FUNNEL_V(i, e, l, nt)                                                                             \
  if constexpr (FastCfg<L, e, l, nt>::valid && (PREC == kPrecFP32 || (nt == 1 && mfma_fits(L, e, FastCfg<L, e, l, nt>::THREADS)))) \
    m |= 1u << i;
  FUNNEL_COL_VARIANTS(FUNNEL_V)
#undef FUNNEL_V
  if (PREC != kPrecFP32) return m;
  // the LDS-resident variants, numbered from kColVariants
  m |= 1u << kColVariants;
  if constexpr (ColCfg<L, 1>::distinct()) m |= 1u << (kColVariants + 1);
  if constexpr (ColCfg<L, 2>::distinct()) m |= 1u << (kColVariants + 2);
  return m;
}

template <int M, int PREC>
unsigned row_variant_mask_t() {
  unsigned m = 0;
#define FUNNEL_V(i, e, t) \
  if constexpr (RowFastCfg<M, e, t>::valid && (PREC == kPrecFP32 || mfma_fits(M, e, RowFastCfg<M, e, t>::THREADS))) m |= 1u << i;
  FUNNEL_ROW_VARIANTS(FUNNEL_V)
#undef FUNNEL_V
  if (PREC != kPrecFP32) return m;
  // the LDS-resident variants, numbered from kRowVariants
  m |= 1u << kRowVariants;
  if constexpr (RowCfg<M, 1>::distinct()) m |= 1u << (kRowVariants + 1);
  return m;
}

template <int L, int PREC>
hipError_t launch_r2c_t(int variant, bool trans, const float* in, float2* out, int nlines, int lin, int off,
                        ImgMap map, float scale, const float2* tw, int batch, hipStream_t s) {
  switch (variant) {
#define FUNNEL_V(i, e, l, nt)                                                                                \
  case i:                                                                                                    \
    if constexpr (FastCfg<L, e, l, nt>::valid &&                                                             \
                  (PREC == kPrecFP32 || (nt == 1 && mfma_fits(L, e, FastCfg<L, e, l, nt>::THREADS)))) {                    \
      using F = FastCfg<L, e, l, nt>;                                                                        \
      const int tiles = (nlines / 2 + F::LINES * nt - 1) / (F::LINES * nt), total = tiles * batch;           \
      if (trans)                                                                                             \
        k_r2c_fast<L, e, l, nt, true, PREC><<<total, F::THREADS, 0, s>>>(in, out, nlines, lin, off, map, scale, tw, tiles, total); \
      else                                                                                                   \
        k_r2c_fast<L, e, l, nt, false, PREC><<<total, F::THREADS, 0, s>>>(in, out, nlines, lin, off, map, scale, tw, tiles, total); \
      return hipGetLastError();                                                                              \
    }                                                                                                        \
    break;
    FUNNEL_COL_VARIANTS(FUNNEL_V)
#undef FUNNEL_V
    default: break;
  }
  if constexpr (PREC != kPrecFP32) {
    return hipErrorInvalidValue;
  } else {
    const unsigned m = col_variant_mask_t<L, PREC>();
    if (variant < kColVariants || variant >= kColVariants + kGenVariants || !(m & (1u << variant)))
      return hipErrorInvalidValue;
    variant -= kColVariants;
    auto go = [&](auto vc) {
      constexpr int V = decltype(vc)::value;
      if constexpr (ColCfg<L, V>::distinct()) {
        using Cfg = ColCfg<L, V>;
        dim3 grid((nlines / 2 + Cfg::LINES - 1) / Cfg::LINES, batch), block(Cfg::THREADS);
        if (trans)
          k_r2c_half<L, true, V><<<grid, block, 0, s>>>(in, out, nlines, lin, off, map, scale, tw);
        else
          k_r2c_half<L, false, V><<<grid, block, 0, s>>>(in, out, nlines, lin, off, map, scale, tw);
      }
      return hipGetLastError();
    };
    if (variant == 0) return go(std::integral_constant<int, 0>());
    if (variant == 1) return go(std::integral_constant<int, 1>());
    return go(std::integral_constant<int, 2>());
  }
}

template <int L, int PREC>
hipError_t launch_c2r_t(int variant, bool trans, bool accum, const float2* in, float* out, int nlines, int r0,
                        int nout, ImgMap map, float scale, const float2* tw, int batch, hipStream_t s) {
  switch (variant) {
#define FUNNEL_V(i, e, l, nt)                                                                                \
  case i:                                                                                                    \
    if constexpr (FastCfg<L, e, l, nt>::valid &&                                                             \
                  (PREC == kPrecFP32 || (nt == 1 && mfma_fits(L, e, FastCfg<L, e, l, nt>::THREADS)))) {                    \
      using F = FastCfg<L, e, l, nt>;                                                                        \
      const int tiles = (nlines / 2 + F::LINES * nt - 1) / (F::LINES * nt), total = tiles * batch;           \
      auto go = [&](auto* k) {                                                                               \
        k<<<total, F::THREADS, 0, s>>>(in, out, nlines, r0, nout, map, scale, tw, tiles, total);              \
      };                                                                                                     \
      if (trans) {                                                                                           \
        if (accum) go(k_c2r_fast<L, e, l, nt, true, true, PREC>);                                      \
        else go(k_c2r_fast<L, e, l, nt, true, false, PREC>);                                           \
      } else {                                                                                               \
        if (accum) go(k_c2r_fast<L, e, l, nt, false, true, PREC>);                                     \
        else go(k_c2r_fast<L, e, l, nt, false, false, PREC>);                                          \
      }                                                                                                      \
      return hipGetLastError();                                                                              \
    }                                                                                                        \
    break;
    FUNNEL_COL_VARIANTS(FUNNEL_V)
#undef FUNNEL_V
    default: break;
  }
  if constexpr (PREC != kPrecFP32) {
    return hipErrorInvalidValue;
  } else {
    const unsigned m = col_variant_mask_t<L, PREC>();
    if (variant < kColVariants || variant >= kColVariants + kGenVariants || !(m & (1u << variant)))
      return hipErrorInvalidValue;
    variant -= kColVariants;
    auto go = [&](auto vc) {
      constexpr int V = decltype(vc)::value;
      if constexpr (ColCfg<L, V>::distinct()) {
        using Cfg = ColCfg<L, V>;
        dim3 grid((nlines / 2 + Cfg::LINES - 1) / Cfg::LINES, batch), block(Cfg::THREADS);
        if (trans) {
          if (accum)
            k_c2r_half<L, true, true, V><<<grid, block, 0, s>>>(in, out, nlines, r0, nout, map, scale, tw);
          else
            k_c2r_half<L, true, false, V><<<grid, block, 0, s>>>(in, out, nlines, r0, nout, map, scale, tw);
        } else {
          if (accum)
            k_c2r_half<L, false, true, V><<<grid, block, 0, s>>>(in, out, nlines, r0, nout, map, scale, tw);
          else
            k_c2r_half<L, false, false, V><<<grid, block, 0, s>>>(in, out, nlines, r0, nout, map, scale, tw);
        }
      }
      return hipGetLastError();
    };
    if (variant == 0) return go(std::integral_constant<int, 0>());
    if (variant == 1) return go(std::integral_constant<int, 1>());
    return go(std::integral_constant<int, 2>());
  }
}

template <int M, int PREC>
hipError_t launch_row_t(int variant, bool adj, float2* data, int Lp, int h, int rpf, long long img_stride,
                        const float2* tw, int batch, hipStream_t s) {
  switch (variant) {
#define FUNNEL_V(i, e, tpb)                                                                                    \
  case i:                                                                                                      \
    if constexpr (RowFastCfg<M, e, tpb>::valid &&                                                              \
                  (PREC == kPrecFP32 || mfma_fits(M, e, RowFastCfg<M, e, tpb>::THREADS))) {                    \
      using F = RowFastCfg<M, e, tpb>;                                                                         \
      dim3 grid((h * rpf + F::ROWS - 1) / F::ROWS, batch), block(F::THREADS);                                  \
      if (adj)                                                                                                 \
        k_row_fast<M, e, tpb, true, PREC><<<grid, block, 0, s>>>(data, Lp, h, rpf, img_stride, tw);            \
      else                                                                                                     \
        k_row_fast<M, e, tpb, false, PREC><<<grid, block, 0, s>>>(data, Lp, h, rpf, img_stride, tw);           \
      return hipGetLastError();                                                                                \
    }                                                                                                          \
    break;
    FUNNEL_ROW_VARIANTS(FUNNEL_V)
#undef FUNNEL_V
    default: break;
  }
  if constexpr (PREC != kPrecFP32) {
    return hipErrorInvalidValue;
  } else {
    const unsigned m = row_variant_mask_t<M, PREC>();
    if (variant < kRowVariants || variant >= kRowVariants + kGenRowVariants || !(m & (1u << variant)))
      return hipErrorInvalidValue;
    variant -= kRowVariants;
    auto go = [&](auto vc) {
      constexpr int V = decltype(vc)::value;
      if constexpr (RowCfg<M, V>::distinct()) {
        using Cfg = RowCfg<M, V>;
        dim3 grid((h * rpf + Cfg::ROWS - 1) / Cfg::ROWS, batch), block(Cfg::THREADS);
        if (adj)
          k_row_nvmt<M, true, V><<<grid, block, 0, s>>>(data, Lp, h, rpf, img_stride, tw);
        else
          k_row_nvmt<M, false, V><<<grid, block, 0, s>>>(data, Lp, h, rpf, img_stride, tw);
      }
      return hipGetLastError();
    };
    if (variant == 0) return go(std::integral_constant<int, 0>());
    return go(std::integral_constant<int, 1>());
  }
}

}  // namespace funnel
