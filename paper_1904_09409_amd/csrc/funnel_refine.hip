// funnel_refine.hip -- sub-cell refinement of detected peaks.
//
// Between cells the parameter plane is the last two steps of Sec. 3.1 with
// the x' DFT taken at a real slope bin m (the DTFT of each resampled row g)
// and the inverse y DFT at a real intercept y:
//   P(m, y) = (2/Np) Re sum_n2 A(n2; m) exp(+j 2 pi n2 y / Np),
//   A(n2; m) = sum_x' g[n2][x'] exp(-j 2 pi m x' / W),
// equal to the plane at integer (m, y).  Line parameters (Eqs. 22-25) read at
// its local maximum near a detected cell are continuous, which is where
// Eq. 19 focuses a line.  The rows g are the resampled spectrum rows: the
// row pass's linear interpolation alone (k_row_lerp), or for the chirp-z
// NVMT the inverse x' DFT of the G rows its row pass leaves in the
// workspace (k_row_idft).  Each iteration forms, for every
// peak, A and its first two m-derivatives over all rows (k_refine_dtft_mfma:
// a (rows x W) by (W x peaks) product per plane on the matrix cores), then
// reduces over n2 into P,
// its gradient and Hessian and takes one safeguarded Newton step
// (k_refine_step).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.hpp"
#include "funnel_internal.hpp"

namespace funnel {

// ------------------------------------------------------------------ rows G -> g
//
// g[x'] = (1/W) sum_m1 G[m1] exp(+j 2 pi m1 x' / W) over centred indices:
// with array indices p = m1 + W/2 and q = x' + W/2 this is
// (1/W) (-1)^(q + W/2) sum_p (-1)^p G[p] exp(+j 2 pi p q / W).
constexpr int kIdftThreads = 256;

template <int W>
__global__ void __launch_bounds__(kIdftThreads) k_row_idft(float2* __restrict__ data, int h, long long img_stride,
                                                           const float2* __restrict__ tw) {
  constexpr int P = W / 16;
  constexpr int ROWS = kIdftThreads / P;
  using Eng = FftR<W, P, true, false>;
  constexpr int E = Eng::EM;
  constexpr RadixPlan PL = Eng::kPlan;
  constexpr int LAST = PL.n - 1;
  constexpr int R0 = PL.r[0], NB0 = W / R0, BPT0 = Eng::template bpt<0, false>();
  constexpr int RL = PL.r[LAST], NBL = W / RL, BPTL = Eng::template bpt<LAST, false>();
  using Lay = LayRow<ROWS, W>;
  __shared__ float2 lds[Lay::size(W)];
  const int row = threadIdx.x / P, t = threadIdx.x % P;
  const int n2 = blockIdx.x * ROWS + row + 1;
  const bool active = n2 <= h;
  float2* rowp = data + (long long)blockIdx.y * img_stride + (long long)(active ? n2 - 1 : 0) * W;
  float2 v[E];
#pragma unroll
  for (int s = 0; s < E; ++s) v[s] = make_float2(0.f, 0.f);
#pragma unroll
  for (int b = 0; b < BPT0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int p = t + P * b + r * NB0;
      float2 x = active ? rowp[p] : make_float2(0.f, 0.f);
      if (p & 1) x = make_float2(-x.x, -x.y);
      v[b * R0 + r] = x;
    }
  Eng::template run<false, false, false, Lay>(v, row, t, lds, tw);
  if (!active) return;
  const float inv = 1.0f / (float)W;
#pragma unroll
  for (int b = 0; b < BPTL; ++b)
#pragma unroll
    for (int q2 = 0; q2 < RL; ++q2) {
      const int q = t + P * b + q2 * NBL;
      const float sg = ((q + W / 2) & 1) ? -inv : inv;
      rowp[q] = make_float2(sg * v[b * RL + q2].x, sg * v[b * RL + q2].y);
    }
}

// ------------------------------------------------------------------ rows S -> g
//
// With the linear NVMT the rows g are the row pass's interpolation itself:
// its DFT followed by the inverse above gives back g[q] = the interpolated
// sample at x' = q - W/2 exactly (up to rounding).  This gathers them
// straight from the spectrum rows S (same index algebra as the row pass:
// x = (x' Lp + W n2) / (2 n2) - W/2 on centred indices, zero outside the row),
// one block per row, in place through an LDS copy of the row.
constexpr int kLerpThreads = 256;

template <int W>
__global__ void __launch_bounds__(kLerpThreads) k_row_lerp(float2* __restrict__ data, int Lp, long long img_stride) {
  __shared__ float2 srow[W];
  const int n2 = blockIdx.x + 1;
  float2* rowp = data + (long long)blockIdx.y * img_stride + (long long)(n2 - 1) * W;
  constexpr int NL = (W + kLerpThreads - 1) / kLerpThreads;
  float2 st[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) {   // every load in flight before the first store
    const int i = threadIdx.x + kLerpThreads * j;
    st[j] = rowp[i < W ? i : 0];
  }
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const int i = threadIdx.x + kLerpThreads * j;
    if (W % kLerpThreads == 0 || i < W) srow[i] = st[j];
  }
  __syncthreads();
  const int den = 2 * n2, wn2 = W * n2;
  const float rden = 1.0f / (float)den;
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const int q = threadIdx.x + kLerpThreads * j;
    if (W % kLerpThreads != 0 && q >= W) continue;
    const int num = (q - W / 2) * Lp + wn2;
    const int i0 = floor_div_rcp(num, den, rden);
    const float tt = (float)(num - i0 * den) * rden;
    const float2 f0 = i0 >= 0 && i0 < W ? srow[i0] : make_float2(0.f, 0.f);
    const float2 f1 = i0 + 1 >= 0 && i0 + 1 < W ? srow[i0 + 1] : make_float2(0.f, 0.f);
    rowp[q] = make_float2((1.f - tt) * f0.x + tt * f1.x, (1.f - tt) * f0.y + tt * f1.y);
  }
}

#define FUNNEL_REFINE_LENGTHS(X) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

bool refine_length_supported(int W) {
  switch (W) {
#define CASE(n) case n: return true;
    FUNNEL_REFINE_LENGTHS(CASE)
#undef CASE
    default: return false;
  }
}

hipError_t launch_row_lerp(int W, float2* data, int h, int Lp, long long img_stride, int batch, hipStream_t s) {
  if (h <= 0 || batch <= 0) return hipSuccess;
  switch (W) {
#define CASE(n)                                                                            \
  case n:                                                                                  \
    k_row_lerp<n><<<dim3(h, batch), kLerpThreads, 0, s>>>(data, Lp, img_stride);           \
    return hipGetLastError();
    FUNNEL_REFINE_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row_idft(int W, float2* data, int h, long long img_stride, const float2* tw, int batch,
                           hipStream_t s) {
  switch (W) {
#define CASE(n)                                                                                   \
  case n: {                                                                                       \
    constexpr int rows = kIdftThreads / (n / 16);                                                 \
    k_row_idft<n><<<dim3((h + rows - 1) / rows, batch), kIdftThreads, 0, s>>>(data, h, img_stride, tw); \
    return hipGetLastError();                                                                     \
  }
    FUNNEL_REFINE_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------ iteration state
//
// state[(img * ns + s) * K + p] = {m, y, m0, y0, sign}: slope bin and intercept
// (centred, real), the start cell, and the sign of P there (0 until known).
struct RefState {
  float m, y, m0, y0, sg;
};

__global__ void k_refine_init(const ft_peak* __restrict__ peaks, const int32_t* __restrict__ n_found, int ns, int K,
                              int W0, int W1, int Np, RefState* __restrict__ st, int total) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int s = (i / K) % ns, p = i % K, img = i / (K * ns);
  RefState r{0.f, 0.f, 0.f, 0.f, 0.f};
  if (p < n_found[img * ns + s]) {
    const ft_peak pk = peaks[i];
    const int W = s == 0 ? W0 : W1;
    r.m0 = r.m = (float)(pk.col - W / 2);
    r.y0 = r.y = (float)(pk.row - Np / 2);
  }
  st[i] = r;
}

// ------------------------------------------------------------------ the DTFT sums
//
// For rows n2 of one space and peaks p of a group of 16:
//   A0 = sum_x' g e_p,  S1 = sum_x' x' g e_p,  S2 = sum_x' x'^2 g e_p,
// e_p(x') = exp(-j 2 pi m_p x' / W), centred x'.  A1 = (-j 2 pi / W) S1 and
// A2 = -(2 pi / W)^2 S2 are the first two m-derivatives of A0.  The phase
// m x'/W is split as (m0 x' mod W)/W + u x'/W with the start cell m0 and
// |u| <= 1, so the large part is exact in integers.
// Output layout: A[((img * ns + s) * K + p) * 3 + d][n2 - 1], d = A0, S1, S2.
constexpr int kRefPeaks = 16;

// The sums are a matrix product, computed on the matrix cores.  Per image,
// with k = 2x' + c (c = 0:
// real part, 1: imaginary part of g[n2][x']), they are one real product
//   C[n2][o] = sum_k Gr[n2][k] B[k][o],  o < 48: real parts, o >= 48:
//   imaginary parts of the 48 complex sums (3 per peak: e, x' e, x'^2 e),
// B[2x'][o] = (Re, Im) of the weight, B[2x'+1][o] = (-Im, Re).  A block
// takes 128 rows with twelve waves, each 32 rows x 32 columns as one
// 32 x 32 FP32 accumulator (v_mfma_f32_32x32x2f32, one x' per instruction),
// three waves per SIMD so that one wave's LDS waits are covered by another's
// matrix instructions.
// Chunks of 32 samples are double-buffered in LDS: while a chunk is
// multiplied, the next chunk's g (loaded into registers one chunk earlier)
// and weights (the phase reduced exactly in integers as above) are written
// to the other buffer, so there is one barrier per chunk and the staging
// work sits between the matrix instructions.
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kMRows = 128, kMChunk = 32, kMThreads = 768, kMCols = 3 * kRefPeaks;   // 48 complex columns

__global__ void __launch_bounds__(kMThreads)
    k_refine_dtft_mfma(const float2* __restrict__ g, long long img_stride, int h, int W, int s, int ns, int K,
                       const int32_t* __restrict__ n_found, const RefState* __restrict__ st, float2* __restrict__ A) {
  __shared__ float2 gt[2][kMRows][kMChunk + 1];   // rows x samples of g (as floats: k = 2x' + c)
  __shared__ float bt[2][2 * kMChunk][2 * kMCols + 1];   // the real weight matrix B[k][o] of a chunk
  __shared__ float pm[kRefPeaks];
  __shared__ int pm0[kRefPeaks];
  const int img = blockIdx.y, grp = blockIdx.z;
  const int r0 = blockIdx.x * kMRows;          // first row (n2 - 1) of the block
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cnt = n_found[img * ns + s];
  if (grp * kRefPeaks >= cnt) return;          // uniform: no peaks in this group
  const long long sbase = ((long long)img * ns + s) * K;
  if (tid < kRefPeaks) {
    const int p = grp * kRefPeaks + tid;
    const RefState r = p < cnt ? st[sbase + p] : RefState{0.f, 0.f, 0.f, 0.f, 0.f};
    pm0[tid] = (int)r.m0;
    pm[tid] = r.m - r.m0;
  }
  const float2* gimg = g + (long long)img * img_stride;

  // g tile of a chunk: 128 rows x 32 samples = 2048 float4 (two samples each), 3 slots per thread
  constexpr int NGT = kMRows * kMChunk / 2, NG = (NGT + kMThreads - 1) / kMThreads;
  float4 gr[NG];
  auto load_g = [&](int x0) {
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      const int i = tid + kMThreads * j, row = i / (kMChunk / 2), c2 = i % (kMChunk / 2);
      gr[j] = i < NGT && r0 + row < h
                  ? *reinterpret_cast<const float4*>(gimg + (long long)(r0 + row) * W + x0 + 2 * c2)
                  : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto store_g = [&](int buf, int j0, int j1) {   // register slots j0 .. j1-1
#pragma unroll
    for (int j = j0; j < j1; ++j) {
      const int i = tid + kMThreads * j, row = i / (kMChunk / 2), c2 = i % (kMChunk / 2);
      if (i >= NGT) continue;
      gt[buf][row][2 * c2] = make_float2(gr[j].x, gr[j].y);
      gt[buf][row][2 * c2 + 1] = make_float2(gr[j].z, gr[j].w);
    }
  };
  auto build_w = [&](int buf, int x0, int i) {   // weight entry i of 32 samples x 16 peaks
    {
      const int xl = i / kRefPeaks, p = i % kRefPeaks;
      const int xc = x0 + xl - W / 2;
      const int whole = ((pm0[p] * xc) % W + W) % W;
      const float frac = (float)whole / (float)W + pm[p] * (float)xc / (float)W;
      float sn, cs;
      sincospif(-2.0f * frac, &sn, &cs);
      const float fx = (float)xc;
      // weights e, x' e, x'^2 e as B[2x'][q] = Re, B[2x'][48 + q] = Im,
      // B[2x' + 1][q] = -Im, B[2x' + 1][48 + q] = Re
      float* r0w = bt[buf][2 * xl];
      float* r1w = bt[buf][2 * xl + 1];
      float re = cs, im = sn;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int q = 3 * p + d;
        r0w[q] = re;
        r0w[kMCols + q] = im;
        r1w[q] = -im;
        r1w[kMCols + q] = re;
        re *= fx;
        im *= fx;
      }
    }
  };

  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  constexpr int NW = kMChunk * kRefPeaks;   // weight entries of a chunk, one per thread at most
  static_assert(NW <= kMThreads && NG == 3, "staging pieces below");
  load_g(0);
  store_g(0, 0, NG);
  __syncthreads();   // pm, pm0
  if (tid < NW) build_w(0, 0, tid);
  if (kMChunk < W) load_g(kMChunk);
  __syncthreads();

  const int li = lane & 31, lk = lane >> 5;    // operand row / column and k of this lane
  const int stripe = wave / 3, t = wave % 3;   // rows 32 stripe .., columns 32 t ..
  const int o = 32 * t + li, q = o % kMCols;   // this lane's output column
  const int nch = W / kMChunk;
  for (int c = 0; c < nch; ++c) {
    const int cur = c & 1, nb = cur ^ 1;
    const bool next = c + 1 < nch, next2 = c + 2 < nch;
    const int x1 = (c + 1) * kMChunk, x2 = (c + 2) * kMChunk;
    // lane (li, lk) supplies A[row li][k = 2x' + lk] and B[k = 2x' + lk][column li].
    // The next chunk is staged into the other buffer in pieces between the
    // products (its g from registers, then the loads of the chunk after it,
    // then its weights), so that this work issues while the matrix core runs.
    const float* ga = reinterpret_cast<const float*>(&gt[cur][32 * stripe + li][0]) + lk;
#pragma unroll
    for (int xl = 0; xl < kMChunk; ++xl) {
      const float a = ga[2 * xl];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bt[cur][2 * xl + lk][o], acc, 0, 0, 0);
      if (next) {
        if (xl == 4) store_g(nb, 0, 2);
        if (xl == 8) store_g(nb, 2, 3);
        if (xl == 12 && next2) load_g(x2);
        if (xl == 20 && tid < NW) build_w(nb, x1, tid);
      }
    }
    __syncthreads();
  }

  // D[i][j] of a 32 x 32 accumulator: column j = lane mod 32, row
  // i = 8 (v / 4) + 4 (lane / 32) + v mod 4 for register v
  const int comp = o / kMCols;
  const int p = grp * kRefPeaks + q / 3, d = q % 3;
  if (p >= cnt) return;
  float* dst = reinterpret_cast<float*>(A + ((sbase + p) * 3 + d) * (long long)h) + comp;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = r0 + 32 * stripe + 8 * (v / 4) + 4 * lk + (v % 4);
    if (row < h) dst[2 * (long long)row] = acc[v];
  }
}

// ------------------------------------------------------------------ the Newton step
//
// One block per peak.  With w = exp(+j 2 pi n2 y / Np), c = 2 pi n2 / Np,
// kw = 2 pi / W and f = 2 / Np:
//   P    =  f      sum Re(A0 w)        P_y  = -f    sum c Im(A0 w)
//   P_yy = -f      sum c^2 Re(A0 w)    P_m  =  f kw sum Im(S1 w)
//   P_my =  f kw   sum c Re(S1 w)      P_mm = -f kw^2 sum Re(S2 w)
// Then (thread 0) the same safeguarded step as the definition: Newton when
// the Hessian of F = sign(P) P is negative definite, else a gradient step of
// 1/4 cell; each component clamped to 1/2 cell, the total displacement to 1
// cell from the start.  With `final` set P is only evaluated and the record
// written.
__global__ void __launch_bounds__(256)
    k_refine_step(const float2* __restrict__ A, int h, int Np, int W, int s, int ns, int K, int space_id, int N,
                  int M, const int32_t* __restrict__ n_found, RefState* __restrict__ st, int final,
                  ft_refined* __restrict__ out) {
  const int p = blockIdx.x, img = blockIdx.y, tid = threadIdx.x;
  const long long idx = ((long long)img * ns + s) * K + p;
  if (p >= n_found[img * ns + s]) {
    if (final && tid == 0) {
      ft_refined z;
      z.col = z.row = z.value = z.slope = z.intercept = z.shift = 0.f;
      out[idx] = z;
    }
    return;
  }
  const RefState r = st[idx];
  const int y0 = (int)r.y0;
  const float uy = r.y - r.y0;
  const float2* a = A + idx * 3 * (long long)h;
  float q[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int n2 = 1 + tid; n2 <= h; n2 += 256) {
    // phase n2 y / Np = (n2 y0 mod Np) / Np + n2 (y - y0) / Np
    const int whole = (int)(((long long)n2 * y0 % Np + Np) % Np);
    const float frac = (float)whole / (float)Np + (float)n2 * uy / (float)Np;
    float sn, cs;
    sincospif(2.0f * frac, &sn, &cs);
    const float c = 6.283185307179586f * (float)n2 / (float)Np;
    const float2 a0 = a[n2 - 1], b1 = a[h + n2 - 1], b2 = a[2 * (long long)h + n2 - 1];
    const float re0 = a0.x * cs - a0.y * sn, im0 = a0.x * sn + a0.y * cs;
    const float re1 = b1.x * cs - b1.y * sn, im1 = b1.x * sn + b1.y * cs;
    const float re2 = b2.x * cs - b2.y * sn;
    q[0] += re0;
    q[1] = fmaf(c, im0, q[1]);
    q[2] = fmaf(c * c, re0, q[2]);
    q[3] += im1;
    q[4] = fmaf(c, re1, q[4]);
    q[5] += re2;
  }
  __shared__ float part[256 / 64][6];
#pragma unroll
  for (int k = 0; k < 6; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) q[k] += __shfl_xor(q[k], off, 64);
  if ((tid & 63) == 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) part[tid >> 6][k] = q[k];
  __syncthreads();
  if (tid != 0) return;
#pragma unroll
  for (int k = 0; k < 6; ++k) q[k] = part[0][k] + part[1][k] + part[2][k] + part[3][k];
  const float f = 2.0f / (float)Np, kw = 6.283185307179586f / (float)W;
  const float P = f * q[0];
  RefState nr = r;
  if (nr.sg == 0.f) nr.sg = P >= 0.f ? 1.f : -1.f;
  if (final) {
    ft_refined rec;
    const int Wp = space_id == 0 ? M : N, Hp = space_id == 0 ? N : M;
    rec.col = r.m + (float)(Wp / 2);
    rec.row = r.y + (float)(Np / 2);
    rec.value = fabsf(P);
    rec.slope = -2.0f * r.m / (float)Wp;
    rec.intercept = r.y - rec.slope * (float)(Wp / 2) + (float)(Hp / 2);
    rec.shift = hypotf(r.m - r.m0, r.y - r.y0);
    out[idx] = rec;
    return;
  }
  const float sg = nr.sg;
  const float Fm = sg * f * kw * q[3], Fy = -sg * f * q[1];
  const float Fmm = -sg * f * kw * kw * q[5], Fmy = sg * f * kw * q[4], Fyy = -sg * f * q[2];
  const float det = Fmm * Fyy - Fmy * Fmy;
  float dm, dy;
  if (Fmm < 0.f && det > 0.f) {
    dm = -(Fyy * Fm - Fmy * Fy) / det;
    dy = -(Fmm * Fy - Fmy * Fm) / det;
  } else {
    const float nrm = hypotf(Fm, Fy);
    dm = nrm > 0.f ? 0.25f * Fm / nrm : 0.f;
    dy = nrm > 0.f ? 0.25f * Fy / nrm : 0.f;
  }
  nr.m = fminf(fmaxf(r.m + fminf(fmaxf(dm, -0.5f), 0.5f), r.m0 - 1.f), r.m0 + 1.f);
  nr.y = fminf(fmaxf(r.y + fminf(fmaxf(dy, -0.5f), 0.5f), r.y0 - 1.f), r.y0 + 1.f);
  st[idx] = nr;
}

hipError_t launch_refine_init(const ft_peak* peaks, const int32_t* n_found, int batch, int ns, int K, int W0, int W1,
                              int Np, void* state, hipStream_t s) {
  const int total = batch * ns * K;
  k_refine_init<<<(total + 255) / 256, 256, 0, s>>>(peaks, n_found, ns, K, W0, W1, Np, static_cast<RefState*>(state),
                                                    total);
  return hipGetLastError();
}

hipError_t launch_refine_iter(const float2* g, long long img_stride, int h, int W, int s, int ns, int K, int batch,
                              const int32_t* n_found, void* state, float2* A, int Np, int space_id, int N, int M,
                              int final, ft_refined* out, hipStream_t st) {
  RefState* sv = static_cast<RefState*>(state);
  if (W % kMChunk != 0) return hipErrorInvalidValue;   // every refinement length is a multiple of the chunk
  dim3 g1((h + kMRows - 1) / kMRows, batch, (K + kRefPeaks - 1) / kRefPeaks);
  k_refine_dtft_mfma<<<g1, kMThreads, 0, st>>>(g, img_stride, h, W, s, ns, K, n_found, sv, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_refine_step<<<dim3(K, batch), 256, 0, st>>>(A, h, Np, W, s, ns, K, space_id, N, M, n_found, sv, final, out);
  return hipGetLastError();
}

size_t refine_state_bytes() { return sizeof(RefState); }

}  // namespace funnel
