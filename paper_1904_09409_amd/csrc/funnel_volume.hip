// funnel_volume.hip -- the y' pass of the funnel transform of a volume
// (App. A), for gfx950.
//
// The volume transform runs four passes over the half spectrum
// S[n3][y][x] (n3 = 1 .. Nzp/2-1 along z, Eq. A.2):
//   A   DFT along z of every (y, x) line: the image pass A with Ny * Nx lines;
//   Bx  per row (n3, y): x' = s x by linear interpolation fused with the
//       centred DFT along x' (the image row pass, Ny rows per ratio s);
//   By  per column (n3, m1): y' = s y likewise, fused with the centred DFT
//       along y' -- this file;
//   C   Hermitian inverse DFT along omega_3 of every (m2, m1) line: the
//       image pass C with Ny * Nx lines.
// Bilinear interpolation is the product of the two linear ones and
// interpolating along x commutes with the DFT along y (they act on
// different axes), so Bx followed by By is Eqs. A.3-A.4.
//
// One block per (slice n3, tile of LINES adjacent columns): the L x LINES
// tile is staged in LDS with 16-byte loads (the LINES columns of a row are
// contiguous in HBM), the gather reads the two neighbours of each output
// sample from LDS into the registers of the first butterfly pass, and the
// results go back row by row, LINES columns at a time.  The LDS copy then
// serves as the exchange buffer of the register-resident DFT.
#include <hip/hip_runtime.h>

#include "funnel_passes.hpp"

namespace funnel {

template <int L, int E_, int LINES_>
struct YColCfg {
  static constexpr int LINES = LINES_;
  static constexpr bool POW2 = (L & (L - 1)) == 0;
  static constexpr int P = POW2 ? (L / E_ > 0 ? L / E_ : 1) : cdiv(L, E_);
  static constexpr int THREADS = LINES * P;
  static constexpr int E = FftR<L, P, false, false>::EM;   // registers per thread
  static constexpr bool valid = L >= 16 && L <= 1024 && radix_plan(L).n > 0 && P >= 2 &&
                                (POW2 ? L % E_ == 0 : E * 2 <= 3 * E_) && THREADS >= 64 && THREADS <= 1024 &&
                                LayInterR<LINES>::size(L) * 8 <= 96 * 1024;
};

// y'-pass variants: (elements per thread, columns per block)
#define FUNNEL_YCOL_VARIANTS(X) X(0, 16, 16) X(1, 16, 32) X(2, 16, 8) X(3, 32, 16)
constexpr int kYColVariants = 4;

#define FUNNEL_YCOL_LENGTHS(X) \
  X(32) X(48) X(64) X(96) X(128) X(160) X(192) X(256) X(320) X(384) X(512) X(640) X(768) X(1024)

// data: per volume [h][L][nx] complex, slice n3 - 1 = rows of frequency n3;
// Lz: padded depth (s = 2 n3 / Lz); grid: (tiles * h, batch).
template <int L, int E_, int LINES>
__global__ void __launch_bounds__((YColCfg<L, E_, LINES>::THREADS))
    k_ycol_nvmt(float2* __restrict__ data, int Lz, int nx, int tiles, long long vol_stride,
                const float2* __restrict__ tw) {
  using Cfg = YColCfg<L, E_, LINES>;
  constexpr int P = Cfg::P, THREADS = Cfg::THREADS;
  using Eng = FftR<L, P, false, false>;
  constexpr int E = Eng::EM;
  constexpr RadixPlan PL = Eng::kPlan;
  constexpr int LAST = PL.n - 1;
  constexpr int R0 = PL.r[0], NB0 = L / R0, BPT0 = Eng::template bpt<0, false>();
  constexpr int RL = PL.r[LAST], NBL = L / RL, BPTL = Eng::template bpt<LAST, false>();
  using Lay = LayInterR<LINES>;
  __shared__ float2 lds[Lay::size(L)];

  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = logical % tiles, n3 = logical / tiles + 1;
  const int tid = threadIdx.x, line = tid % LINES, t = tid / LINES;
  const int c0 = tile * LINES;
  float2* slab = data + (long long)blockIdx.y * vol_stride + (long long)(n3 - 1) * L * nx + c0;

  {  // stage rows 0 .. L-1 of the tile's columns, two columns per 16-byte load
    constexpr int Q = LINES / 2, NLD = cdiv(L * Q, THREADS);
    float4 st[NLD];
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int idx = tid + THREADS * j, i = idx / Q, q = idx % Q;
      // nx and c0 are even, so column c0 + 2q + 1 exists whenever c0 + 2q does
      st[j] = ((L * Q) % THREADS == 0 || idx < L * Q) && c0 + 2 * q < nx
                  ? *reinterpret_cast<const float4*>(slab + (long long)i * nx + 2 * q)
                  : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int idx = tid + THREADS * j, i = idx / Q, q = idx % Q;
      if ((L * Q) % THREADS != 0 && idx >= L * Q) continue;
      lds[Lay::addr(2 * q, i)] = make_float2(st[j].x, st[j].y);
      lds[Lay::addr(2 * q + 1, i)] = make_float2(st[j].z, st[j].w);
    }
  }
  __syncthreads();

  // output sample y' = q - L/2 reads the column at i = (y' Lz + L n3) / (2 n3);
  // (-1)^q and (-1)^(p + L/2) centre the DFT's input and output indices
  const int den = 2 * n3, ln3 = L * n3;
  const float rden = 1.0f / (float)den;
  float2 v[E];
#pragma unroll
  for (int s2 = 0; s2 < E; ++s2) v[s2] = make_float2(0.f, 0.f);
#pragma unroll
  for (int b = 0; b < BPT0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      if (!Eng::template ok<0, false>(t, b)) continue;
      const int q = t + P * b + r * NB0;
      const int num = (q - L / 2) * Lz + ln3;
      const int i0 = floor_div_rcp(num, den, rden);
      const float tt = (float)(num - i0 * den) * rden;
      float2 f0 = make_float2(0.f, 0.f), f1 = make_float2(0.f, 0.f);
      if (i0 >= 0 && i0 < L) f0 = lds[Lay::addr(line, i0)];
      if (i0 + 1 >= 0 && i0 + 1 < L) f1 = lds[Lay::addr(line, i0 + 1)];
      const float sg = (q & 1) ? -1.f : 1.f;
      v[b * R0 + r] = make_float2(sg * ((1.f - tt) * f0.x + tt * f1.x), sg * ((1.f - tt) * f0.y + tt * f1.y));
    }
  Eng::template run<false, false, false, Lay>(v, line, t, lds, tw);
  if (c0 + line >= nx) return;
#pragma unroll
  for (int b = 0; b < BPTL; ++b)
#pragma unroll
    for (int q = 0; q < RL; ++q) {
      if (!Eng::template ok<LAST, false>(t, b)) continue;
      const int p = t + P * b + q * NBL;
      float2 g = v[b * RL + q];
      if ((p + L / 2) & 1) g = make_float2(-g.x, -g.y);
      slab[(long long)p * nx + line] = g;
    }
}

template <int L>
unsigned ycol_variant_mask_t() {
  unsigned m = 0;
#define FUNNEL_V(i, e, l) \
  if constexpr (YColCfg<L, e, l>::valid) m |= 1u << i;
  FUNNEL_YCOL_VARIANTS(FUNNEL_V)
#undef FUNNEL_V
  return m;
}

template <int L>
hipError_t launch_ycol_t(int variant, float2* data, int Lz, int h, int nx, long long vol_stride, const float2* tw,
                         int batch, hipStream_t s) {
  switch (variant) {
#define FUNNEL_V(i, e, l)                                                                              \
  case i:                                                                                              \
    if constexpr (YColCfg<L, e, l>::valid) {                                                           \
      using F = YColCfg<L, e, l>;                                                                      \
      const int tiles = (nx + l - 1) / l;                                                              \
      dim3 grid(tiles * h, batch), block(F::THREADS);                                                  \
      k_ycol_nvmt<L, e, l><<<grid, block, 0, s>>>(data, Lz, nx, tiles, vol_stride, tw);                \
      return hipGetLastError();                                                                        \
    }                                                                                                  \
    break;
    FUNNEL_YCOL_VARIANTS(FUNNEL_V)
#undef FUNNEL_V
    default: break;
  }
  return hipErrorInvalidValue;
}

// The y space of a volume (depth y, rows z, columns x) reads its lines
// along y as contiguous rows: each slice [Ny][Nx] is transposed to [Nx][Ny]
// through a 64 x 64 LDS tile (coalesced 256-byte row reads and writes; one
// pad column keeps the transposed reads off a single bank).
constexpr int kTpTile = 64, kTpThreads = 256;

__global__ void __launch_bounds__(kTpThreads)
    k_transpose_slices(const float* __restrict__ in, float* __restrict__ out, int slices, int ny, int nx) {
  __shared__ float tile[kTpTile][kTpTile + 1];
  const int x0 = blockIdx.x * kTpTile, y0 = blockIdx.y * kTpTile;
  const int tx = threadIdx.x % kTpTile, ty = threadIdx.x / kTpTile;
  for (int sl = blockIdx.z; sl < slices; sl += gridDim.z) {   // same count for every thread of the block
    const long long base = (long long)sl * ny * nx;
#pragma unroll
    for (int r = ty; r < kTpTile; r += kTpThreads / kTpTile) {
      const int y = y0 + r, x = x0 + tx;
      tile[r][tx] = (y < ny && x < nx) ? in[base + (long long)y * nx + x] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int r = ty; r < kTpTile; r += kTpThreads / kTpTile) {
      const int x = x0 + r, y = y0 + tx;
      if (x < nx && y < ny) out[base + (long long)x * ny + y] = tile[tx][r];
    }
    __syncthreads();
  }
}

hipError_t launch_transpose_slices(const float* in, float* out, int slices, int ny, int nx, hipStream_t s) {
  if (slices <= 0) return hipSuccess;
  dim3 grid((nx + kTpTile - 1) / kTpTile, (ny + kTpTile - 1) / kTpTile, slices < 65535 ? slices : 65535);
  k_transpose_slices<<<grid, kTpThreads, 0, s>>>(in, out, slices, ny, nx);
  return hipGetLastError();
}

unsigned ycol_variant_mask(int L) {
  switch (L) {
#define CASE(n) case n: return ycol_variant_mask_t<n>();
    FUNNEL_YCOL_LENGTHS(CASE)
#undef CASE
    default: return 0;
  }
}

int ycol_lines(int variant) {
  switch (variant) {
#define FUNNEL_V(i, e, l) case i: return l;
    FUNNEL_YCOL_VARIANTS(FUNNEL_V)
#undef FUNNEL_V
    default: return 0;
  }
}

hipError_t launch_ycol(int L, int variant, float2* data, int Lz, int h, int nx, long long vol_stride,
                       const float2* tw, int batch, hipStream_t s) {
  if (h <= 0 || batch <= 0) return hipSuccess;
  if (nx <= 0 || (nx & 1)) return hipErrorInvalidValue;
  switch (L) {
#define CASE(n) case n: return launch_ycol_t<n>(variant, data, Lz, h, nx, vol_stride, tw, batch, s);
    FUNNEL_YCOL_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace funnel
