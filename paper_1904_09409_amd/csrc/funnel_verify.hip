// funnel_verify.hip -- line verification of Sec. 4.5 on the GPU.
//
// For every detected peak the candidate line (its slope and intercept in
// pixel-index coordinates) is followed through the image: at each position
// along the line's major axis (columns for the regular space, rows for the
// inverse space) the line crosses the minor axis at y = slope * pos +
// intercept, and the band holds the 2D+1 samples at y + d, d = -D..D,
// linearly interpolated between the two neighbouring pixels across the line.
// A position counts when all the pixels it reads, floor(y) - D ..
// floor(y) + D + 1, are inside the image.  The band is integrated along the
// line (steps 2-3) and the mean profile decides (step 4): contrast = larger
// of |centre - mean of the two outermost offsets| (a ridge) and |last - first|
// (a step edge); verified when contrast >= min_contrast and at least
// min_length positions were read.  A wrapping peak (Sec. 4.5, Fig. 9) names
// a line that is not in the image, so its band is flat and it is rejected.
//
// y is evaluated with one rounding (fused multiply-add), which fixes the
// pixels read independently of the evaluation order.  One block per peak;
// partial sums are combined in a fixed tree, so results are reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "funnel_internal.hpp"

namespace funnel {

constexpr int kVerifyThreads = 256;
constexpr int kMaxBand = 7;

__global__ void __launch_bounds__(kVerifyThreads)
    k_verify(const float* __restrict__ images, ImgMap map, const int* __restrict__ gidx, int ns, int N, int M,
             const ft_peak* __restrict__ peaks, const int32_t* __restrict__ n_found, int K, int D,
             float min_contrast, int min_length, ft_line_check* __restrict__ out) {
  const int k = blockIdx.x, s = blockIdx.y, i = blockIdx.z;
  const int g = gidx ? gidx[i] : i;
  const long long rec = ((long long)g * ns + s) * K + k;
  const int nb = 2 * D + 1;
  const int tid = threadIdx.x;
  if (k >= n_found[(long long)g * ns + s]) {
    if (tid == 0) {
      ft_line_check z;
      for (int d = 0; d < kMaxBand; ++d) z.profile[d] = 0.f;
      z.contrast = 0.f;
      z.length = 0;
      z.verified = 0;
      out[rec] = z;
    }
    return;
  }
  const ft_peak pk = peaks[rec];
  const float* img = images + map.in(i);
  // regular: positions are columns (M of them), the band runs across rows (N);
  // inverse: positions are rows, the band runs across columns
  const bool inv = pk.space != 0;
  const int npos = inv ? N : M, across = inv ? M : N;
  const long long pos_step = inv ? M : 1, across_step = inv ? 1 : M;

  float acc[kMaxBand];
#pragma unroll
  for (int d = 0; d < kMaxBand; ++d) acc[d] = 0.f;
  int cnt = 0;
  // U positions per thread at a time, every sample load issued before the
  // first use: positions outside the image or with the band crossing its
  // edge read a valid band (the first one) and add nothing, and samples
  // past the band (D < 3) repeat its last row, so every address is in
  // bounds and no load waits behind a branch
  constexpr int U = 4;
  for (int p0 = 0; p0 < npos; p0 += U * kVerifyThreads) {
    float v[U][kMaxBand + 1], tt[U];
    bool inn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + tid + u * kVerifyThreads;
      const int pc = p < npos ? p : npos - 1;
      const float y = fmaf(pk.slope, (float)pc, pk.intercept);
      const float fl = floorf(y);
      const bool in = p < npos && fl - D >= 0.f && fl + D + 1 <= (float)(across - 1);   // also drops NaN
      const int r0 = in ? (int)fl : D;
      tt[u] = y - fl;
      inn[u] = in;
      const float* base = img + (long long)pc * pos_step + (long long)(r0 - D) * across_step;
#pragma unroll
      for (int d = 0; d <= kMaxBand; ++d) v[u][d] = base[(long long)(d < nb ? d : nb) * across_step];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int d = 0; d < kMaxBand; ++d)   // (1 - t) a + t b between the samples d and d + 1
        acc[d] += (inn[u] && d < nb) ? fmaf(tt[u], v[u][d + 1] - v[u][d], v[u][d]) : 0.f;
      cnt += inn[u] ? 1 : 0;
    }
  }

  // block reduction: within each wave by shuffles, then across the waves in LDS
  __shared__ float part[kVerifyThreads / 64][kMaxBand];
  __shared__ int partn[kVerifyThreads / 64];
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int d = 0; d < kMaxBand; ++d)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[d] += __shfl_xor(acc[d], off, 64);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < kMaxBand; ++d) part[wave][d] = acc[d];
    partn[wave] = cnt;
  }
  __syncthreads();
  if (tid != 0) return;
  ft_line_check r;
  int n = 0;
  for (int w = 0; w < kVerifyThreads / 64; ++w) n += partn[w];
  for (int d = 0; d < kMaxBand; ++d) {
    float v = 0.f;
    for (int w = 0; w < kVerifyThreads / 64; ++w) v += part[w][d];
    r.profile[d] = (d < nb && n > 0) ? v / (float)n : 0.f;
  }
  const float ridge = fabsf(r.profile[D] - 0.5f * (r.profile[0] + r.profile[2 * D]));
  const float step = fabsf(r.profile[2 * D] - r.profile[0]);
  r.contrast = fmaxf(ridge, step);
  r.length = n;
  r.verified = (n >= min_length && r.contrast >= min_contrast) ? 1 : 0;
  out[rec] = r;
}

hipError_t launch_verify(const float* images, ImgMap map, const int* gidx, int count, int ns, int N, int M,
                         const ft_peak* peaks, const int32_t* n_found, int K, int D, float min_contrast,
                         int min_length, ft_line_check* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (D < 1 || 2 * D + 1 > kMaxBand) return hipErrorInvalidValue;
  dim3 grid(K, ns, count), block(kVerifyThreads);
  k_verify<<<grid, block, 0, s>>>(images, map, gidx, ns, N, M, peaks, n_found, K, D, min_contrast, min_length, out);
  return hipGetLastError();
}

}  // namespace funnel
