// funnel_peaks.hip -- peak detection of Sec. 4.4 and the line read-out of
// Eqs. 22-25.
//
// The paper's procedure visits all cells in the order (|P| descending) and
// accepts a cell when no neighbour was visited before it.  Since every cell is
// marked when visited, "a neighbour was visited" is the same as "a neighbour
// precedes the cell in the order", so the accepted cells are exactly the local
// maxima under that total order, taken first-K in order.  Ties of |P| are
// broken by the lower linear index, which makes the order total and the
// result unique.  Each cell carries the 64-bit key (~bits(|P|) << 32 | index):
// smaller key = earlier in the order.
//
// Stage 1: one block per tile of 1024 cells flags its local maxima (above the
//          threshold, outside the expansion-border cells), sorts the keys of
//          the tile in LDS (bitonic) and keeps its first K.
// Stage 2: one block per plane merges the tile lists chunk by chunk, keeping
//          a running first-K, and writes the records.  No atomics anywhere, so
//          results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "funnel_internal.hpp"

namespace funnel {

constexpr int kPeakTile = 1024;     // cells per stage-1 block
constexpr int kPeakThreads = 256;
constexpr int kMergeLen = 2048;     // keys sorted per stage-2 step
constexpr int kMergeThreads = 512;
constexpr uint64_t kNoKey = ~0ull;

struct PlaneGeom {
  int rows, cols;      // plane shape: Np x W
  int himg;            // image extent along the padded axis (N regular, M inverse)
  long long offset;    // floats from the image's plane block to this plane
};

__device__ __forceinline__ uint64_t cell_key(float v, int idx) {
  const uint32_t b = __float_as_uint(fabsf(v));
  return ((uint64_t)(~b) << 32) | (uint32_t)idx;
}

__device__ __forceinline__ bool in_border(const PlaneGeom& g, int r, int c) {
  const int cc = c - g.cols / 2;
  if (cc < -1 || cc > 1) return false;
  const int y = r - g.rows / 2;
  const int e0 = -g.himg / 2, e1 = g.himg / 2;
  return (y >= e0 - 2 && y <= e0 + 1) || (y >= e1 - 2 && y <= e1 + 1);
}

template <int N, int THREADS>
__device__ __forceinline__ void bitonic_sort(uint64_t* a) {
  for (int size = 2; size <= N; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < N / 2; i += THREADS) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t x = a[lo], y = a[hi];
        if ((x > y) == up) { a[lo] = y; a[hi] = x; }
      }
      __syncthreads();
    }
  }
}

// Per-image plane blocks start at map.out(img); gidx maps the launch's image
// index to the caller's (ragged batches), NULL meaning the identity.
__global__ void __launch_bounds__(kPeakThreads)
    k_peaks_tile(const float* __restrict__ planes, ImgMap map, PlaneGeom g0, PlaneGeom g1, int nspaces, int tiles,
                 int K, float thr, int radius, int wrap, int keep_border, uint64_t* __restrict__ out) {
  __shared__ uint64_t keys[kPeakTile];
  const int plane = blockIdx.y;                 // image * nspaces + space
  const int img = plane / nspaces, sp = plane % nspaces;
  const PlaneGeom g = sp == 0 ? g0 : g1;
  const float* P = planes + map.out(img) + g.offset;
  const int ncell = g.rows * g.cols;
  const int tile = blockIdx.x;

  for (int e = threadIdx.x; e < kPeakTile; e += kPeakThreads) {
    const int c = tile * kPeakTile + e;
    uint64_t key = kNoKey;
    if (tile < tiles && c < ncell) {
      const float v = P[c];
      const uint64_t me = cell_key(v, c);
      const int r = c / g.cols, col = c % g.cols;
      bool peak = fabsf(v) >= thr && (keep_border || !in_border(g, r, col));
      for (int dr = -radius; peak && dr <= radius; ++dr) {
        int rr = r + dr;
        if (wrap) rr = (rr % g.rows + g.rows) % g.rows;
        else if (rr < 0 || rr >= g.rows) continue;
        for (int dc = -radius; dc <= radius; ++dc) {
          int cc = col + dc;
          if (wrap) cc = (cc % g.cols + g.cols) % g.cols;
          else if (cc < 0 || cc >= g.cols) continue;
          const int q = rr * g.cols + cc;
          if (q == c) continue;
          if (cell_key(P[q], q) < me) { peak = false; break; }
        }
      }
      if (peak) key = me;
    }
    keys[e] = key;
  }
  __syncthreads();
  bitonic_sort<kPeakTile, kPeakThreads>(keys);
  uint64_t* dst = out + ((long long)plane * tiles + tile) * K;
  for (int i = threadIdx.x; i < K; i += kPeakThreads) dst[i] = i < kPeakTile ? keys[i] : kNoKey;
}

__global__ void __launch_bounds__(kMergeThreads)
    k_peaks_merge(const float* __restrict__ planes, ImgMap map, const int* __restrict__ gidx, PlaneGeom g0,
                  PlaneGeom g1, int nspaces, int space0, int tiles, int K, const uint64_t* __restrict__ cand,
                  ft_peak* __restrict__ peaks, int32_t* __restrict__ n_found) {
  __shared__ uint64_t keys[kMergeLen];
  const int plane = blockIdx.x;
  const int img = plane / nspaces, sp = plane % nspaces;
  const int gimg = gidx ? gidx[img] : img;
  const PlaneGeom g = sp == 0 ? g0 : g1;
  const float* P = planes + map.out(img) + g.offset;
  const uint64_t* src = cand + (long long)plane * tiles * K;
  const long long total = (long long)tiles * K;

  for (int i = threadIdx.x; i < kMergeLen; i += kMergeThreads) keys[i] = kNoKey;
  __syncthreads();
  const int chunk = kMergeLen - K;
  for (long long base = 0; base < total; base += chunk) {
    for (int i = threadIdx.x; i < chunk; i += kMergeThreads) {
      const long long j = base + i;
      keys[K + i] = j < total ? src[j] : kNoKey;
    }
    __syncthreads();
    bitonic_sort<kMergeLen, kMergeThreads>(keys);
  }
  // records
  int count = 0;
  for (int i = 0; i < K; ++i) count += keys[i] != kNoKey;
  ft_peak* dst = peaks + ((long long)gimg * nspaces + sp) * K;
  for (int i = threadIdx.x; i < count; i += kMergeThreads) {
    const int c = (int)(uint32_t)(keys[i] & 0xffffffffu);
    const int r = c / g.cols, col = c % g.cols;
    ft_peak pk;
    pk.image = gimg;
    pk.space = space0 + sp;   // 0 regular, 1 inverse, whichever spaces the plan has
    pk.row = r;
    pk.col = col;
    pk.value = fabsf(P[c]);
    const float slope = -2.0f * (float)(col - g.cols / 2) / (float)g.cols;
    pk.slope = slope;
    pk.intercept = (float)(r - g.rows / 2) - slope * (float)(g.cols / 2) + (float)(g.himg / 2);
    dst[i] = pk;
  }
  if (threadIdx.x == 0) n_found[(long long)gimg * nspaces + sp] = count;
}

size_t peaks_workspace_bytes(int nplanes_total, int tiles, int K) {
  return (size_t)nplanes_total * (size_t)tiles * (size_t)K * sizeof(uint64_t);
}

int peaks_tiles(int rows, int cols) { return (int)(((long long)rows * cols + kPeakTile - 1) / kPeakTile); }

hipError_t launch_peaks(const float* planes, ImgMap map, const int* gidx, int batch, int nspaces, int space0,
                        const int* rows, const int* cols, const int* himg, const long long* offset, int K, float thr,
                        int radius, int wrap, int keep_border, ft_peak* peaks, int32_t* n_found, void* ws,
                        hipStream_t s) {
  PlaneGeom g[2];
  int tiles = 0;
  for (int i = 0; i < nspaces; ++i) {
    g[i] = PlaneGeom{rows[i], cols[i], himg[i], offset[i]};
    const int t = peaks_tiles(rows[i], cols[i]);
    tiles = t > tiles ? t : tiles;
  }
  if (nspaces == 1) g[1] = g[0];
  uint64_t* cand = static_cast<uint64_t*>(ws);
  dim3 grid1(tiles, batch * nspaces);
  k_peaks_tile<<<grid1, kPeakThreads, 0, s>>>(planes, map, g[0], g[1], nspaces, tiles, K, thr, radius, wrap,
                                              keep_border, cand);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_peaks_merge<<<batch * nspaces, kMergeThreads, 0, s>>>(planes, map, gidx, g[0], g[1], nspaces, space0, tiles, K,
                                                          cand, peaks, n_found);
  return hipGetLastError();
}

}  // namespace funnel
